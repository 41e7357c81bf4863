"""Graph mode and the autotuner of local_cost_grad.

A recorded HIP graph must give, on every replay, exactly what the eager
launches give, also after other eager work on the device between replays and
after new controls are written into the same buffer (the graph reads the
buffers at replay time).  The autotuner must keep the fastest candidate it
timed, and the plan it picks must still meet the parity bars."""
import numpy as np
import pytest

import synth
from conftest import custom_problem, problem
from oracle import dd, ddmaps, local

pytestmark = pytest.mark.gpu


def _setup(which, prec, seed=0):
    import torch
    from paper_2205_06649_amd.context import Context
    # "tz": the Turkel-Zwas variant (offsets 2, 2; frozen pads) on the c1 decomposition
    p = (custom_problem(dict(synth.CONFIGS["c1"], index=140, tz=(2, 2, 0.5))) if which == "tz"
         else problem(which))
    ctx = Context(p, prec)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    sb = torch.tensor(p.sigma_b, dtype=torch.float64, device="cuda")
    scale = torch.cat([sb[f].expand(int(i[1]) * int(i[3])) for i in ctx.info for f in range(3)])
    xb = ctx.background_controls()

    def draw():
        return xb + 0.3 * scale * torch.randn(ctx.ctrl_len, generator=gen, dtype=torch.float64,
                                              device="cuda")
    return p, ctx, draw, torch


PLANS = [("fp64", 0), ("fp32", 0), ("fp32", 2), ("fp32", 3)]


# the Turkel-Zwas variant runs the step kernels only (modes 0 and 1)
@pytest.mark.parametrize("which,prec,mode", [(w, pr, m) for w in ("c1", "small") for pr, m in PLANS]
                         + [("tz", "fp64", 0), ("tz", "fp32", 0), ("tz", "fp64", 1)])
def test_graph_replays_match_eager(which, prec, mode):
    p, ctx, draw, torch = _setup(which, prec)
    ctx.set_exec_mode(mode)
    x = draw()
    x2 = draw()
    J = torch.empty(ctx.nsub, dtype=torch.float64, device="cuda")
    g = torch.empty(ctx.ctrl_len, dtype=torch.float64, device="cuda")
    ctx.cost_grad(x, J, g)
    J_ref, g_ref = J.clone(), g.clone()
    ctx.cost_grad(x2, J, g)
    J_ref2, g_ref2 = J.clone(), g.clone()
    ctx.set_graph(True)
    for rep in range(3):
        J.fill_(0.0)
        g.fill_(0.0)
        ctx.cost_grad(x, J, g)                                   # record, then replays
        torch.cuda.synchronize()
        assert torch.equal(J, J_ref) and torch.equal(g, g_ref), rep
        # eager work between replays: other evaluations and torch kernels
        ctx.cost_grad(x2, sub_ids=[0, ctx.nsub - 1])
        ctx.forward(x2, with_traj=False)
        _ = (x2 * 2.0).sum().item()
    # new controls in the same buffer are read by the replay
    xsave = x.clone()
    x.copy_(x2)
    ctx.cost_grad(x, J, g)
    torch.cuda.synchronize()
    assert torch.equal(J, J_ref2) and torch.equal(g, g_ref2)
    x.copy_(xsave)
    # a different output buffer records a second graph
    J3 = torch.empty_like(J)
    g3 = torch.empty_like(g)
    ctx.cost_grad(x, J3, g3)
    torch.cuda.synchronize()
    assert torch.equal(J3, J_ref) and torch.equal(g3, g_ref)
    ctx.set_graph(False)
    ctx.close()


@pytest.mark.parametrize("graph", [False, True])
def test_autotune_keeps_the_fastest_plan(graph):
    from paper_2205_06649_amd import _lib as L
    p, ctx, draw, torch = _setup("small", "fp32", seed=3)
    x = draw()
    ctx.set_graph(graph)
    rep = ctx.autotune(x, reps=3)
    cands = rep["candidates"]
    assert len(cands) >= 1 and cands[0]["mode"] == 0
    modes = {c["mode"] for c in cands}
    assert modes <= {0, 2, 3, 4}
    ms = [c["ms"] for c in cands]
    assert all(np.isfinite(ms)) and all(m > 0 for m in ms)
    assert rep["chosen"] == int(np.argmin(ms))
    # the chosen plan meets the FP32 bars against the oracle
    J, grad = ctx.cost_grad(x)
    maps = ddmaps.build(p)
    bg, trajs = dd.background(p, maps)
    rings, _ = dd.exchange(maps, trajs)
    xs = ctx.unpack_ctrl(x)
    grads = ctx.unpack_ctrl(grad)
    J = J.cpu().numpy()
    for b in maps.boxes:
        s = b.sub
        Jr, gr = local.cost_grad(p, maps, s, xs[s], trajs[s][0], rings[s],
                                 {k: trajs[k] for k in maps.neighbors[s]})
        assert abs(J[s] - Jr) / abs(Jr) <= 1e-4
        assert np.linalg.norm(grads[s] - gr) / np.linalg.norm(gr) <= 1e-4
    with pytest.raises(L.DD4DVarError) as e:
        ctx.autotune(x, reps=0)
    assert e.value.status == L.DD4DVAR_E_INVALID
    ctx.close()
