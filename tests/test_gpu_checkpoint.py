"""Square-root checkpointing of the local trajectories.

With checkpoints the adjoint recomputes each segment from its stored level
pair with the same kernels on the same inputs, and the exchange integrates
the boxes in step by global level; every result must therefore equal the
all-levels-stored one bit for bit: costs, gradients, adjoints of a caller
forcing, trajectory output, exchanged rings and targets (through the costs
that follow an exchange), whole solves, and the autograd backward."""
import numpy as np
import pytest

import synth
from conftest import custom_problem, problem

pytestmark = pytest.mark.gpu

# the Turkel-Zwas variant (offsets 2, 2; frozen pads) on the c1 decomposition
TZ_CFG = dict(synth.CONFIGS["c1"], index=140, tz=(2, 2, 0.5))


def _problem(which):
    if which == "dense":
        from test_gpu_parity import DENSE_CFG
        return custom_problem(DENSE_CFG)
    return custom_problem(TZ_CFG) if which == "tz" else problem(which)


def _pair(which, prec, stride):
    from paper_2205_06649_amd.context import Context
    p = _problem(which)
    full = Context(p, prec)
    ck = Context(p, prec)
    nb_full = full.set_checkpointing(0)
    nb_ck = ck.set_checkpointing(stride)
    # with checkpoints the variant's forward runs as column-walk steps (kind
    # 1, not the persistent sweep of kind 2): the stored run takes the same
    # kernels
    if full.tz_kernels()["max_kind"] == 2:
        assert ck.tz_kernels() == {"kind": 1, "column_walk_applies": True, "max_kind": 1}
        full.set_tz_kernels(1)
    return p, full, ck, nb_full, nb_ck


def _x(p, ctx, seed):
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    sb = torch.tensor(p.sigma_b, dtype=torch.float64, device="cuda")
    scale = torch.cat([sb[f].expand(int(i[1]) * int(i[3])) for i in ctx.info for f in range(3)])
    return ctx.background_controls() + 0.3 * scale * torch.randn(
        ctx.ctrl_len, generator=gen, dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("stride", [3, 5])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("which", ["c1", "small", "c2", "tz", "dense"])
def test_checkpointed_equals_stored(which, prec, stride):
    import torch
    p, full, ck, nb_full, nb_ck = _pair(which, prec, stride)
    maxlev = max(int(i[5]) for i in full.info)
    if stride + 1 < maxlev:
        assert nb_ck < nb_full
    x = _x(p, full, 1)
    # local cost and gradient, all subdomains and a subset
    J1, g1 = full.cost_grad(x)
    J2, g2 = ck.cost_grad(x)
    assert torch.equal(J1, J2) and torch.equal(g1, g2)
    ids = [0, full.nsub - 1]
    J1s, g1s = full.cost_grad(x, sub_ids=ids)
    J2s, g2s = ck.cost_grad(x, sub_ids=ids)
    assert torch.equal(g1s, g2s) and np.array_equal(J1s.cpu().numpy()[ids], J2s.cpu().numpy()[ids])
    # trajectory output and the adjoint of a caller forcing
    t1 = full.forward(x)
    t2 = ck.forward(x)
    assert torch.equal(t1, t2)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    f = torch.randn(full.traj_len, generator=gen, dtype=torch.float64, device="cuda")
    assert torch.equal(full.adjoint(f), ck.adjoint(f))
    # exchange (rings and targets from the new trajectories), then costs
    xa = _x(p, full, 2)
    full.exchange(xa)
    ck.exchange(xa)
    J1, g1 = full.cost_grad(x)
    J2, g2 = ck.cost_grad(x)
    assert torch.equal(J1, J2) and torch.equal(g1, g2)
    # level 0 is always kept; other levels only where every box keeps them
    assert torch.equal(full.gather(0), ck.gather(0))
    full.close()
    ck.close()


def test_checkpointed_solve_and_autograd():
    import torch
    from paper_2205_06649_amd.autograd import local_sweep
    p, full, ck, nb_full, nb_ck = _pair("small", "fp64", 3)
    xa1, r1, s1, _ = full.solve(max_outer=2, max_iter=10, outer_tol=0.0)
    xa2, r2, s2, _ = ck.solve(max_outer=2, max_iter=10, outer_tol=0.0)
    assert np.array_equal(xa1, xa2) and r1.total_evals == r2.total_evals
    x = _x(p, full, 3)
    W = torch.randn(full.traj_len, dtype=torch.float64, device="cuda")
    grads = []
    for ctx in (full, ck):
        xr = x.clone().requires_grad_(True)
        (local_sweep(ctx, xr) * W).sum().backward()
        grads.append(xr.grad)
    assert torch.equal(grads[0], grads[1])
    full.close()
    ck.close()


def test_checkpointing_rules():
    from paper_2205_06649_amd import _lib as L
    from paper_2205_06649_amd.context import Context
    p = problem("c1")
    ctx = Context(p, "fp32")
    for bad in (1, 2, -1):
        with pytest.raises(L.DD4DVarError) as e:
            ctx.set_checkpointing(bad)
        assert e.value.status == L.DD4DVAR_E_INVALID
    ctx.set_checkpointing(3)
    # persistent sweeps keep every level
    with pytest.raises(L.DD4DVarError) as e:
        ctx.set_exec_mode(2)
    assert e.value.status == L.DD4DVAR_E_INVALID
    # no stored forward after the arena changed
    with pytest.raises(L.DD4DVarError) as e:
        ctx.adjoint(None)
    assert e.value.status == L.DD4DVAR_E_STATE
    x = _x(p, ctx, 4)
    ctx.forward(x, with_traj=False)
    with pytest.raises(L.DD4DVarError) as e:
        ctx.gather(2)                        # a recomputed level of interval 0
    assert e.value.status == L.DD4DVAR_E_STATE
    ctx.set_checkpointing(0)
    ctx.set_exec_mode(2)
    with pytest.raises(L.DD4DVarError) as e:
        ctx.set_checkpointing(3)
    assert e.value.status == L.DD4DVAR_E_INVALID
    ctx.close()
