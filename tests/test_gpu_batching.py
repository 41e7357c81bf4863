"""Batching of uneven boxes: the 256 x 512, 200-step brick partition (64
spatial pieces of sides 24-96 cells x 8 intervals, overlap 3; 512 boxes of
945 to 8466 cells) evaluated in FP32 with the plan the library's autotuner
picks, as HIP graph replays.

The persistent plans apply to every box (each fits one workgroup's LDS), so
all 512 boxes run in one launch per sweep; the graph replays equal the eager
launches bit for bit, and sampled boxes of every size class meet the FP32
bars against the oracle (J and gradient 1e-4)."""
import numpy as np
import pytest

from conftest import problem
from oracle import dd, ddmaps, local

pytestmark = pytest.mark.gpu


def test_brick_partition_batched_graph():
    import torch
    from paper_2205_06649_amd.context import Context
    p = problem("c3")
    maps = ddmaps.build(p)
    bg, trajs = dd.background(p, maps)
    rings, _ = dd.exchange(maps, trajs)
    ctx = Context(p, "fp32")
    rng = np.random.default_rng(9)
    xs = [trajs[b.sub][0] + 0.3 * p.sigma_b[:, None, None] * rng.standard_normal(trajs[b.sub][0].shape)
          for b in maps.boxes]
    x = ctx.pack_ctrl(xs)
    ctx.set_graph(True)
    tune = ctx.autotune(x, reps=3)
    modes = [c["mode"] for c in tune["candidates"]]
    assert {0, 2, 3} <= set(modes)
    chosen = modes[tune["chosen"]]
    print(f"brick partition: {len(maps.boxes)} boxes, autotuner "
          + ", ".join(f"mode {c['mode']}/{c['passes']}: {c['ms']:.3f} ms" for c in tune["candidates"])
          + f"; chosen mode {chosen}", flush=True)
    J1, g1 = ctx.cost_grad(x)
    J2, g2 = ctx.cost_grad(x)
    ctx.set_graph(False)
    J3, g3 = ctx.cost_grad(x)
    assert torch.equal(J1, J2) and torch.equal(g1, g2)
    assert torch.equal(J1, J3) and torch.equal(g1, g3)
    # one launch per sweep for all boxes in the persistent plans
    if chosen in (2, 4):
        ctx.set_timing(True)
        ctx.cost_grad(x)
        t = ctx.get_timing()
        ctx.set_timing(False)
        assert t["fwd_launches"] == 1 and t["adj_launches"] == 1
    J = J1.cpu().numpy()
    grads = ctx.unpack_ctrl(g1)
    order = np.argsort([b.ncell for b in maps.boxes])
    sample = [int(order[0]), int(order[len(order) // 2]), int(order[-1]), len(maps.boxes) - 1]
    for s in sample:
        Jr, gr = local.cost_grad(p, maps, s, xs[s], trajs[s][0], rings[s],
                                 {k: trajs[k] for k in maps.neighbors[s]})
        ej = float(abs(J[s] - Jr) / abs(Jr))
        eg = float(np.linalg.norm(grads[s] - gr) / np.linalg.norm(gr))
        print(f"  box {s} ({maps.boxes[s].ny}x{maps.boxes[s].nx}): J rel {ej:.2e}, grad rel {eg:.2e}",
              flush=True)
        assert ej <= 1e-4 and eg <= 1e-4, (s, ej, eg)
    ctx.close()
