"""GPU parity of the persistent plans at the benchmark's box shape.

The 1024 x 2048 decomposition has extended boxes of 72 x 136 (interior
bands) and 68 x 136 (polar bands).  With 136 columns a 1024-thread workgroup
holds 7 column strips, so the strip adjoint (execution mode 4) walks
ceil(72 / 7) = 11 rows per strip, and the box-mapped kernels of mode 2 need
10 passes of 1024 cells (the autotuner also times 11).  This problem has the
same box shapes (core 64 x 128, overlap 4 cells, three latitude bands, so
both the polar and the interior height occur) on a 192 x 384 grid with short
windows, small enough for the oracle to evaluate every box.

Every plan is compared with the oracle box by box (eq. eq:cost:parallel1; the
adjoint of Sec. 2, eq. adjProd): J, and per field (h, u, v) both the
element-wise maximum error relative to the field's largest reference value
and the norm-wise relative error, for the gradient and (forward) the
trajectories.
"""
import functools

import numpy as np
import pytest

from conftest import custom_problem
from oracle import dd, ddmaps, local, model

pytestmark = pytest.mark.gpu

# the benchmark's box shapes: 3 bands of 64 core rows, pieces of 128 columns,
# overlap 4 cells / 2 steps
STRIP_CFG = dict(index=114, nlat=192, nlon=384, nsteps=10, bands=3, pieces=3, ntime=2,
                 overlap_cells=4, overlap_steps=2, obs_frac=0.02, obs_every=2)

TOL_FP32 = 1e-4          # J, gradients: the FP32 bar
TOL_FP32_TRAJ = 2e-5     # trajectories (h as its anomaly)


def field_errors(a, ref):
    """Per field: (max |a - ref| / max |ref|, |a - ref|_2 / |ref|_2); arrays
    [..., 3, ny, nx] with the field axis third from the end."""
    a = np.asarray(a, dtype=np.longdouble)
    ref = np.asarray(ref, dtype=np.longdouble)
    out = []
    for f in range(3):
        d = a[..., f, :, :] - ref[..., f, :, :]
        r = ref[..., f, :, :]
        out.append((float(np.abs(d).max() / np.abs(r).max()),
                    float(np.linalg.norm(d) / np.linalg.norm(r))))
    return out


def assert_fields(a, ref, tol, what):
    errs = field_errors(a, ref)
    for f, (einf, e2) in zip("huv", errs):
        assert einf <= tol and e2 <= tol, (what, f, einf, e2)
    return errs


@functools.lru_cache(maxsize=None)
def _state():
    p = custom_problem(STRIP_CFG)
    maps = ddmaps.build(p)
    bg, trajs = dd.background(p, maps)
    rings, _ = dd.exchange(maps, trajs)
    rng = np.random.default_rng(21)
    xs = [trajs[b.sub][0] + 0.3 * p.sigma_b[:, None, None] * rng.standard_normal(trajs[b.sub][0].shape)
          for b in maps.boxes]
    g = model.Grid.of(p)
    ref = {}
    for b in maps.boxes:
        s = b.sub
        lt = local.forward(local.LocalGeometry(g, maps, s), xs[s], rings[s])
        J, gr = local.cost_grad(p, maps, s, xs[s], trajs[s][0], rings[s],
                                {k: trajs[k] for k in maps.neighbors[s]})
        ref[s] = (lt, J, gr)
    return p, maps, xs, ref


def _anom(Z, h_ref):
    Z = np.array(Z, copy=True)
    Z[..., 0, :, :] -= h_ref
    return Z


def test_box_shapes_match_the_benchmark():
    p, maps, xs, ref = _state()
    shapes = {(b.ny, b.nx) for b in maps.boxes}
    assert shapes == {(68, 136), (72, 136)}


@pytest.mark.parametrize("mode,passes", [(4, 0), (2, 10), (2, 11), (3, 11)])
def test_persistent_plans_against_oracle(mode, passes):
    from paper_2205_06649_amd.context import Context
    p, maps, xs, ref = _state()
    ctx = Context(p, "fp32")
    ctx.set_exec_plan(mode, passes)
    plan = ctx.exec_plan()
    print(f"plan {plan}", flush=True)
    assert plan["strip_rows"] == 11 and plan["persistent"]
    assert plan["mode"] == mode and plan["passes"] == (passes or 10)
    xp = ctx.pack_ctrl(xs)
    traj = ctx.unpack_traj(ctx.forward(xp))
    J, grad = ctx.cost_grad(xp)
    ctx.synchronize()
    J = J.cpu().numpy()
    grads = ctx.unpack_ctrl(grad)
    worst = 0.0
    for b in maps.boxes:
        s = b.sub
        lt, Jr, gr = ref[s]
        assert_fields(_anom(traj[s], p.h_ref), _anom(lt, p.h_ref), TOL_FP32_TRAJ, ("traj", s))
        ej = float(abs(J[s] - Jr) / abs(Jr))
        assert ej <= TOL_FP32, (s, ej)
        errs = assert_fields(grads[s], gr, TOL_FP32, ("grad", s))
        worst = max(worst, max(e for pair in errs for e in pair))
    print(f"mode {mode} passes {plan['passes']}: worst per-field gradient error {worst:.2e}",
          flush=True)
    ctx.close()


def test_strip_and_box_adjoints_agree():
    """Mode 4 (11-row strips) and mode 2 run the same FP32 arithmetic up to
    the compiler's fused multiply-adds: gradients, adjoints of a caller
    forcing and Gauss-Newton products agree to 1e-5 per field."""
    p, maps, xs, ref = _state()
    from paper_2205_06649_amd.context import Context
    ctx = Context(p, "fp32")
    xp = ctx.pack_ctrl(xs)
    rng = np.random.default_rng(22)
    forcing = ctx.pack_traj([rng.standard_normal((b.nlev, 3, b.ny, b.nx)) for b in maps.boxes])
    dx = ctx.pack_ctrl([p.sigma_b[:, None, None] * rng.standard_normal((3, b.ny, b.nx))
                        for b in maps.boxes])
    res = {}
    for mode in (2, 4):
        ctx.set_exec_plan(mode, 11)
        J, g = ctx.cost_grad(xp)
        a = ctx.adjoint(forcing)
        h = ctx.gn_hessvec(dx)
        res[mode] = [ctx.unpack_ctrl(v) for v in (g, a, h)] + [J.cpu().numpy()]
    ctx.synchronize()
    for k in range(3):
        for b in maps.boxes:
            assert_fields(res[4][k][b.sub], res[2][k][b.sub], 1e-5, (k, b.sub))
    assert np.allclose(res[4][3], res[2][3], rtol=1e-9, atol=0)
    ctx.close()
