"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (norm-wise relative errors, per subdomain):
  FP64 mode: 1e-12 for trajectories, J and gradients, against the oracle
  pipeline in extended precision: the background run (and with it the frozen
  rings, overlap targets and x^b_s) and the local evaluation in long double
  from the same FP64 inputs (x_b0, observations, controls).  The observation
  and overlap residuals are differences of nearly equal depths (metres out
  of 1e4 m), so any FP64 evaluation carrying the full depth, the oracle's
  own included, lands up to ~2e-12 from the exact gradient (pinned in the
  oracle tests); the device stores h - h_ref and lands within ~3e-14.
  FP32 state mode: 2e-5 for trajectories (h as its anomaly), 1e-4 for J and
  gradients -- float rounding (6e-8) amplified by at most a few hundred over
  the <= 40 leapfrog steps of these cases; observation/overlap residuals and
  all sums are FP64 on the device.
Integer maps are compared bit for bit in the host-plan tests.
"""
import functools

import numpy as np
import pytest

from conftest import custom_problem, problem
from oracle import dd, ddmaps, local, model
from test_oracle_pins import MIXED_CFG, SPAN_CFG

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-4}
TOL_GRAD = {"fp64": 1e-12, "fp32": 1e-4}
TOL_TRAJ = {"fp64": 1e-12, "fp32": 2e-5}
# FP64 results are compared with the oracle pipeline in extended precision
# (see the module docstring), FP32 results with the FP64 oracle.
REF_DTYPE = {"fp64": np.longdouble, "fp32": np.float64}


def _rel(a, b):
    a = np.asarray(a, dtype=np.longdouble)
    b = np.asarray(b, dtype=np.longdouble)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


# boxes spanning the circle, 128 columns wide (several rows per column strip)
WIDE_CFG = dict(index=112, nlat=48, nlon=128, nsteps=8, bands=3, pieces=1, ntime=2,
                overlap_cells=2, overlap_steps=1, obs_frac=0.05, obs_every=2)


# heavy overlap: up to 11 other space-time boxes cover a cell at a level, so the
# target kernel's batched loads (8 neighbours of a level) are exceeded
DENSE_CFG = dict(index=113, nlat=24, nlon=48, nsteps=24, bands=4, pieces=4, ntime=3,
                 overlap_cells=5, overlap_steps=3, obs_frac=0.1, obs_every=2)


# a time decomposition into two boxes covering the sphere, 112 x 256 cells:
# 112 cost tiles per box (the per-box reduction's lanes sum more than one
# tile each) and 86,016 control entries per box (six solver parts, the last
# ragged)
LARGE_CFG = dict(index=114, nlat=112, nlon=256, nsteps=8, bands=1, pieces=1, ntime=2,
                 overlap_cells=0, overlap_steps=2, obs_frac=0.02, obs_every=2)


def _prob(which):
    if which == "large":
        return custom_problem(LARGE_CFG)
    if which == "dense":
        return custom_problem(DENSE_CFG)
    if which == "span":
        return custom_problem(SPAN_CFG)
    if which == "mixed":
        return custom_problem(MIXED_CFG)
    if which == "wide":
        return custom_problem(WIDE_CFG)
    return problem(which)


@functools.lru_cache(maxsize=None)
def _oracle_state(which):
    p = _prob(which)
    maps = ddmaps.build(p)
    bg, trajs = dd.background(p, maps)
    rings, _ = dd.exchange(maps, trajs)
    return p, maps, bg, trajs, rings


@functools.lru_cache(maxsize=None)
def _oracle_ext(which):
    """Background run, box trajectories and rings in extended precision."""
    p = _prob(which)
    maps = ddmaps.build(p)
    bg, trajs = dd.background(p, maps, np.longdouble)
    rings, _ = dd.exchange(maps, trajs)
    return trajs, rings


def _reference(which, prec):
    """(box trajectories, rings) of the reference pipeline for a precision."""
    if prec == "fp64":
        return _oracle_ext(which)
    p, maps, bg, trajs, rings = _oracle_state(which)
    return trajs, rings


def _ctx(which, prec):
    from paper_2205_06649_amd.context import Context
    return Context(_prob(which), precision=prec)


def _perturbed(p, maps, trajs, seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    sb = p.sigma_b[:, None, None]
    return [trajs[b.sub][0] + scale * sb * rng.standard_normal(trajs[b.sub][0].shape)
            for b in maps.boxes]


def _anom(Z, h_ref):
    Z = np.array(Z, copy=True)
    Z[..., 0, :, :] -= h_ref
    return Z


@pytest.mark.parametrize("which", ["tiny1", "c1", "small"])
def test_global_forward_fp64(which):
    import torch
    p, maps, bg, trajs, rings = _oracle_state(which)
    ctx = _ctx(which, "fp64")
    x0 = torch.from_numpy(np.ascontiguousarray(p.xb0)).cuda()
    gt = ctx.forward_global(x0).cpu().numpy()
    ref = model.forward(model.Grid.of(p), p.xb0, p.nsteps)
    assert _rel(_anom(gt, p.h_ref), _anom(ref, p.h_ref)) <= 1e-12
    # background controls are the background trajectory at each first level
    xb = ctx.unpack_ctrl(ctx.background_controls())
    for b in maps.boxes:
        assert _rel(xb[b.sub], trajs[b.sub][0]) <= 1e-13


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("which", ["tiny1", "c1", "small", "span", "mixed"])
def test_local_forward(which, prec):
    p, maps, bg, trajs, _ = _oracle_state(which)
    _, rings = _reference(which, prec)
    ctx = _ctx(which, prec)
    xs = _perturbed(p, maps, trajs)
    g = model.Grid.of(p, REF_DTYPE[prec])
    traj = ctx.unpack_traj(ctx.forward(ctx.pack_ctrl(xs)))
    for b in maps.boxes:
        geo = local.LocalGeometry(g, maps, b.sub)
        ref = local.forward(geo, np.asarray(xs[b.sub], REF_DTYPE[prec]), rings[b.sub])
        assert _rel(_anom(traj[b.sub], p.h_ref), _anom(ref, p.h_ref)) <= TOL_TRAJ[prec], b.sub


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("which", ["tiny1", "c1", "small", "span", "mixed", "c2", "large"])
def test_local_cost_grad(which, prec):
    """J and gradient of every box; also per field, element-wise (largest
    error over the field's largest reference value)."""
    from test_gpu_strips import field_errors
    p, maps, bg, trajs0, _ = _oracle_state(which)
    trajs, rings = _reference(which, prec)
    ctx = _ctx(which, prec)
    xs = _perturbed(p, maps, trajs0, seed=1)
    J, grad = ctx.cost_grad(ctx.pack_ctrl(xs))
    ctx.synchronize()
    J = J.cpu().numpy()
    grads = ctx.unpack_ctrl(grad)
    worst = 0.0
    for b in maps.boxes:
        s = b.sub
        Jr, gr = local.cost_grad(p, maps, s, xs[s], trajs[s][0], rings[s],
                                 {k: trajs[k] for k in maps.neighbors[s]}, dtype=REF_DTYPE[prec])
        ej, eg = float(abs(J[s] - Jr) / abs(Jr)), float(_rel(grads[s], gr))
        ef = max(e for pair in field_errors(grads[s], gr) for e in pair)
        worst = max(worst, eg, ef)
        # per field element-wise: 10x the norm-wise bar (a field's largest
        # value can sit far below the norm of all three)
        assert ej <= TOL[prec] and eg <= TOL_GRAD[prec] and ef <= 10 * TOL_GRAD[prec], \
            (s, ej, eg, ef)
    print(f"{which} {prec}: worst gradient error {worst:.2e}")


def test_cost_grad_at_background_and_subsets():
    """At x = x_b the background term vanishes; subset calls equal full calls;
    the one-launch-per-subdomain mode equals the batched mode bit for bit."""
    p, maps, bg, trajs, rings = _oracle_state("c1")
    trajs_e, rings_e = _oracle_ext("c1")
    ctx = _ctx("c1", "fp64")
    xb = ctx.background_controls()
    J, grad = ctx.cost_grad(xb)
    J = J.cpu().numpy()
    for b in maps.boxes:
        Jr, gr = local.cost_grad(p, maps, b.sub, trajs_e[b.sub][0], trajs_e[b.sub][0],
                                 rings_e[b.sub], {k: trajs_e[k] for k in maps.neighbors[b.sub]},
                                 dtype=np.longdouble)
        assert float(abs(J[b.sub] - Jr) / abs(Jr)) <= 1e-12
    xs = ctx.pack_ctrl(_perturbed(p, maps, trajs, seed=2))
    J1, g1 = ctx.cost_grad(xs)
    ids = [5, 1, 6]
    J2, g2 = ctx.cost_grad(xs, sub_ids=ids)
    J1, J2 = J1.cpu().numpy(), J2.cpu().numpy()
    u1, u2 = ctx.unpack_ctrl(g1), ctx.unpack_ctrl(g2)
    for s in range(ctx.nsub):
        if s in ids:
            assert J2[s] == J1[s] and np.array_equal(u1[s], u2[s])
        else:
            assert np.isnan(J2[s]) and not np.any(u2[s])
    ctx.set_exec_mode(1)
    J3, g3 = ctx.cost_grad(xs)
    assert np.array_equal(J3.cpu().numpy(), J1) and np.array_equal(g3.cpu().numpy(), g1.cpu().numpy())


@pytest.mark.parametrize("which", ["tiny1", "c1", "span", "mixed", "wide", "c2"])
def test_persistent_strip_adjoint_fp32(which):
    """Execution mode 4 (the persistent adjoint walking column strips of up to
    11 rows per thread): the oracle's local cost and gradient to the FP32
    bars, and the FP32 arithmetic of mode 2 up to the compiler's choice of
    fused multiply-adds -- gradients, adjoints of a caller forcing and
    Gauss-Newton products within 1e-5 of mode 2's, J within 1e-9."""
    p, maps, bg, trajs, rings = _oracle_state(which)
    ctx = _ctx(which, "fp32")
    xs = _perturbed(p, maps, trajs, seed=8)
    xp = ctx.pack_ctrl(xs)
    res = {}
    rng = np.random.default_rng(4)
    forcing = ctx.pack_traj([rng.standard_normal((b.nlev, 3, b.ny, b.nx)) for b in maps.boxes])
    dx = ctx.pack_ctrl([p.sigma_b[:, None, None] * rng.standard_normal((3, b.ny, b.nx))
                        for b in maps.boxes])
    for mode in (2, 4):
        ctx.set_exec_mode(mode)
        J, grad = ctx.cost_grad(xp)
        adj = ctx.adjoint(forcing)
        hv = ctx.gn_hessvec(dx)
        res[mode] = (J.cpu().numpy(), grad.cpu().numpy(), adj.cpu().numpy(), hv.cpu().numpy())
    J, g4, a4, h4 = res[4]
    grads = ctx.unpack_ctrl(g4)
    for b in maps.boxes:
        s = b.sub
        Jr, gr = local.cost_grad(p, maps, s, xs[s], trajs[s][0], rings[s],
                                 {k: trajs[k] for k in maps.neighbors[s]})
        ej, eg = float(abs(J[s] - Jr) / abs(Jr)), float(_rel(grads[s], gr))
        assert ej <= TOL["fp32"] and eg <= TOL_GRAD["fp32"], (s, ej, eg)
    J2, g2, a2, h2 = res[2]
    for a, b in ((g4, g2), (a4, a2), (h4, h2)):
        assert _rel(a, b) <= 1e-5, _rel(a, b)
    assert np.allclose(J, J2, rtol=1e-9, atol=0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("which", ["c1", "span", "mixed"])
def test_adjoint_integrate_random_forcing(which, prec):
    p, maps, bg, trajs, _ = _oracle_state(which)
    _, rings = _reference(which, prec)
    D = REF_DTYPE[prec]
    ctx = _ctx(which, prec)
    xs = _perturbed(p, maps, trajs, seed=3)
    ctx.forward(ctx.pack_ctrl(xs), with_traj=False)
    rng = np.random.default_rng(4)
    forcing = [rng.standard_normal((b.nlev, 3, b.ny, b.nx)) for b in maps.boxes]
    adj = ctx.unpack_ctrl(ctx.adjoint(ctx.pack_traj(forcing)))
    g = model.Grid.of(p, D)
    for b in maps.boxes:
        geo = local.LocalGeometry(g, maps, b.sub)
        lt = local.forward(geo, np.asarray(xs[b.sub], D), rings[b.sub])
        ref = local.adjoint(geo, lt, rings[b.sub], np.asarray(forcing[b.sub], D))
        assert _rel(adj[b.sub], ref) <= TOL[prec], b.sub


@pytest.mark.parametrize("which,prec", [("c1", "fp64"), ("dense", "fp64"), ("dense", "fp32")])
def test_exchange_then_cost_grad(which, prec):
    """After an exchange, rings and targets come from the local trajectories
    (also where more boxes cover a cell than the target kernel loads at once)."""
    p, maps, bg, trajs, rings = _oracle_state(which)
    if which == "dense":       # some cell-level is covered by more than 8 other boxes
        assert max(int((maps.cover_sp[b.row0:b.row0 + b.ny][:, (b.col0 + np.arange(b.nx)) % p.nlon]
                        ).max()) * int(maps.time_count[b.lev0:b.lev0 + b.nlev].max())
                   for b in maps.boxes) - 1 > 8
    ctx = _ctx(which, prec)
    xa = _perturbed(p, maps, trajs, seed=5)
    ctx.exchange(ctx.pack_ctrl(xa))
    D = REF_DTYPE[prec]
    ref_trajs, ref_rings = _reference(which, prec)
    g = model.Grid.of(p, D)
    new = {b.sub: local.forward(local.LocalGeometry(g, maps, b.sub), np.asarray(xa[b.sub], D),
                                ref_rings[b.sub])
           for b in maps.boxes}
    new_rings, _ = dd.exchange(maps, new)
    xs = _perturbed(p, maps, trajs, seed=6)
    J, grad = ctx.cost_grad(ctx.pack_ctrl(xs))
    J = J.cpu().numpy()
    grads = ctx.unpack_ctrl(grad)
    for b in maps.boxes:
        s = b.sub
        Jr, gr = local.cost_grad(p, maps, s, xs[s], ref_trajs[s][0], new_rings[s],
                                 {k: new[k] for k in maps.neighbors[s]}, dtype=D)
        ej, eg = float(abs(J[s] - Jr) / abs(Jr)), float(_rel(grads[s], gr))
        assert ej <= TOL[prec] and eg <= TOL_GRAD[prec], (s, ej, eg)


def test_gather_partition_of_unity():
    p, maps, bg, trajs, rings = _oracle_state("small")
    ctx = _ctx("small", "fp64")
    xs = _perturbed(p, maps, trajs, seed=7)
    ctx.forward(ctx.pack_ctrl(xs), with_traj=False)
    g = model.Grid.of(p)
    lt = {b.sub: local.forward(local.LocalGeometry(g, maps, b.sub), xs[b.sub], rings[b.sub])
          for b in maps.boxes}
    for level in (0, 5, p.nsteps):
        out = ctx.gather(level).cpu().numpy()
        ref = dd.gather(p, maps, lt, level)
        assert _rel(_anom(out[None], p.h_ref), _anom(ref[None], p.h_ref)) <= 1e-13


def test_adjoint_before_forward_is_state_error():
    from paper_2205_06649_amd import _lib as L
    ctx = _ctx("tiny2", "fp64")
    with pytest.raises(L.DD4DVarError) as e:
        ctx.adjoint(None)
    assert e.value.status == L.DD4DVAR_E_STATE


@pytest.mark.parametrize("mode", [2, 3])
@pytest.mark.parametrize("which", ["tiny1", "c1", "small", "span", "mixed"])
def test_persistent_box_sweeps_fp32(which, mode):
    """One workgroup per box, level held in LDS (execution modes 2: one launch
    per sweep, 3: forward and adjoint fused in one launch): same trajectories
    and local cost/gradient as the oracle, FP32 bars."""
    from paper_2205_06649_amd import _lib as L
    p, maps, bg, trajs, rings = _oracle_state(which)
    ctx = _ctx(which, "fp32")
    ctx.set_exec_mode(mode)
    xs = _perturbed(p, maps, trajs, seed=8)
    g = model.Grid.of(p)
    traj = ctx.unpack_traj(ctx.forward(ctx.pack_ctrl(xs)))
    for b in maps.boxes:
        geo = local.LocalGeometry(g, maps, b.sub)
        ref = local.forward(geo, xs[b.sub], rings[b.sub])
        assert _rel(_anom(traj[b.sub], p.h_ref), _anom(ref, p.h_ref)) <= TOL_TRAJ["fp32"], b.sub
    J, grad = ctx.cost_grad(ctx.pack_ctrl(xs))
    J = J.cpu().numpy()
    grads = ctx.unpack_ctrl(grad)
    for b in maps.boxes:
        s = b.sub
        Jr, gr = local.cost_grad(p, maps, s, xs[s], trajs[s][0], rings[s],
                                 {k: trajs[k] for k in maps.neighbors[s]})
        ej, eg = float(abs(J[s] - Jr) / abs(Jr)), float(_rel(grads[s], gr))
        assert ej <= TOL["fp32"] and eg <= TOL_GRAD["fp32"], (s, ej, eg)
    # the fused and the separate launches run the same arithmetic
    ctx.set_exec_mode(5 - mode)
    J2, grad2 = ctx.cost_grad(ctx.pack_ctrl(xs))
    assert np.array_equal(J2.cpu().numpy(), J) and np.array_equal(grad2.cpu().numpy(), grad.cpu().numpy())
    # FP64 contexts keep the step kernels
    ctx64 = _ctx(which, "fp64")
    with pytest.raises(L.DD4DVarError) as e:
        ctx64.set_exec_mode(mode)
    assert e.value.status == L.DD4DVAR_E_INVALID


@functools.lru_cache(maxsize=None)
def _c3_sampled(dtype_name):
    """The 256 x 512 brick decomposition: sampled boxes of every size class
    and of the first, a middle and the last interval, with the trajectories
    of the background run (FP64, or extended precision) that they, their
    ring owners and their overlap neighbours need."""
    p = _prob("c3")
    maps = ddmaps.build(p)
    sizes = sorted(maps.boxes, key=lambda b: b.ncell)
    sample = sorted({sizes[0].sub, sizes[len(sizes) // 2].sub, sizes[-1].sub,
                     next(b.sub for b in maps.boxes if b.interval == 3),
                     next(b.sub for b in maps.boxes if b.interval == 7 and b.band == 4)})
    D = {"f64": np.float64, "ext": np.longdouble}[dtype_name]
    bg = model.forward(model.Grid.of(p, D), np.asarray(p.xb0, D), p.nsteps)
    need = set(sample)
    for s in sample:
        need |= {int(k) for k in maps.neighbors[s]} | {int(k) for k in maps.halo_src[s] if k >= 0}
    trajs = {k: local.restrict_global(maps, k, bg) for k in need}
    rings = {s: local.ring_from_trajs(maps, s, trajs) for s in sample}
    return p, maps, sample, trajs, rings


@pytest.mark.parametrize("prec,mode", [("fp64", 0), ("fp32", 0), ("fp32", 2), ("fp32", 4)])
def test_c3_sampled_subdomains(prec, mode):
    """The 256 x 512, 200-step brick decomposition (512 boxes of 945 to 8466
    cells) evaluated in one batched call; sampled boxes against the oracle,
    norm-wise and per field element-wise."""
    from test_gpu_strips import field_errors
    p, maps, sample, trajs0, _ = _c3_sampled("f64")
    _, _, _, trajs, rings = _c3_sampled("ext" if prec == "fp64" else "f64")
    rng = np.random.default_rng(31)
    ctx = _ctx("c3", prec)
    xb = ctx.unpack_ctrl(ctx.background_controls())
    xs = [(trajs0[b.sub][0] if b.sub in sample else x) +
          0.3 * p.sigma_b[:, None, None] * rng.standard_normal(x.shape)
          for b, x in zip(maps.boxes, xb)]
    ctx.set_exec_mode(mode)
    J, grad = ctx.cost_grad(ctx.pack_ctrl(xs))
    ctx.synchronize()
    J = J.cpu().numpy()
    grads = ctx.unpack_ctrl(grad)
    for s in sample:
        Jr, gr = local.cost_grad(p, maps, s, xs[s], trajs[s][0], rings[s],
                                 {k: trajs[k] for k in maps.neighbors[s]}, dtype=REF_DTYPE[prec])
        ej, eg = float(abs(J[s] - Jr) / abs(Jr)), float(_rel(grads[s], gr))
        ef = max(e for pair in field_errors(grads[s], gr) for e in pair)
        b = maps.boxes[s]
        print(f"c3 {prec} mode {mode} box {s} ({b.ny}x{b.nx}, interval {b.interval}): "
              f"J {ej:.2e} grad {eg:.2e} per-field {ef:.2e}", flush=True)
        assert ej <= TOL[prec] and eg <= TOL_GRAD[prec] and ef <= 10 * TOL_GRAD[prec], \
            (s, ej, eg, ef)
    ctx.close()
