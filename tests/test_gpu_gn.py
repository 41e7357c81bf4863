"""GPU parity of the Gauss-Newton local solver (Alg. 5 / Alg. 6) against the
FP64 oracle: the tangent-linear sweeps (the TLM step of Alg. 6), the normal
matrix products of eq. line5and7, and whole DD solves with Gauss-Newton
local solves.

Bars (norm-wise, relative, per subdomain): FP64 1e-12 for the tangent-linear
trajectories and the normal-matrix products; FP32 1e-4 (the FP32 state bar).
Solves: FP64 analysis within 1e-8 of the oracle's Gauss-Newton analysis,
relative to the analysis increment (the CG dot products round in another
order); FP32 within 1e-4 of the FP64 device solve, as for L-BFGS.
"""
import functools

import numpy as np
import pytest

from conftest import custom_problem, problem
from oracle import dd, ddmaps, gn, local, model
from test_oracle_pins import MIXED_CFG, SPAN_CFG

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-4, "fp32-box": 1e-4}
CASES = ["tiny1", "c1", "small", "span", "mixed"]
# "fp32-box": FP32 state with the persistent per-box kernels (execution mode 2)
PRECS = ["fp64", "fp32", "fp32-box"]


def _rel(a, b):
    a = np.asarray(a, dtype=np.longdouble)
    b = np.asarray(b, dtype=np.longdouble)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def _prob(which):
    if which == "span":
        return custom_problem(SPAN_CFG)
    if which == "mixed":
        return custom_problem(MIXED_CFG)
    return problem(which)


@functools.lru_cache(maxsize=None)
def _oracle_state(which):
    p = _prob(which)
    maps = ddmaps.build(p)
    bg, trajs = dd.background(p, maps)
    rings, _ = dd.exchange(maps, trajs)
    return p, maps, bg, trajs, rings


def _ctx(which, prec):
    from paper_2205_06649_amd.context import Context
    ctx = Context(_prob(which), precision=prec.split("-")[0])
    if prec.endswith("-box"):
        ctx.set_exec_mode(2)
    return ctx


def _controls(p, maps, trajs, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    sb = p.sigma_b[:, None, None]
    xs = [trajs[b.sub][0] + scale * sb * rng.standard_normal(trajs[b.sub][0].shape)
          for b in maps.boxes]
    dxs = [sb * rng.standard_normal(trajs[b.sub][0].shape) for b in maps.boxes]
    return xs, dxs


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("which", CASES)
def test_tangent_linear(which, prec):
    """dZ = M' dx about the stored trajectory, every level of every box,
    against the oracle's TLM (frozen ring unperturbed, wraps and poles)."""
    p, maps, bg, trajs, rings = _oracle_state(which)
    ctx = _ctx(which, prec)
    xs, dxs = _controls(p, maps, trajs, seed=21)
    ctx.forward(ctx.pack_ctrl(xs), with_traj=False)
    dt = ctx.unpack_traj(ctx.tangent_linear(ctx.pack_ctrl(dxs)))
    g = model.Grid.of(p)
    for b in maps.boxes:
        geo = local.LocalGeometry(g, maps, b.sub)
        lt = local.forward(geo, xs[b.sub], rings[b.sub])
        ref = local.tlm(geo, lt, rings[b.sub], dxs[b.sub])
        assert _rel(dt[b.sub], ref) <= TOL[prec], b.sub
    ctx.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("fp32-box", 1e-5)])
@pytest.mark.parametrize("which", ["c1", "span", "mixed"])
def test_tangent_linear_adjoint_dot_product(which, prec, tol):
    """<M' dx, y> = <dx, M'^T y> with the device TLM and the device adjoint
    (adjoint definition of Sec. 2), per subdomain."""
    p, maps, bg, trajs, rings = _oracle_state(which)
    ctx = _ctx(which, prec)
    xs, dxs = _controls(p, maps, trajs, seed=22)
    ctx.forward(ctx.pack_ctrl(xs), with_traj=False)
    dx = ctx.pack_ctrl(dxs)
    dt = ctx.unpack_traj(ctx.tangent_linear(dx))
    rng = np.random.default_rng(23)
    ys = [rng.standard_normal((b.nlev, 3, b.ny, b.nx)) for b in maps.boxes]
    at = ctx.unpack_ctrl(ctx.adjoint(ctx.pack_traj(ys)))
    for b in maps.boxes:
        s = b.sub
        lhs = float(np.sum(dt[s] * ys[s]))
        rhs = float(np.sum(dxs[s] * at[s]))
        assert abs(lhs - rhs) <= tol * abs(lhs), (s, lhs, rhs)
    ctx.close()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("which", CASES)
def test_gn_hessvec(which, prec):
    """(B_w^-1 + M'^T W M') dx against the oracle's normal-matrix product."""
    p, maps, bg, trajs, rings = _oracle_state(which)
    ctx = _ctx(which, prec)
    xs, dxs = _controls(p, maps, trajs, seed=24)
    ctx.forward(ctx.pack_ctrl(xs), with_traj=False)
    hv = ctx.unpack_ctrl(ctx.gn_hessvec(ctx.pack_ctrl(dxs)))
    g = model.Grid.of(p)
    for b in maps.boxes:
        geo = local.LocalGeometry(g, maps, b.sub)
        lt = local.forward(geo, xs[b.sub], rings[b.sub])
        ref = gn.hessvec(p, maps, b.sub, lt, rings[b.sub], dxs[b.sub])
        assert _rel(hv[b.sub], ref) <= TOL[prec], b.sub
    ctx.close()


def test_gn_hessvec_by_small_parts():
    """The background block of the normal-matrix product over parts of 64
    entries: the same bits as with the default parts (an entrywise term)."""
    p, maps, bg, trajs, rings = _oracle_state("mixed")
    ctx = _ctx("mixed", "fp64")
    xs, dxs = _controls(p, maps, trajs, seed=27)
    ctx.forward(ctx.pack_ctrl(xs), with_traj=False)
    h0 = ctx.gn_hessvec(ctx.pack_ctrl(dxs)).cpu().numpy()
    ctx.set_solver_parts(64)
    assert ctx.solver_parts()["parts"] > len(maps.boxes)
    h1 = ctx.gn_hessvec(ctx.pack_ctrl(dxs)).cpu().numpy()
    assert np.array_equal(h0, h1)
    ctx.close()


def test_gn_hessvec_symmetric_and_positive():
    """The normal matrix is symmetric positive definite: <u, A v> = <v, A u>
    and <v, A v> > 0 for every subdomain (FP64)."""
    p, maps, bg, trajs, rings = _oracle_state("mixed")
    ctx = _ctx("mixed", "fp64")
    xs, us = _controls(p, maps, trajs, seed=25)
    _, vs = _controls(p, maps, trajs, seed=26)
    ctx.forward(ctx.pack_ctrl(xs), with_traj=False)
    Au = ctx.unpack_ctrl(ctx.gn_hessvec(ctx.pack_ctrl(us)))
    Av = ctx.unpack_ctrl(ctx.gn_hessvec(ctx.pack_ctrl(vs)))
    for b in maps.boxes:
        s = b.sub
        a, c = float(np.sum(us[s] * Av[s])), float(np.sum(vs[s] * Au[s]))
        assert abs(a - c) <= 1e-12 * abs(a), s
        assert float(np.sum(vs[s] * Av[s])) > 0.0
    ctx.close()


@pytest.mark.parametrize("which,opts", [
    ("tiny2", dict(max_outer=2, max_iter=3, cg_max_iter=40)),
    ("c1", dict(max_outer=2, max_iter=2, cg_max_iter=25)),
    ("mixed", dict(max_outer=1, max_iter=2, cg_max_iter=20)),
])
@pytest.mark.parametrize("parts", [None, 100])
def test_gn_solve_matches_oracle(which, opts, parts):
    """Alg. 1 with Gauss-Newton local solves (fixed update and CG counts) in
    FP64 against the oracle's, on the analysis and on the local controls;
    also with the solver's vector work in parts of 100 entries (every box
    of several parts, CG's per-box scalars between part launches)."""
    p, maps, bg, trajs, rings = _oracle_state(which)
    xa_ref, rep_ref = dd.solve(p, maps, outer_tol=0.0, local_solver="gn", cg_rtol=0.0, **opts)
    ctx = _ctx(which, "fp64")
    if parts:
        ctx.set_solver_parts(parts)
    xa, rep, st, xo = ctx.solve(outer_tol=0.0, local_solver="gn", cg_rtol=0.0,
                                want_controls=True, **opts)
    inc = np.linalg.norm((xa_ref - p.xb0) / p.sigma_b[:, None, None])
    assert np.linalg.norm((xa - xa_ref) / p.sigma_b[:, None, None]) <= 1e-8 * inc
    xs = ctx.unpack_ctrl(xo)
    for b in maps.boxes:
        ref = rep_ref["controls"][b.sub]
        d = _rel((xs[b.sub] - trajs[b.sub][0]) / p.sigma_b[:, None, None],
                 (ref - trajs[b.sub][0]) / p.sigma_b[:, None, None])
        assert d <= 1e-8, (b.sub, d)
    assert rep.outer_iters == opts["max_outer"]
    assert rep.lbfgs_iters == opts["max_outer"] * opts["max_iter"]
    assert rep.gn_products == opts["max_outer"] * opts["max_iter"] * opts["cg_max_iter"]
    assert rep.total_evals == opts["max_outer"] * (opts["max_iter"] + 1)
    ctx.close()


@pytest.mark.parametrize("which,opts", [
    ("tiny2", dict(max_outer=2, max_iter=2, cg_max_iter=30)),
    ("c1", dict(max_outer=1, max_iter=2, cg_max_iter=20)),
])
@pytest.mark.parametrize("parts", [None, 100])
def test_gn_lanczos_solve_matches_oracle(which, opts, parts):
    """Gauss-Newton local solves whose normal equations are solved by the
    Lanczos method (Alg. 7), FP64, against the oracle's: analysis and local
    controls, product counts, the extreme Ritz values of the local
    preconditioned normal matrices; and against the device CG solve; also
    with the vector work in parts of 100 entries."""
    from paper_2205_06649_amd import _lib as L
    p, maps, bg, trajs, rings = _oracle_state(which)
    kw = dict(outer_tol=0.0, local_solver="gn", cg_rtol=0.0, **opts)
    xa_ref, rep_ref = dd.solve(p, maps, krylov="lanczos", **kw)
    ctx = _ctx(which, "fp64")
    if parts:
        ctx.set_solver_parts(parts)
    xa, rep, st, xo = ctx.solve(krylov="lanczos", want_controls=True, **kw)
    sb = p.sigma_b[:, None, None]
    inc = np.linalg.norm((xa_ref - p.xb0) / sb)
    assert np.linalg.norm((xa - xa_ref) / sb) <= 1e-8 * inc
    xs = ctx.unpack_ctrl(xo)
    for b in maps.boxes:
        ref = rep_ref["controls"][b.sub]
        d = _rel((xs[b.sub] - trajs[b.sub][0]) / sb, (ref - trajs[b.sub][0]) / sb)
        assert d <= 1e-8, (b.sub, d)
    assert rep.gn_products == opts["max_outer"] * opts["max_iter"] * opts["cg_max_iter"]
    rmax = rep_ref["ritz_max"]
    print(f"{which}: Ritz values {rep.ritz_min:.6e} .. {rep.ritz_max:.6e} "
          f"(oracle {rep_ref['ritz_min']:.6e} .. {rmax:.6e})", flush=True)
    assert 0.0 < rep.ritz_min <= rep.ritz_max
    assert abs(rep.ritz_max - rmax) <= 1e-6 * rmax
    assert abs(rep.ritz_min - rep_ref["ritz_min"]) <= 1e-6 * rmax
    xc, repc, _, _ = ctx.solve(**kw)
    assert repc.ritz_min == 0.0 and repc.ritz_max == 0.0
    assert np.linalg.norm((xa - xc) / sb) <= 1e-6 * inc
    with pytest.raises(L.DD4DVarError) as e:
        ctx.solve(max_outer=1, max_iter=1, krylov="lanczos")
    assert e.value.status == L.DD4DVAR_E_INVALID
    ctx.close()


def test_gn_lanczos_fp32_products():
    """Lanczos with FP32 state sweeps (persistent kernels) against the FP64
    Lanczos solve: analysis within the FP32 bar."""
    opts = dict(max_outer=2, max_iter=3, cg_max_iter=30, cg_rtol=1e-8, outer_tol=0.0,
                local_solver="gn", krylov="lanczos")
    res = {}
    for pr in ("fp64", "fp32-box"):
        ctx = _ctx("c2", pr)
        xa, rep, st, _ = ctx.solve(**opts)
        res[pr] = (xa, rep.ritz_max)
        ctx.close()
    ref = res["fp64"][0]
    err = max(np.linalg.norm(res["fp32-box"][0][f] - ref[f]) / np.linalg.norm(ref[f] - ref[f].mean())
              for f in range(3))
    assert err <= 1e-4, err
    assert abs(res["fp32-box"][1] - res["fp64"][1]) <= 1e-3 * res["fp64"][1]


@pytest.mark.parametrize("prec", ["fp32", "fp32-box"])
def test_gn_solve_fp32_against_fp64(prec):
    """FP32 state sweeps (step kernels, or the persistent per-box kernels)
    with the FP64 CG: analysis within the FP32 bar of the FP64 device solve
    (per field, relative to the spread of the analysis)."""
    opts = dict(max_outer=2, max_iter=3, cg_max_iter=30, cg_rtol=1e-8, outer_tol=0.0,
                local_solver="gn")
    res = {}
    for pr in ("fp64", prec):
        ctx = _ctx("c2", pr)
        xa, rep, st, _ = ctx.solve(**opts)
        res[pr] = xa
        ctx.close()
    ref = res["fp64"]
    err = max(np.linalg.norm(res[prec][f] - ref[f]) / np.linalg.norm(ref[f] - ref[f].mean())
              for f in range(3))
    assert err <= 1e-4, err


def test_gn_mixed_solve_reaches_the_fp64_stationary_point():
    """Mixed precision (FP64 evaluations, FP32 normal-matrix products): the
    local gradients fall below 1e-6 of their start like the FP64 solve's,
    where the FP32-only solve stops at its rounding floor, and the analysis
    is the FP64 solve's to 1e-7 of the increment."""
    from paper_2205_06649_amd.context import Context
    p = _prob("c2")
    opts = dict(max_outer=2, max_iter=4, cg_max_iter=60, cg_rtol=1e-8, grad_rtol=1e-9,
                outer_tol=0.0, local_solver="gn")
    c64 = Context(p, "fp64")
    xa64, r64, _, _ = c64.solve(**opts)
    c32 = Context(p, "fp32")
    c32.set_exec_mode(2)
    xa32, r32, _, _ = c32.solve(**opts)
    c64b = Context(p, "fp64")
    xam, rm, _, _ = c64b.solve(products=c32, **opts)
    print(f"gradient ratios: fp64 {r64.gnorm_ratio_max:.2e}, fp32 {r32.gnorm_ratio_max:.2e}, "
          f"mixed {rm.gnorm_ratio_max:.2e}", flush=True)
    assert r64.gnorm_ratio_max <= 1e-6 and rm.gnorm_ratio_max <= 1e-6
    assert r32.gnorm_ratio_max > rm.gnorm_ratio_max
    sb = p.sigma_b[:, None, None]
    inc = np.linalg.norm((xa64 - p.xb0) / sb)
    assert np.linalg.norm((xam - xa64) / sb) <= 1e-7 * inc
    for c in (c64, c32, c64b):
        c.close()


def test_gn_mixed_rules():
    from paper_2205_06649_amd import _lib as L
    from paper_2205_06649_amd.context import Context
    p = _prob("c1")
    c64, c32, c32b = Context(p, "fp64"), Context(p, "fp32"), Context(p, "fp32")
    other = Context(_prob("tiny1"), "fp32")
    gn_opts = dict(max_outer=1, max_iter=1, cg_max_iter=2, local_solver="gn")
    for ctx, lo, kw in ((c32b, c32, gn_opts), (c64, c64, gn_opts), (c64, other, gn_opts),
                        (c64, c32, dict(max_outer=1, max_iter=1))):
        with pytest.raises(L.DD4DVarError) as e:
            ctx.solve(products=lo, **kw)
        assert e.value.status == L.DD4DVAR_E_INVALID
    c32.set_checkpointing(3)
    with pytest.raises(L.DD4DVarError) as e:
        c64.solve(products=c32, **gn_opts)
    assert e.value.status == L.DD4DVAR_E_INVALID
    c32.set_checkpointing(0)
    xa, rep, st, _ = c64.solve(products=c32, **gn_opts)
    assert np.all(np.isfinite(xa)) and rep.gn_products == 2
    for c in (c64, c32, c32b, other):
        c.close()


def test_gn_rules():
    from paper_2205_06649_amd import _lib as L
    p, maps, bg, trajs, rings = _oracle_state("c1")
    ctx = _ctx("c1", "fp64")
    xs, dxs = _controls(p, maps, trajs, seed=28)
    dx = ctx.pack_ctrl(dxs)
    with pytest.raises(L.DD4DVarError) as e:
        ctx.tangent_linear(dx)
    assert e.value.status == L.DD4DVAR_E_STATE
    with pytest.raises(L.DD4DVarError) as e:
        ctx.gn_hessvec(dx)
    assert e.value.status == L.DD4DVAR_E_STATE
    ctx.forward(ctx.pack_ctrl(xs), with_traj=False)
    with pytest.raises(L.DD4DVarError) as e:
        L.dd4dvar_gn_hessvec(ctx.handle, dx.data_ptr(), dx.data_ptr())
    assert e.value.status == L.DD4DVAR_E_INVALID
    for kw in (dict(cg_max_iter=-1), dict(cg_rtol=-1.0), dict(cg_rtol=float("nan"))):
        with pytest.raises(L.DD4DVarError) as e:
            ctx.solve(max_outer=1, max_iter=1, local_solver="gn", **kw)
        assert e.value.status == L.DD4DVAR_E_INVALID
    o = L.dd4dvar_solve_opts(lbfgs_m=8, max_iter=1, max_outer=1, max_ls=30, grad_rtol=0.0,
                             outer_tol=0.0, armijo_c1=1e-4, j_noise_rtol=0.0, local_solver=2,
                             cg_max_iter=5, cg_rtol=0.0)
    with pytest.raises(L.DD4DVarError) as e:
        L.dd4dvar_solve(ctx.handle, o, None, None, np.empty((3, p.nlat, p.nlon)))
    assert e.value.status == L.DD4DVAR_E_INVALID
    # checkpointed trajectories are refused by every Gauss-Newton path
    ctx.set_checkpointing(3)
    ctx.forward(ctx.pack_ctrl(xs), with_traj=False)
    for call in (lambda: ctx.tangent_linear(dx), lambda: ctx.gn_hessvec(dx),
                 lambda: ctx.solve(max_outer=1, max_iter=1, local_solver="gn")):
        with pytest.raises(L.DD4DVarError) as e:
            call()
        assert e.value.status == L.DD4DVAR_E_INVALID
    ctx.close()
