"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names the passage it pins.  None of these re-types an oracle
formula: they check identities (adjoint definition, reverse product rule),
closed forms (normal equations), conservation, continuous steady states,
special cases (one subdomain = global 4D-Var, J = sum of local J), and brute
force on tiny inputs.
"""
import math

import numpy as np
import pytest

import synth
from conftest import custom_problem, problem
from oracle import brute, dd, ddmaps, gn, lbfgs, local, model, tz_local


def _grid(p):
    return model.Grid.of(p)


# --- P1: the rest state is an exact fixed point ------------------------------
def test_rest_state_is_fixed_point():
    """All tendencies of EquU/EquV/EquH vanish at h = const, u = v = 0 (Sec. 7)."""
    p = problem("c1")
    g = _grid(p)
    Z = np.stack([np.full((p.nlat, p.nlon), p.h_ref), np.zeros((p.nlat, p.nlon)),
                  np.zeros((p.nlat, p.nlon))])
    assert np.all(model.increment(g, Z) == 0.0)
    tr = model.forward(g, Z, 5)
    assert np.all(tr == Z[None])
    maps = ddmaps.build(p)
    for s in (0, 3, 5):
        b = maps.boxes[s]
        geo = local.LocalGeometry(g, maps, s)
        zb = local.restrict_global(maps, s, np.repeat(Z[None], p.nsteps + 1, 0))
        ring = local.ring_from_trajs(maps, s, {k: local.restrict_global(
            maps, k, np.repeat(Z[None], p.nsteps + 1, 0)) for k in range(len(maps.boxes))})
        lt = local.forward(geo, zb[0], ring)
        assert np.all(lt == zb[0][None]), b


# --- P2: mass conservation of the flux form ----------------------------------
@pytest.mark.parametrize("name", ["c1", "small"])
def test_mass_conservation(name):
    """Flux-form continuity (EquH) conserves sum_j cos(theta_j) h_ij exactly."""
    p = problem(name)
    g = _grid(p)
    tr = model.forward(g, p.xb0, p.nsteps)
    m = np.array([model.mass(g, z) for z in tr])
    assert np.max(np.abs(m - m[0])) / m[0] <= 1e-13
    # the total increment of h is exactly mass-neutral, level by level
    for z in tr[::3]:
        H = model.increment(g, z)[0]
        assert abs(np.sum(g.cos[:, None] * H)) <= 1e-13 * np.sum(g.cos[:, None] * np.abs(z[0]))


# --- the discrete U, V, H approximate the continuous SWE --------------------
def _tc2(nlat, omega, alpha):
    """Solid-body rotation about an axis tilted by alpha (steady for alpha=0,
    or for any alpha when omega = 0)."""
    nlon = 2 * nlat
    a, gr = 6.37122e6, 9.80616
    g = model.Grid(nlat, nlon, 10.0, a, gr, omega)
    u0 = 2 * math.pi * a / (12 * 86400.0)
    th = g.theta[:, None] * np.ones((1, nlon))
    la = (np.arange(nlon) * g.dlon)[None, :] * np.ones((nlat, 1))
    u = u0 * (np.cos(th) * math.cos(alpha) + np.cos(la) * np.sin(th) * math.sin(alpha))
    v = -u0 * np.sin(la) * math.sin(alpha)
    mu = -np.cos(la) * np.cos(th) * math.sin(alpha) + np.sin(th) * math.cos(alpha)
    h = 2.94e4 / gr - (a * omega * u0 + u0 ** 2 / 2) * mu ** 2 / gr
    return g, np.stack([h, u, v])


@pytest.mark.parametrize("omega,alpha", [(7.292e-5, 0.0), (0.0, math.pi / 4), (0.0, 0.3)])
def test_steady_flow_second_order(omega, alpha):
    """Williamson-type solid-body rotation is a steady solution of EquU/EquV/EquH.

    The discrete increment must vanish at second order in the grid spacing:
    halving the spacing divides the residual (relative to the pressure-gradient
    term) by about four.  A wrong sign or factor in any advection, metric,
    Coriolis or pressure term leaves an O(1) residual instead.
    """
    res = []
    for nlat in (32, 64, 128):
        g, Z = _tc2(nlat, omega, alpha)
        F = model.increment(g, Z)
        h = Z[0]
        # compare on |latitude| < 60 deg: towards the poles the 1/cos(theta)
        # factors turn the centred-difference error at a fixed number of rows
        # from the pole into a first-order one
        band = np.abs(g.theta) < math.pi / 3
        scale = np.linalg.norm((g.sig_lat * g.gravity * (np.roll(h, -1, 0) - np.roll(h, 1, 0)))[band])
        res.append(max(np.linalg.norm(F[k][band]) for k in range(3)) / scale)
    assert res[0] < 0.05
    assert 3.0 < res[0] / res[1] < 5.0 and 3.0 < res[1] / res[2] < 5.0, res


def test_time_integration_second_order():
    """Leapfrog with a forward-Euler half increment is second order in dt."""
    p = problem("c1")
    T = 20 * p.dt
    out = []
    for k in (1, 2, 4):
        g = model.Grid(p.nlat, p.nlon, p.dt / k, p.radius, p.gravity, p.omega)
        out.append(model.forward(g, p.truth0, 20 * k)[-1])
    e1 = np.linalg.norm(out[0] - out[1])
    e2 = np.linalg.norm(out[1] - out[2])
    assert 3.0 < e1 / e2 < 5.0
    assert T > 0


def test_brute_force_increment():
    """Vectorised increment equals a per-cell loop transcription on tiny grids."""
    for name in ("tiny1", "c1"):
        p = problem(name)
        g = _grid(p)
        for Z in (p.truth0, p.xb0):
            F = model.increment(g, Z)
            Fb = np.array(brute.increment(p, Z.tolist()))
            assert np.max(np.abs(F - Fb)) <= 1e-15 * np.max(np.abs(F)) + 1e-300


# --- P3 / P4: dot-product tests (adjoint definition, eq. Eq_propAdj) --------
def test_global_dot_product(rng):
    p = problem("c1")
    g = _grid(p)
    tr = model.forward(g, p.xb0, p.nsteps)
    dx = rng.standard_normal(p.xb0.shape)
    y = rng.standard_normal(tr.shape)
    lhs = np.sum(model.tlm(g, tr, dx) * y)
    rhs = np.sum(dx * model.adjoint(g, tr, y))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_single_step_dot_product(rng):
    """Per-step transposes (reverse product rule, eq. adjProd)."""
    p = problem("c1")
    g = _grid(p)
    for Z in (p.truth0, p.xb0):
        dZ = rng.standard_normal(Z.shape)
        lam = rng.standard_normal(Z.shape)
        lhs = np.sum(model.increment_tl(g, Z, dZ) * lam)
        rhs = np.sum(dZ * model.increment_ad(g, Z, lam))
        assert abs(lhs - rhs) <= 1e-14 * abs(lhs)
    # startup step alone: trajectory with one step
    tr = model.forward(g, p.xb0, 1)
    dx = rng.standard_normal(p.xb0.shape)
    y = rng.standard_normal(tr.shape)
    lhs = np.sum(model.tlm(g, tr, dx) * y)
    rhs = np.sum(dx * model.adjoint(g, tr, y))
    assert abs(lhs - rhs) <= 1e-14 * abs(lhs)


SPAN_CFG = dict(index=110, nlat=16, nlon=32, nsteps=8, bands=3, pieces=1, ntime=2,
                overlap_cells=2, overlap_steps=1, obs_frac=0.1, obs_every=2)
MIXED_CFG = dict(index=111, nlat=24, nlon=32, brick=(3, 2, 6, 18), ntime=2,
                 nsteps=8, overlap_cells=2, overlap_steps=2, obs_frac=0.1, obs_every=2)


def _local_setup(p):
    g = _grid(p)
    maps = ddmaps.build(p)
    bg, trajs = dd.background(p, maps)
    rings, _ = dd.exchange(maps, trajs)
    return g, maps, trajs, rings


@pytest.mark.parametrize("which", ["c1", "small", "span", "mixed"])
def test_local_dot_product(rng, which):
    """Local sweep control -> all levels, boxes with rings, seams and poles."""
    p = {"span": lambda: custom_problem(SPAN_CFG), "mixed": lambda: custom_problem(MIXED_CFG)}.get(
        which, lambda: problem(which))()
    g, maps, trajs, rings = _local_setup(p)
    for s in range(len(maps.boxes)):
        geo = local.LocalGeometry(g, maps, s)
        x = trajs[s][0] + 0.3 * p.sigma_b[:, None, None] * rng.standard_normal(trajs[s][0].shape)
        lt = local.forward(geo, x, rings[s])
        dx = rng.standard_normal(x.shape)
        y = rng.standard_normal(lt.shape)
        lhs = np.sum(local.tlm(geo, lt, rings[s], dx) * y)
        rhs = np.sum(dx * local.adjoint(geo, lt, rings[s], y))
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs), s
        # one step
        P = geo.pad(x, rings[s][0])
        dP = geo.pad(dx, None)
        lam = rng.standard_normal(x.shape)
        lhs = np.sum(local.increment_tl(geo, P, dP) * lam)
        rhs = np.sum(dx * local.increment_ad(geo, P, lam))
        assert abs(lhs - rhs) <= 1e-14 * abs(lhs)


# --- P6: TLM against finite differences of the forward ----------------------
def test_tlm_matches_finite_differences(rng):
    p = problem("small")
    g, maps, trajs, rings = _local_setup(p)
    s = 4
    geo = local.LocalGeometry(g, maps, s)
    x = trajs[s][0]
    dx = p.sigma_b[:, None, None] * rng.standard_normal(x.shape)
    lt = local.forward(geo, x, rings[s])
    tl = local.tlm(geo, lt, rings[s], dx)
    errs = []
    for eps in (1e-1, 5e-2):
        fd = (local.forward(geo, x + eps * dx, rings[s]) - local.forward(geo, x - eps * dx, rings[s])) / (2 * eps)
        errs.append(np.linalg.norm(fd - tl) / np.linalg.norm(tl))
    assert errs[0] < 1e-4
    assert 3.0 < errs[0] / errs[1] < 5.0   # O(eps^2)


# --- P5: gradient of the full local functional vs finite differences -------
@pytest.mark.parametrize("which", ["c1", "span"])
def test_local_gradient_finite_differences(rng, which):
    """Discretize-then-optimize (Sec. 1): the gradient is that of the discrete J."""
    p = problem("c1") if which == "c1" else custom_problem(SPAN_CFG)
    g, maps, trajs, rings = _local_setup(p)
    sb = p.sigma_b[:, None, None]
    for s in range(len(maps.boxes)):
        xb = trajs[s][0]
        x = xb + 0.5 * sb * rng.standard_normal(xb.shape)
        nb = {k: trajs[k] for k in maps.neighbors[s]}
        J, gr = local.cost_grad(p, maps, s, x, xb, rings[s], nb)
        d = sb * rng.standard_normal(xb.shape)
        an = np.sum(gr * d)
        errs = []
        for eps in (1e-3, 5e-4):
            Jp = local.cost_grad(p, maps, s, x + eps * d, xb, rings[s], nb, with_grad=False)
            Jm = local.cost_grad(p, maps, s, x - eps * d, xb, rings[s], nb, with_grad=False)
            errs.append(abs((Jp - Jm) / (2 * eps) - an) / abs(an))
        assert errs[1] < 1e-6, (s, errs)


def test_global_gradient_finite_differences(rng):
    p = problem("c1")
    sb = p.sigma_b[:, None, None]
    x = p.xb0 + 0.5 * sb * rng.standard_normal(p.xb0.shape)
    J, gr = model.cost_grad(p, x)
    d = sb * rng.standard_normal(x.shape)
    an = np.sum(gr * d)
    eps = 5e-4
    fd = (model.cost_grad(p, x + eps * d, False) - model.cost_grad(p, x - eps * d, False)) / (2 * eps)
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_fp64_rounding_floor_against_extended_precision(rng):
    """The same local functional evaluated in 80-bit extended precision: the
    FP64 evaluation agrees to the rounding floor of the computation (J to
    ~1e-13, the gradient to ~1e-12 because the adjoint sums h-weighted terms
    that cancel).  This fixes how close any FP64 implementation can get."""
    p = problem("c1")
    g, maps, trajs, rings = _local_setup(p)
    sb = p.sigma_b[:, None, None]
    worst_j = worst_g = 0.0
    for s in range(len(maps.boxes)):
        x = trajs[s][0] + 0.3 * sb * rng.standard_normal(trajs[s][0].shape)
        nb = {k: trajs[k] for k in maps.neighbors[s]}
        J, gr = local.cost_grad(p, maps, s, x, trajs[s][0], rings[s], nb)
        JL, gL = local.cost_grad(p, maps, s, x, trajs[s][0], rings[s], nb, dtype=np.longdouble)
        assert JL.dtype == np.longdouble
        worst_j = max(worst_j, float(abs(J - JL) / abs(JL)))
        worst_g = max(worst_g, float(np.linalg.norm(gr - gL) / np.linalg.norm(gL)))
    assert worst_j < 1e-12 and worst_g < 2e-12, (worst_j, worst_g)
    assert worst_g > 1e-15     # the extended evaluation really is different


def test_fp64_pipeline_floor_against_extended_pipeline(rng):
    """The whole pipeline in extended precision (background run, rings,
    overlap targets, background controls and evaluation, from the same FP64
    x_b0, observations and controls) is the FP64 parity reference.  The FP64
    pipeline lands up to a few 1e-12 from it: its background run carries the
    full depth (1e4 m), so its rounding (~1e-12 m) enters the observation and
    overlap residuals, which are metre-sized differences of depths.  An
    evaluation that keeps h - h_ref avoids most of that."""
    p = problem("c1")
    g, maps, trajs, rings = _local_setup(p)
    _, trajs_e = dd.background(p, maps, np.longdouble)
    rings_e, _ = dd.exchange(maps, trajs_e)
    bg = np.stack([trajs[s][0] for s in range(len(maps.boxes))])
    bg_e = np.stack([trajs_e[s][0] for s in range(len(maps.boxes))])
    d_anom = float(np.abs(bg[:, 0] - bg_e[:, 0]).max())
    assert 1e-14 < d_anom < 1e-10            # rounding of the FP64 run, in metres
    sb = p.sigma_b[:, None, None]
    worst = 0.0
    for s in range(len(maps.boxes)):
        x = trajs[s][0] + 0.3 * sb * rng.standard_normal(trajs[s][0].shape)
        J, gr = local.cost_grad(p, maps, s, x, trajs[s][0], rings[s],
                                {k: trajs[k] for k in maps.neighbors[s]})
        JE, gE = local.cost_grad(p, maps, s, x, trajs_e[s][0], rings_e[s],
                                 {k: trajs_e[k] for k in maps.neighbors[s]}, dtype=np.longdouble)
        assert float(abs(J - JE) / abs(JE)) < 1e-12
        worst = max(worst, float(np.linalg.norm(gr - gE) / np.linalg.norm(gE)))
    assert 1e-14 < worst < 4e-12, worst


# --- P12: brute-force Jacobian of a tiny box vs adjoint rows ----------------
def test_bruteforce_jacobian_tiny_box():
    p = problem("tiny2")
    g, maps, trajs, rings = _local_setup(p)
    s = 5
    geo = local.LocalGeometry(g, maps, s)
    x = trajs[s][0]
    lt = local.forward(geo, x, rings[s])
    n_in = x.size
    n_out = lt.size
    Jfd = np.empty((n_out, n_in))
    for i in range(n_in):
        e = np.zeros(n_in)
        e[i] = 1e-3 * p.sigma_b[i // (x.size // 3)]
        xp = local.forward(geo, x + e.reshape(x.shape), rings[s])
        xm = local.forward(geo, x - e.reshape(x.shape), rings[s])
        Jfd[:, i] = ((xp - xm) / (2 * e[i])).ravel()
    Jad = np.empty_like(Jfd)
    for j in range(n_out):
        y = np.zeros(n_out)
        y[j] = 1.0
        Jad[j] = local.adjoint(geo, lt, rings[s], y.reshape(lt.shape)).ravel()
    assert np.max(np.abs(Jad - Jfd)) <= 1e-6 * np.max(np.abs(Jad))


# --- P8: one subdomain reproduces global 4D-Var -----------------------------
def test_one_subdomain_equals_global(rng):
    """With P = Q = 1 the local functional is the global one (eq. min3sec)."""
    p = problem("tiny1")
    maps = ddmaps.build(p)
    assert len(maps.boxes) == 1 and (maps.halo_src[0] < 0).all()
    for _ in range(3):
        x = p.xb0 + p.sigma_b[:, None, None] * rng.standard_normal(p.xb0.shape)
        Jg, gg = model.cost_grad(p, x)
        Jl, gl = local.cost_grad(p, maps, 0, x, p.xb0, None, {})
        assert abs(Jg - Jl) <= 1e-14 * Jg
        assert np.max(np.abs(gg - gl)) <= 1e-13 * np.max(np.abs(gg))
    # a bigger single box too
    cfg = dict(synth.CONFIGS["c1"], bands=1, pieces=1, ntime=1, overlap_cells=0,
               overlap_steps=0, index=112)
    p = custom_problem(cfg)
    maps = ddmaps.build(p)
    x = p.xb0 + p.sigma_b[:, None, None] * rng.standard_normal(p.xb0.shape)
    Jg, gg = model.cost_grad(p, x)
    Jl, gl = local.cost_grad(p, maps, 0, x, p.xb0, None, {})
    assert abs(Jg - Jl) <= 1e-14 * Jg
    assert np.linalg.norm(gg - gl) <= 1e-13 * np.linalg.norm(gg)


# --- P9: J = sum of the extended local functionals (eq. restJ) --------------
@pytest.mark.parametrize("which", ["c1", "mixed", "span"])
def test_cost_is_sum_of_local_costs(rng, which):
    """With one time interval and rings/targets from the global trajectory of x,
    the weighted local functionals sum to the global one at any x."""
    base = {"c1": synth.CONFIGS["c1"], "mixed": MIXED_CFG, "span": SPAN_CFG}[which]
    cfg = dict(base, ntime=1, index=base["index"] + 50)
    p = custom_problem(cfg)
    g = _grid(p)
    maps = ddmaps.build(p)
    x = p.xb0 + p.sigma_b[:, None, None] * rng.standard_normal(p.xb0.shape)
    gt = model.forward(g, x, p.nsteps)
    trajs = {b.sub: local.restrict_global(maps, b.sub, gt) for b in maps.boxes}
    xb0 = p.xb0[None]
    total = 0.0
    for b in maps.boxes:
        ring = local.ring_from_trajs(maps, b.sub, trajs)
        xbs = local.restrict_global(maps, b.sub, xb0)[0]
        J, parts = local.cost_grad(p, maps, b.sub, trajs[b.sub][0], xbs, ring,
                                   {k: trajs[k] for k in maps.neighbors[b.sub]},
                                   with_grad=False, parts=True)
        assert parts[2] == 0.0   # overlap copies agree exactly
        total += J
    Jg = model.cost_grad(p, x, with_grad=False)
    assert abs(total - Jg) <= 1e-13 * Jg


# --- P11: background is the minimizer without observations -----------------
def test_background_minimizer_without_obs():
    p = problem("c1")
    p = p.replace(obs_step=p.obs_step[:0], obs_cell=p.obs_cell[:0], obs_field=p.obs_field[:0],
                  obs_value=p.obs_value[:0], obs_sigma=p.obs_sigma[:0], obs_noise=p.obs_noise[:0])
    cfg_q1 = p.replace(time_edges=np.array([0, p.nsteps], dtype=np.int32))
    for q in (p, cfg_q1):
        maps = ddmaps.build(q)
        bg, trajs = dd.background(q, maps)
        rings, _ = dd.exchange(maps, trajs)
        for s in range(len(maps.boxes)):
            nb = {k: trajs[k] for k in maps.neighbors[s]}
            if q is p:
                qq = q.replace(mu_overlap=0.0)
            else:
                qq = q     # one interval: the local model reproduces the background
            J, gr = local.cost_grad(qq, maps, s, trajs[s][0], trajs[s][0], rings[s], nb)
            assert J == 0.0 and np.all(gr == 0.0)


# --- P7: normal equations closed form on a tiny linearized case -------------
def _dense_tlm(step_fn, n_in):
    cols = []
    for i in range(n_in):
        e = np.zeros(n_in)
        e[i] = 1.0
        cols.append(step_fn(e).ravel())
    return np.array(cols).T


def test_normal_equations_global():
    """delta x* = (B^-1 + G^T R^-1 G)^-1 G^T R^-1 d (eqs. line5and7, line6and7)
    equals the L-BFGS minimizer of the linearized J built from TLM/adjoint, and
    grad J(x_b) = -G^T R^-1 d."""
    p = problem("tiny1")
    g = _grid(p)
    tr = model.forward(g, p.xb0, p.nsteps)
    n = p.xb0.size
    Mfull = _dense_tlm(lambda e: model.tlm(g, tr, e.reshape(p.xb0.shape)), n)
    rows = (p.obs_step.astype(np.int64) * n + p.obs_field.astype(np.int64) * (n // 3)
            + p.obs_cell.astype(np.int64))
    G = Mfull[rows]
    Rinv = p.lambda_obs / p.obs_sigma ** 2
    Binv = np.repeat(1.0 / p.sigma_b ** 2, n // 3)
    d = p.obs_value - tr.ravel()[rows]
    A = np.diag(Binv) + G.T @ (Rinv[:, None] * G)
    rhs = G.T @ (Rinv * d)
    dx_star = np.linalg.solve(A, rhs)
    # gradient identity at the background
    _, gb = model.cost_grad(p, p.xb0)
    assert np.max(np.abs(gb.ravel() + rhs)) <= 1e-12 * np.max(np.abs(rhs))
    # L-BFGS on the linearized functional, in xi = dx / sigma_b

    sb = np.repeat(p.sigma_b, n // 3)

    def fun(xi):
        dx = sb * xi
        Gd = (model.tlm(g, tr, dx.reshape(p.xb0.shape)).ravel())[rows]
        r = Gd - d
        J = 0.5 * np.sum(Binv * dx * dx) + 0.5 * np.sum(Rinv * r * r)
        forcing = np.zeros(tr.size)
        np.add.at(forcing, rows, Rinv * r)
        gr = Binv * dx + model.adjoint(g, tr, forcing.reshape(tr.shape)).ravel()
        return J, sb * gr

    res = lbfgs.minimize(fun, np.zeros(n), m=8, max_iter=500, grad_rtol=1e-13)
    dx_l = sb * res["x"]
    assert np.linalg.norm(dx_l - dx_star) <= 1e-8 * np.linalg.norm(dx_star)


def _dense_normal_matrix(p, maps, s, g, rings, x):
    """Dense B^-1 + M^T W M of subdomain s about control x, from TLM columns
    and weights W enumerated residual by residual."""
    b = maps.boxes[s]
    geo = local.LocalGeometry(g, maps, s)
    lt = local.forward(geo, x, rings[s])
    n = x.size
    M = _dense_tlm(lambda e: local.tlm(geo, lt, rings[s], e.reshape(x.shape)), n)
    W = np.zeros(lt.size)
    flat_idx = np.arange(lt.size).reshape(b.nlev, 3, -1)
    _, csp = local.weights(p, maps, s)
    for o in maps.obs_bin[s]:
        cell = int(p.obs_cell[o])
        loc = int(maps.box_index(b, cell // p.nlon, cell % p.nlon))
        k = int(p.obs_step[o])
        w = 1.0 / (csp[loc] * maps.time_count[k])
        W[flat_idx[k - b.lev0, int(p.obs_field[o]), loc]] += p.lambda_obs * w / p.obs_sigma[o] ** 2
    gr_, gc_ = maps.box_cells_global(b)
    for sp in maps.neighbors[s]:
        bp = maps.boxes[int(sp)]
        mine = np.nonzero(maps.box_index(bp, gr_, gc_) >= 0)[0]
        for lev in range(max(b.lev0, bp.lev0), min(b.lev0 + b.nlev, bp.lev0 + bp.nlev)):
            for f in range(3):
                W[flat_idx[lev - b.lev0, f, mine]] += p.mu_overlap / p.sigma_b[f] ** 2
    Binv = (local.weights(p, maps, s)[0][None, :] / (p.sigma_b ** 2)[:, None]).ravel()
    return np.diag(Binv) + M.T @ (W[:, None] * M), lt, W


def test_normal_equations_local():
    """Same closed form for one subdomain of a 2x2x2 decomposition: obs and
    overlap penalties act as weighted observations of the local trajectory,
    so the Gauss-Newton normal matrix is B^-1 + M^T W M with M the dense TLM."""
    p = problem("tiny2")
    g, maps, trajs, rings = _local_setup(p)
    s = 6
    b = maps.boxes[s]
    geo = local.LocalGeometry(g, maps, s)
    xb = trajs[s][0]
    lt = local.forward(geo, xb, rings[s])
    n = xb.size
    M = _dense_tlm(lambda e: local.tlm(geo, lt, rings[s], e.reshape(xb.shape)), n)
    nb = {k: trajs[k] for k in maps.neighbors[s]}
    J0, g0 = local.cost_grad(p, maps, s, xb, xb, rings[s], nb)
    # weights of the squared residuals, entry by entry of the local trajectory
    W = np.zeros(lt.size)
    flat_idx = np.arange(lt.size).reshape(b.nlev, 3, -1)
    _, csp = local.weights(p, maps, s)
    for o in maps.obs_bin[s]:
        cell = int(p.obs_cell[o])
        loc = int(maps.box_index(b, cell // p.nlon, cell % p.nlon))
        k = int(p.obs_step[o])
        w = 1.0 / (csp[loc] * maps.time_count[k])
        W[flat_idx[k - b.lev0, int(p.obs_field[o]), loc]] += p.lambda_obs * w / p.obs_sigma[o] ** 2
    gr_, gc_ = maps.box_cells_global(b)
    for sp in maps.neighbors[s]:
        bp = maps.boxes[int(sp)]
        mine = np.nonzero(maps.box_index(bp, gr_, gc_) >= 0)[0]
        for lev in range(max(b.lev0, bp.lev0), min(b.lev0 + b.nlev, bp.lev0 + bp.nlev)):
            for f in range(3):
                W[flat_idx[lev - b.lev0, f, mine]] += p.mu_overlap / p.sigma_b[f] ** 2
    Binv = (local.weights(p, maps, s)[0][None, :] / (p.sigma_b ** 2)[:, None]).ravel()
    A = np.diag(Binv) + M.T @ (W[:, None] * M)
    dx_star = np.linalg.solve(A, -g0.ravel())
    sb = np.repeat(p.sigma_b, n // 3)

    def quad(xi):
        dx = sb * xi
        Md = local.tlm(geo, lt, rings[s], dx.reshape(xb.shape)).ravel()
        Hd = Binv * dx + local.adjoint(geo, lt, rings[s], (W * Md).reshape(lt.shape)).ravel()
        return g0.ravel() @ dx + 0.5 * dx @ Hd, sb * (g0.ravel() + Hd)

    res = lbfgs.minimize(quad, np.zeros(n), m=8, max_iter=1000, grad_rtol=1e-12)
    assert np.linalg.norm(sb * res["x"] - dx_star) <= 1e-8 * np.linalg.norm(dx_star)
    # the Gauss-Newton matrix predicts the change of the true gradient for a
    # small step (the residual-times-curvature term is second order here)
    dprobe = 1e-3 * sb * np.linspace(-1, 1, n)
    _, g1 = local.cost_grad(p, maps, s, xb + dprobe.reshape(xb.shape), xb, rings[s], nb)
    pred = A @ dprobe
    assert np.linalg.norm((g1 - g0).ravel() - pred) <= 1e-2 * np.linalg.norm(pred)


# --- P7 (Gauss-Newton): the local solver of Alg. 5 / Alg. 6 ------------------
def _perturbed_local(p, maps, trajs, s, seed, scale=0.3):
    r = np.random.default_rng(seed)
    return trajs[s][0] + scale * p.sigma_b[:, None, None] * r.standard_normal(trajs[s][0].shape)


@pytest.mark.parametrize("s", [0, 6])
def test_gn_normal_matrix_product(s):
    """gn.hessvec is the dense normal matrix of eq. line5and7 (TLM columns,
    weights enumerated residual by residual) applied to a vector, about a
    perturbed control; gn.residual_weights equals that enumeration."""
    p = problem("tiny2")
    g, maps, trajs, rings = _local_setup(p)
    x = _perturbed_local(p, maps, trajs, s, seed=11)
    A, lt, W = _dense_normal_matrix(p, maps, s, g, rings, x)
    np.testing.assert_allclose(gn.residual_weights(p, maps, s).ravel(), W, rtol=1e-15, atol=0)
    v = np.random.default_rng(12).standard_normal(x.shape)
    Av = gn.hessvec(p, maps, s, lt, rings[s], v)
    ref = A @ v.ravel()
    assert np.linalg.norm(Av.ravel() - ref) <= 1e-12 * np.linalg.norm(ref)


def test_gn_step_solves_normal_equations():
    """One Gauss-Newton update with conjugate gradients run to convergence is
    the closed-form solution of the normal equations, delta x* = -A^-1 grad J."""
    p = problem("tiny2")
    g, maps, trajs, rings = _local_setup(p)
    s = 6
    x0 = _perturbed_local(p, maps, trajs, s, seed=13)
    xb = trajs[s][0]
    nb = {k: trajs[k] for k in maps.neighbors[s]}
    A, _, _ = _dense_normal_matrix(p, maps, s, g, rings, x0)
    _, g0 = local.cost_grad(p, maps, s, x0, xb, rings[s], nb)
    dx_star = np.linalg.solve(A, -g0.ravel())
    res = gn.minimize(p, maps, s, x0, xb, rings[s], nb, max_iter=1, cg_max_iter=10 * x0.size,
                      cg_rtol=1e-14)
    assert res["iters"] == 1 and res["cg_iters"] <= 10 * x0.size
    assert np.linalg.norm((res["x"] - x0).ravel() - dx_star) <= 1e-8 * np.linalg.norm(dx_star)


def test_gn_quadratic_functional_one_step():
    """Without observations and overlap penalty J_s is the background term
    alone, a quadratic: one Gauss-Newton update lands on x^b from any start."""
    p = problem("c1")
    p = p.replace(obs_step=p.obs_step[:0], obs_cell=p.obs_cell[:0], obs_field=p.obs_field[:0],
                  obs_value=p.obs_value[:0], obs_sigma=p.obs_sigma[:0], obs_noise=p.obs_noise[:0],
                  mu_overlap=0.0)
    g, maps, trajs, rings = _local_setup(p)
    for s in (0, len(maps.boxes) - 1):
        xb = trajs[s][0]
        x0 = _perturbed_local(p, maps, trajs, s, seed=14)
        nb = {k: trajs[k] for k in maps.neighbors[s]}
        res = gn.minimize(p, maps, s, x0, xb, rings[s], nb, max_iter=1, cg_max_iter=200,
                          cg_rtol=1e-15)
        err = np.abs(res["x"] - xb) / p.sigma_b[:, None, None]
        assert np.max(err) <= 1e-10 and res["J"] <= 1e-18 * max(1.0, res["history"][0])


@pytest.mark.parametrize("which,s", [("tiny2", 6), ("c1", 3)])
def test_gn_converges_to_local_minimizer(which, s):
    """Gauss-Newton drives the gradient of J_s to zero (fast local
    convergence on these small-residual problems) at the minimizer that
    L-BFGS (pinned on quadratics) reaches."""
    p = problem(which)
    g, maps, trajs, rings = _local_setup(p)
    xb = trajs[s][0]
    x0 = _perturbed_local(p, maps, trajs, s, seed=15, scale=0.2)
    nb = {k: trajs[k] for k in maps.neighbors[s]}
    res = gn.minimize(p, maps, s, x0, xb, rings[s], nb, max_iter=6, cg_max_iter=400, cg_rtol=1e-12)
    assert res["gnorm"] <= 1e-8 * res["g0norm"]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(res["history"], res["history"][1:]))
    sb = p.sigma_b[:, None, None]

    def fun(xi):
        xx = xb + sb * xi.reshape(xb.shape)
        J, gr = local.cost_grad(p, maps, s, xx, xb, rings[s], nb)
        return J, (sb * gr).ravel()

    lb = lbfgs.minimize(fun, ((x0 - xb) / sb).ravel(), max_iter=2000, grad_rtol=1e-10)
    x_lb = xb + sb * lb["x"].reshape(xb.shape)
    assert np.linalg.norm((res["x"] - x_lb) / sb) <= 1e-6 * np.linalg.norm((res["x"] - xb) / sb)


def test_dd_solve_gauss_newton():
    """Alg. 1 with the Gauss-Newton local solver: the analysis improves on
    the background, and with converged local solves it is the fixed point
    that the L-BFGS local solver reaches."""
    p = problem("tiny2")
    xa, rep = dd.solve(p, max_outer=3, max_iter=5, local_solver="gn", cg_max_iter=300,
                       cg_rtol=1e-12, outer_tol=0.0)
    assert rep["outer"] == 3 and rep["cg_iters"] > 0
    e_b = np.linalg.norm((p.xb0 - p.truth0) / p.sigma_b[:, None, None])
    e_a = np.linalg.norm((xa - p.truth0) / p.sigma_b[:, None, None])
    assert e_a < e_b
    xl, _ = dd.solve(p, max_outer=3, max_iter=400, grad_rtol=1e-11, outer_tol=0.0)
    sb = p.sigma_b[:, None, None]
    assert np.linalg.norm((xa - xl) / sb) <= 1e-6 * np.linalg.norm((xl - p.xb0) / sb)


# --- Lanczos on the B-preconditioned normal equations (Alg. 7) -------------
def _spd(rng, n, cond):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.geomspace(1.0, cond, n)
    return (Q * lam) @ Q.T, lam


def test_lanczos_matches_cg_and_exact_solve(rng):
    """In exact arithmetic the Lanczos iterate x_j = V_j y_j is the j-th CG
    iterate: the same vectors after every number of products (1e-9), the
    solution of the system at a tight tolerance, and the same stop by
    residual."""
    A, lam = _spd(rng, 40, 1e3)
    b = rng.standard_normal(40)
    for k in range(1, 13):
        xl, jl, _, _ = gn.lanczos(lambda v: A @ v, b, k, 0.0)
        xc, jc = gn.cg(lambda v: A @ v, b, k, 0.0)
        assert jl == jc == k
        assert np.linalg.norm(xl - xc) <= 1e-9 * np.linalg.norm(xc), k
    # run to a tight tolerance: the solution (finite precision costs a few
    # more products than n once the basis loses orthogonality, as for CG)
    x, j, _, _ = gn.lanczos(lambda v: A @ v, b, 400, 1e-12)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    # the residual estimate beta_{j+1} |e_j^T y_j| is the true residual: the
    # same stop as CG while the basis stays orthogonal, and the tolerance met
    for rtol in (3e-1, 1e-1):
        xl, jl, _, _ = gn.lanczos(lambda v: A @ v, b, 100, rtol)
        xc, jc = gn.cg(lambda v: A @ v, b, 100, rtol)
        assert jl == jc
    for rtol in (1e-2, 1e-5):
        xl, jl, _, _ = gn.lanczos(lambda v: A @ v, b, 200, rtol)
        assert np.linalg.norm(b - A @ xl) <= 1.01 * rtol * np.linalg.norm(b)


def test_lanczos_ritz_values(rng):
    """The eigenvalues of T_j interlace the spectrum and the extreme ones
    converge to the extreme eigenvalues (well separated here)."""
    A, lam = _spd(rng, 60, 1e2)
    b = rng.standard_normal(60)
    _, j, al, be = gn.lanczos(lambda v: A @ v, b, 30, 0.0)
    r = gn.ritz_values(al, be)
    assert j == 30 and r.size == 30
    assert lam[0] * (1 - 1e-12) <= r.min() and r.max() <= lam[-1] * (1 + 1e-12)
    assert abs(r.max() - lam[-1]) <= 1e-8 * lam[-1]


def test_gn_lanczos_local_problem():
    """Gauss-Newton with Lanczos on a local normal equation system (Alg. 6,
    Alg. 7): the same updates as with CG, and Ritz values inside the spectrum
    of the dense preconditioned normal matrix V A V, the largest converged
    to its largest eigenvalue."""
    p = problem("tiny2")
    g, maps, trajs, rings = _local_setup(p)
    s = 6
    x0 = _perturbed_local(p, maps, trajs, s, seed=16)
    xb = trajs[s][0]
    nb = {k: trajs[k] for k in maps.neighbors[s]}
    kw = dict(max_iter=3, cg_max_iter=40, cg_rtol=1e-6)
    rc = gn.minimize(p, maps, s, x0, xb, rings[s], nb, **kw)
    rl = gn.minimize(p, maps, s, x0, xb, rings[s], nb, krylov="lanczos", **kw)
    sb = p.sigma_b[:, None, None]
    assert rl["cg_iters"] == rc["cg_iters"]
    assert np.linalg.norm((rl["x"] - rc["x"]) / sb) <= 1e-8 * np.linalg.norm((rc["x"] - x0) / sb)
    # spectrum of V A V about x0, from one update with a long Lanczos run
    res1 = gn.minimize(p, maps, s, x0, xb, rings[s], nb, krylov="lanczos", max_iter=1,
                       cg_max_iter=80, cg_rtol=0.0)
    A, _, _ = _dense_normal_matrix(p, maps, s, g, rings, x0)
    v = (sb * np.ones_like(x0)).ravel()
    ev = np.linalg.eigvalsh(v[:, None] * A * v[None, :])
    r = res1["ritz"]
    assert r.size > 0 and ev[0] * (1 - 1e-9) <= r.min() and r.max() <= ev[-1] * (1 + 1e-9)
    assert abs(r.max() - ev[-1]) <= 1e-6 * ev[-1]


# --- Turkel-Zwas variant (Sec. 7 discrete U, V, H with p, q, alpha) ---------
TZ_VARIANTS = [(1, 1, 0.0), (2, 2, 0.5), (2, 1, 0.0), (1, 2, 1.0), (3, 2, 0.25)]


def _tz_grid(p, tzv):
    return model.Grid(p.nlat, p.nlon, p.dt, p.radius, p.gravity, p.omega, tz=tzv)


@pytest.mark.parametrize("tzv", TZ_VARIANTS)
def test_tz_rest_state_and_identities(rng, tzv):
    """Rest state fixed; tangent linear equal to centred differences of the
    (quadratic) increment; adjoint the transpose of the tangent linear, one
    step and over a trajectory (adjoint definition, eq. adjProd)."""
    p = problem("c1")
    g = _tz_grid(p, tzv)
    R = np.stack([np.full((p.nlat, p.nlon), p.h_ref), np.zeros((p.nlat, p.nlon)),
                  np.zeros((p.nlat, p.nlon))])
    assert np.all(model.increment(g, R) == 0.0)
    Z = p.truth0
    dZ = rng.standard_normal(Z.shape) * p.sigma_b[:, None, None]
    lam = rng.standard_normal(Z.shape)
    tl = model.increment_tl(g, Z, dZ)
    fd = (model.increment(g, Z + 1e-3 * dZ) - model.increment(g, Z - 1e-3 * dZ)) / 2e-3
    assert np.linalg.norm(fd - tl) <= 1e-9 * np.linalg.norm(tl)
    lhs, rhs = np.sum(tl * lam), np.sum(dZ * model.increment_ad(g, Z, lam))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    traj = model.forward(g, Z, 6)
    y = rng.standard_normal(traj.shape)
    lhs = np.sum(model.tlm(g, traj, dZ) * y)
    rhs = np.sum(dZ * model.adjoint(g, traj, y))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_tz_plain_offsets_against_the_plain_scheme():
    """With p = q = 1 and alpha = 0 the U and V of the Turkel-Zwas scheme are
    the plain scheme's exactly, and its advective H differs from the flux
    form by the product-rule remainder
    (s_lon/c)[(hE-h)(uE-u) - (hW-h)(uW-u)] + (s_lat/c)[(hN-h)(vN cN - v c) - (hS-h)(vS cS - v c)]."""
    p = problem("c1")
    g0 = model.Grid.of(p)
    g1 = _tz_grid(p, (1, 1, 0.0))
    Z = p.truth0
    F0, F1 = model.increment(g0, Z), model.increment(g1, Z)
    np.testing.assert_allclose(F1[1:], F0[1:], rtol=1e-13, atol=1e-13 * np.abs(F0[1:]).max())
    h, u, v = Z
    c = g0.cos[:, None]
    cN = np.append(g0.cos[1:], g0.cos[-1])[:, None]
    cS = np.insert(g0.cos[:-1], 0, g0.cos[0])[:, None]
    E, W = (lambda x: np.roll(x, -1, -1)), (lambda x: np.roll(x, 1, -1))
    hN, hS = model._north(h, 1.0), model._south(h, 1.0)
    vN, vS = model._north(v, -1.0), model._south(v, -1.0)
    rem = (g0.sig_lon / c) * ((E(h) - h) * (E(u) - u) - (W(h) - h) * (W(u) - u)) + \
        (g0.sig_lat / c) * ((hN - h) * (vN * cN - v * c) - (hS - h) * (vS * cS - v * c))
    np.testing.assert_allclose(F1[0] - F0[0], rem, rtol=1e-9, atol=1e-9 * np.abs(rem).max())


@pytest.mark.parametrize("tzv", TZ_VARIANTS[1:])
@pytest.mark.parametrize("omega,alpha", [(7.292e-5, 0.0), (0.0, math.pi / 4), (0.0, 0.3)])
def test_tz_steady_flow_second_order(tzv, omega, alpha):
    """The Turkel-Zwas increments of the solid-body rotations above vanish at
    second order in the grid spacing too (consistency of the wide offsets,
    the averaged Coriolis terms and the corner divergence)."""
    res = []
    for nlat in (32, 64, 128):
        g, Z = _tc2(nlat, omega, alpha)
        g.tz = tzv
        F = model.increment(g, Z)
        h = Z[0]
        band = np.abs(g.theta) < math.pi / 3
        scale = np.linalg.norm((g.sig_lat * g.gravity * (np.roll(h, -1, 0) - np.roll(h, 1, 0)))[band])
        res.append(max(np.linalg.norm(F[k][band]) for k in range(3)) / scale)
    assert 3.4 < res[0] / res[1] < 5.5 and 3.4 < res[1] / res[2] < 4.6, res


def _max_wind_run(g, x0, steps, cap=1e3):
    """Leapfrog run (Euler half start) of the global model; the step at which
    the winds pass ``cap`` m/s (or ``steps``) and the largest wind seen."""
    prev, cur = x0, x0 + 0.5 * model.increment(g, x0)
    peak = float(np.abs(x0[1:]).max())
    with np.errstate(all="ignore"):
        for n in range(1, steps):
            prev, cur = cur, prev + model.increment(g, cur)
            a = float(np.abs(cur[1:]).max())
            if not a <= cap:
                return n, a
            peak = max(peak, a)
    return steps, peak


def test_tz_larger_time_step():
    """The point of the coarse offsets: the gravity-wave terms over p columns
    and q rows relax the (polar) CFL limit.  At 2.5x the time step of the
    synthetic problems the plain centred scheme blows up within 20 steps,
    while the Turkel-Zwas scheme with p = q = 2 stays bounded over 400 steps,
    and with alpha = 1/2 still at 4x."""
    p = problem("c1")
    w0 = float(np.abs(p.xb0[1:]).max())
    g = model.Grid(p.nlat, p.nlon, 2.5 * p.dt, p.radius, p.gravity, p.omega)
    n, _ = _max_wind_run(g, p.xb0, 400)
    assert n < 20
    for k, tzv in ((2.5, (2, 2, 0.0)), (2.5, (2, 2, 0.5)), (4.0, (2, 2, 0.5))):
        g = _tz_grid(p.replace(dt=k * p.dt), tzv)
        n, peak = _max_wind_run(g, p.xb0, 400)
        assert n == 400 and peak < 2.0 * w0, (k, tzv, n, peak)


TZ_SPACE_CFGS = {
    "c1": dict(synth.CONFIGS["c1"], index=140),
    "span": dict(SPAN_CFG, index=141),
    "mixed": dict(MIXED_CFG, index=142),
    # five spanning bands: pads reaching across a pole partly into the box
    # itself (internal) and partly into the polar band (frozen)
    "deep": dict(index=145, nlat=16, nlon=32, nsteps=6, bands=5, pieces=1, ntime=2,
                 overlap_cells=2, overlap_steps=1, obs_frac=0.1, obs_every=2),
}


@pytest.mark.parametrize("which", ["c1", "span", "mixed", "deep"])
@pytest.mark.parametrize("tzv", [(2, 2, 0.5), (1, 3, 1.0)])
def test_tz_restricted_model_with_exact_pad(rng, which, tzv):
    """Spatial decompositions under the variant: with the pad of every level
    taken from the global trajectory (one interval), the restricted model on
    each box (pieces, spanning bands, bands touching a pole, pads reaching
    across it, brick widths) reproduces the global trajectory on the box, and
    the weighted local functionals sum to the global one (eq. restJ)."""
    p = custom_problem(dict(TZ_SPACE_CFGS[which], ntime=1, tz=tzv))
    g = _grid(p)
    maps = ddmaps.build(p)
    x = p.xb0 + p.sigma_b[:, None, None] * rng.standard_normal(p.xb0.shape)
    gt = model.forward(g, x, p.nsteps)
    trajs = {b.sub: local.restrict_global(maps, b.sub, gt) for b in maps.boxes}
    xb0 = p.xb0[None]
    total = 0.0
    for b in maps.boxes:
        assert b.nring == len(maps.halo_src[b.sub])
        ring = local.ring_from_trajs(maps, b.sub, trajs)
        lt = local.forward(local.LocalGeometry(g, maps, b.sub), trajs[b.sub][0], ring)
        assert np.abs(lt - trajs[b.sub]).max() <= 1e-12 * np.abs(trajs[b.sub]).max(), b.sub
        xbs = local.restrict_global(maps, b.sub, xb0)[0]
        J = local.cost_grad(p, maps, b.sub, trajs[b.sub][0], xbs, ring,
                            {k: trajs[k] for k in maps.neighbors[b.sub]}, with_grad=False)
        total += J
    Jg = model.cost_grad(p, x, with_grad=False)
    assert abs(total - Jg) <= 1e-12 * Jg


@pytest.mark.parametrize("which", ["c1", "span", "mixed", "deep"])
def test_tz_local_dot_product_and_gradient(rng, which):
    """Local tangent linear and adjoint with frozen pads (adjoint definition,
    eq. adjProd), per step and over the window, on every box; the local
    gradient against centred differences of the local functional."""
    p = custom_problem(dict(TZ_SPACE_CFGS[which], tz=(2, 2, 0.5)))
    g, maps, trajs, rings = _local_setup(p)
    sb = p.sigma_b[:, None, None]
    for s in range(len(maps.boxes)):
        geo = local.LocalGeometry(g, maps, s)
        x = trajs[s][0] + 0.3 * sb * rng.standard_normal(trajs[s][0].shape)
        lt = local.forward(geo, x, rings[s])
        dx = rng.standard_normal(x.shape)
        y = rng.standard_normal(lt.shape)
        lhs = np.sum(local.tlm(geo, lt, rings[s], dx) * y)
        rhs = np.sum(dx * local.adjoint(geo, lt, rings[s], y))
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs), s
        P, dP = geo.tz.pad(x, rings[s][0]), geo.tz.pad(dx, None)
        lam = rng.standard_normal(x.shape)
        lhs = np.sum(tz_local.increment_tl(geo.tz, P, dP) * lam)
        rhs = np.sum(dx * geo.tz.fold(tz_local.increment_ad(geo.tz, P, lam)))
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs), s
    s = len(maps.boxes) - 1
    xb = trajs[s][0]
    x = xb + 0.5 * sb * rng.standard_normal(xb.shape)
    nb = {k: trajs[k] for k in maps.neighbors[s]}
    J, gr = local.cost_grad(p, maps, s, x, xb, rings[s], nb)
    d = sb * rng.standard_normal(xb.shape)
    an = np.sum(gr * d)
    eps = 5e-4
    Jp = local.cost_grad(p, maps, s, x + eps * d, xb, rings[s], nb, with_grad=False)
    Jm = local.cost_grad(p, maps, s, x - eps * d, xb, rings[s], nb, with_grad=False)
    assert abs((Jp - Jm) / (2 * eps) - an) <= 1e-6 * abs(an)


def test_tz_time_decomposition_box_is_the_global_model():
    """A box covering the sphere: the padded-frame increment equals the
    global model's (array shifts and pole reflection) bit for bit."""
    p = custom_problem(dict(synth.CONFIGS["c1"], bands=1, pieces=1, ntime=2, overlap_cells=0,
                            index=143, tz=(3, 2, 0.25)))
    g = _grid(p)
    maps = ddmaps.build(p)
    geo = local.LocalGeometry(g, maps, 0)
    assert geo.tz.frozen.size == 0
    x = p.truth0
    assert np.array_equal(tz_local.increment(geo.tz, geo.tz.pad(x, None)), model.increment(g, x))


def test_tz_pad_columns_must_not_wrap():
    cfg = dict(synth.CONFIGS["c1"], index=144, tz=(15, 1, 0.0))
    with pytest.raises(ValueError):
        ddmaps.build(custom_problem(cfg))


# --- P10: map invariants -----------------------------------------------------
@pytest.mark.parametrize("which", ["c1", "c2", "small", "span", "mixed", "c3"])
def test_map_invariants(which):
    if which == "span":
        p = synth.make_spec(SPAN_CFG)
    elif which == "mixed":
        p = synth.make_spec(MIXED_CFG)
    else:
        p = synth.make_spec(which)
    maps = ddmaps.build(p)
    nl, nn = p.nlat, p.nlon
    # every cell is in exactly one core
    cnt = np.zeros((nl, nn), int)
    for b in maps.boxes[:maps.nspace]:
        cnt[b.core_row0:b.core_row1, b.core_col0:b.core_col1] += 1
    assert (cnt == 1).all()
    # box sizes: core + 2 o per side, clipped at the poles (eqs. Eq-r, nlocx)
    o = p.overlap_cells
    for b in maps.boxes:
        exp_ny = min(nl, b.core_row1 + o) - max(0, b.core_row0 - o)
        assert b.ny == exp_ny
        assert b.nx == (nn if b.span else b.core_col1 - b.core_col0 + 2 * o)
    # ring sources: the (pole-mapped) neighbour cell, inside the source core
    half = nn // 2
    for b in maps.boxes:
        ny, nx = b.ny, b.nx
        for k in range(b.nring):
            if k < nx:
                r, c = -1, k
            elif k < 2 * nx:
                r, c = ny, k - nx
            elif k < 2 * nx + ny:
                r, c = k - 2 * nx, -1
            else:
                r, c = k - 2 * nx - ny, nx
            grow, gcol = b.row0 + r, (b.col0 + c) % nn
            sign = 1
            if grow < 0:
                grow, gcol, sign = 0, (gcol + half) % nn, -1
            elif grow >= nl:
                grow, gcol, sign = nl - 1, (gcol + half) % nn, -1
            src = int(maps.halo_src[b.sub][k])
            off = int(maps.halo_off[b.sub][k])
            assert int(maps.halo_sign[b.sub][k]) == sign
            if src < 0:
                assert b.span
                assert off // nx == grow - b.row0 and off % nx == gcol
            else:
                sb = maps.boxes[src]
                assert sb.interval == b.interval
                assert sb.core_row0 <= grow < sb.core_row1 and sb.core_col0 <= gcol < sb.core_col1
                assert off // sb.nx == grow - sb.row0
                assert (sb.col0 + off % sb.nx) % nn == gcol
    # overlap neighbour sets are symmetric and exactly the intersecting boxes
    for b in maps.boxes:
        for sp in maps.neighbors[b.sub]:
            assert b.sub in set(maps.neighbors[int(sp)].tolist())
    # partition of unity: counts equal the number of boxes containing each point
    cover = np.zeros((nl, nn), int)
    for b in maps.boxes[:maps.nspace]:
        rows = np.arange(b.row0, b.row0 + b.ny)
        cols = (b.col0 + np.arange(b.nx)) % nn
        cover[np.ix_(rows, cols)] += 1
    assert (cover == maps.cover_sp).all()
    # observation bins: each observation lands in every box containing it
    for o in range(0, p.nobs, max(1, p.nobs // 200)):
        cell = int(p.obs_cell[o])
        k = int(p.obs_step[o])
        hits = [b.sub for b in maps.boxes if b.lev0 <= k < b.lev0 + b.nlev and
                maps.box_index(b, cell // nn, cell % nn) >= 0]
        got = [s for s in range(len(maps.boxes)) if o in set(maps.obs_bin[s].tolist())]
        assert hits == got
        assert len(hits) == maps.cover_sp[cell // nn, cell % nn] * maps.time_count[k]


DENSE_PIN_CFG = dict(index=113, nlat=24, nlon=48, nsteps=24, bands=4, pieces=4, ntime=3,
                     overlap_cells=5, overlap_steps=3, obs_frac=0.1, obs_every=2)


@pytest.mark.parametrize("which", ["c1", "small", "span", "mixed", "dense"])
def test_neighbour_sets_by_brute_force(which):
    """Overlap neighbour sets (eqs. overl, ospatial, otime; reading R7: every
    other box whose extended space-time box intersects): each box's set of
    (global level, global cell) points is enumerated as an occupancy array
    over the whole window, and two boxes are neighbours exactly when their
    arrays share a point."""
    cfg = {"span": SPAN_CFG, "mixed": MIXED_CFG, "dense": DENSE_PIN_CFG}.get(which, which)
    p = synth.make_spec(cfg)
    maps = ddmaps.build(p)
    nb = len(maps.boxes)
    occ = np.zeros((nb, p.nsteps + 1, p.nlat, p.nlon), dtype=bool)
    for b in maps.boxes:
        for r in range(b.row0, b.row0 + b.ny):
            for c in range(b.col0, b.col0 + b.nx):
                occ[b.sub, b.lev0:b.lev0 + b.nlev, r, c % p.nlon] = True
    flat = occ.reshape(nb, -1).astype(np.int64)
    shared = flat @ flat.T                     # points each pair of boxes shares
    for b in maps.boxes:
        want = sorted(int(k) for k in np.nonzero(shared[b.sub])[0] if k != b.sub)
        assert sorted(int(k) for k in maps.neighbors[b.sub]) == want, b.sub
    if which == "dense":                       # diagonal and far neighbours occur
        assert max(len(maps.neighbors[b.sub]) for b in maps.boxes) > 20


def test_box_sizes_at_benchmark_configs():
    """Extended sizes from the problem-size arithmetic (eqs. Eq-r, nlocx)."""
    p = synth.make_spec("c5")
    maps = ddmaps.build(p)
    assert len(maps.boxes) == 2048
    sizes = {(b.ny, b.nx) for b in maps.boxes}
    assert sizes == {(68, 136), (72, 136)}
    assert sorted({b.nlev for b in maps.boxes}) == [30, 34]
    local_pt_steps = sum(b.ny * b.nx * (b.nlev - 1) for b in maps.boxes)
    # 32 polar + 224 interior boxes per interval; 2 intervals of 29 steps, 6 of 33
    assert local_pt_steps == (32 * 68 + 224 * 72) * 136 * (2 * 29 + 6 * 33) == 637272064
    assert p.nobs == 999999


# --- L-BFGS on a known quadratic and the DD outer loop ------------------------
def test_lbfgs_quadratic(rng):
    n = 40
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    bvec = rng.standard_normal(n)
    res = lbfgs.minimize(lambda x: (0.5 * x @ A @ x - bvec @ x, A @ x - bvec), np.zeros(n),
                         max_iter=300, grad_rtol=1e-9)
    assert res["status"] == "converged"
    xs = np.linalg.solve(A, bvec)
    assert np.linalg.norm(res["x"] - xs) <= 1e-8 * np.linalg.norm(xs)


def test_dd_solve_one_box_is_global_4dvar():
    """Alg. 1 with P = Q = 1 and no overlap: one local solve whose functional
    is global 4D-Var (eq. min3sec).  Its analysis is a stationary point of the
    independently written global functional (gradient reduced to 1e-7 of its
    value at the background), and it coincides with L-BFGS run directly on
    the global functional in the same variables to the accuracy both stop
    tests leave (1e-6 of the increment)."""
    p = custom_problem(dict(synth.CONFIGS["c1"], bands=1, pieces=1, ntime=1, overlap_cells=0,
                            overlap_steps=0, index=119))
    maps = ddmaps.build(p)
    assert len(maps.boxes) == 1 and maps.boxes[0].span
    opts = dict(max_iter=400, grad_rtol=1e-9)
    xa, rep = dd.solve(p, maps, max_outer=1, outer_tol=0.0, **opts)
    sb = p.sigma_b[:, None, None]
    _, g0 = model.cost_grad(p, p.xb0)
    _, ga = model.cost_grad(p, xa)
    assert np.linalg.norm(sb * ga) <= 1e-7 * np.linalg.norm(sb * g0)

    def fun(xi):
        J, gr = model.cost_grad(p, p.xb0 + sb * xi.reshape(p.xb0.shape))
        return J, (sb * gr).ravel()

    res = lbfgs.minimize(fun, np.zeros(p.xb0.size), **opts)
    xg = p.xb0 + sb * res["x"].reshape(p.xb0.shape)
    inc = np.linalg.norm((xg - p.xb0) / sb)
    assert inc > 0 and np.linalg.norm((xa - xg) / sb) <= 1e-6 * inc


def test_dd_solve_improves_on_background():
    """Alg. 1 on the smallest configuration: the analysis is closer to the truth
    than the background, and the gather reproduces the controls' partition of
    unity."""
    p = problem("tiny2")
    xa, rep = dd.solve(p, max_outer=2, max_iter=30)
    assert rep["outer"] >= 1
    e_b = np.linalg.norm((p.xb0 - p.truth0) / p.sigma_b[:, None, None])
    e_a = np.linalg.norm((xa - p.truth0) / p.sigma_b[:, None, None])
    assert e_a < e_b
    maps = ddmaps.build(p)
    # gather of the background trajectory returns the background
    bg, trajs = dd.background(p, maps)
    np.testing.assert_allclose(dd.gather(p, maps, trajs, 0), p.xb0, rtol=1e-15, atol=0)
