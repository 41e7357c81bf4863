"""Global shallow-water model on the sphere, its TLM and adjoint (FP64).

Test infrastructure only (see the package docstring).

Continuous model: eqs. EquU, EquV, EquH (Sec. 7).  Space discretization: the
unstaggered scheme of Sec. 7 with p = q = 1 and alpha = 0, i.e. plain centred
differences.  Readings used here:

* cell-centred latitudes theta_j = -pi/2 + (j + 1/2) dtheta, j south to north,
  longitudes lambda_i = i dlambda, dtheta = pi/nlat, dlambda = 2 pi/nlon;
* sigma_lon = dt / (a dlambda), sigma_lat = dt / (a dtheta); the discrete
  U, V, H are then increments over 2 dt, so time stepping is leapfrog,
  Z^{n+1} = Z^{n-1} + F(Z^n), with a forward-Euler half increment to start,
  Z^1 = Z^0 + F(Z^0)/2;
* the Coriolis bracket carries the factor 2 dt;
* the discrete V uses v differences for the meridional advection of v and a
  minus sign on (f + u tan(theta)/a) u (the physical sign);
* the height equation is the flux form of EquH with the meridional flux
  h v cos(theta):  H = -(s_lon/c)[(hu)_E - (hu)_W] - (s_lat/c)[(hvc)_N - (hvc)_S];
* a row beyond a pole is the same latitude row shifted by half a circle,
  with u and v negated and the mapped row's cos(theta).

Field order (h, u, v); arrays [3][nlat][nlon].
"""
from __future__ import annotations

import numpy as np

from . import tz


class Grid:
    """Per-row tables and Courant factors of the lat-lon grid."""

    def __init__(self, nlat, nlon, dt, radius, gravity, omega, dtype=np.float64, tz=None):
        """``dtype`` is the arithmetic type of the tables and constants:
        float64 normally; np.longdouble gives an extended-precision reference
        of the same computation (its inputs are still the FP64 values).
        ``tz`` = (p, q, alpha) selects the Turkel-Zwas variant (``tz``
        module); None the plain scheme."""
        if nlon % 2:
            raise ValueError("nlon must be even for the across-pole map")
        D = dtype
        self.dtype = D
        self.nlat, self.nlon = int(nlat), int(nlon)
        self.dt, self.radius, self.gravity, self.omega = D(dt), D(radius), D(gravity), D(omega)
        pi = D(np.pi) if D is np.float64 else D("3.14159265358979323846264338327950288")
        self.dlat = pi / nlat
        self.dlon = D(2) * pi / nlon
        self.theta = -pi / 2 + (np.arange(nlat, dtype=D) + D(0.5)) * self.dlat
        self.cos = np.cos(self.theta)
        self.tan = np.tan(self.theta)
        self.fcor = D(2) * self.omega * np.sin(self.theta)
        self.sig_lon = self.dt / (self.radius * self.dlon)
        self.sig_lat = self.dt / (self.radius * self.dlat)
        self.tz = None if tz is None else (int(tz[0]), int(tz[1]), D(tz[2]))

    @classmethod
    def of(cls, prob, dtype=np.float64):
        p = int(getattr(prob, "tz_p", 0))
        tz = (p, int(prob.tz_q), float(prob.tz_alpha)) if p > 0 else None
        return cls(prob.nlat, prob.nlon, prob.dt, prob.radius, prob.gravity, prob.omega, dtype, tz)


# --- neighbour operators on the global grid ---------------------------------
def _east(x):
    return np.roll(x, -1, axis=-1)


def _west(x):
    return np.roll(x, 1, axis=-1)


def _north(x, sign):
    out = np.empty_like(x)
    out[:-1] = x[1:]
    out[-1] = sign * np.roll(x[-1], -(x.shape[-1] // 2))
    return out


def _south(x, sign):
    out = np.empty_like(x)
    out[1:] = x[:-1]
    out[0] = sign * np.roll(x[0], -(x.shape[-1] // 2))
    return out


# transposes of the neighbour operators (for the adjoint)
def _east_T(y):
    return np.roll(y, 1, axis=-1)


def _west_T(y):
    return np.roll(y, -1, axis=-1)


def _north_T(y, sign):
    x = np.zeros_like(y)
    x[1:] += y[:-1]
    x[-1] += sign * np.roll(y[-1], y.shape[-1] // 2)
    return x


def _south_T(y, sign):
    x = np.zeros_like(y)
    x[:-1] += y[1:]
    x[0] += sign * np.roll(y[0], y.shape[-1] // 2)
    return x


def _row(g, a):
    return a[:, None]


def increment(g: Grid, Z):
    """F(Z): the 2 dt increment (U, V, H) of the discrete SWE; returns (H, U, V)."""
    if g.tz is not None:
        return tz.increment(g, Z, *g.tz)
    h, u, v = Z
    c = g.cos[:, None]
    t = g.tan[:, None]
    f = g.fcor[:, None]
    cN = np.append(g.cos[1:], g.cos[-1])[:, None]
    cS = np.insert(g.cos[:-1], 0, g.cos[0])[:, None]
    sl, st, gr, a, dt = g.sig_lon, g.sig_lat, g.gravity, g.radius, g.dt
    uE, uW, vE, vW, hE, hW = _east(u), _west(u), _east(v), _west(v), _east(h), _west(h)
    uN, uS, vN, vS = _north(u, -1.0), _south(u, -1.0), _north(v, -1.0), _south(v, -1.0)
    hN, hS = _north(h, 1.0), _south(h, 1.0)
    cor = f + u * t / a
    U = (-sl * (u / c) * (uE - uW) - st * v * (uN - uS)
         - sl * (gr / c) * (hE - hW) + 2.0 * dt * cor * v)
    V = (-sl * (u / c) * (vE - vW) - st * v * (vN - vS)
         - st * gr * (hN - hS) - 2.0 * dt * cor * u)
    H = (-(sl / c) * (hE * uE - hW * uW)
         - (st / c) * (hN * vN * cN - hS * vS * cS))
    return np.stack([H, U, V])


def increment_tl(g: Grid, Z, dZ):
    """Tangent linear of ``increment`` at Z applied to dZ."""
    if g.tz is not None:
        return tz.increment_tl(g, Z, dZ, *g.tz)
    h, u, v = Z
    dh, du, dv = dZ
    c = g.cos[:, None]
    t = g.tan[:, None]
    f = g.fcor[:, None]
    cN = np.append(g.cos[1:], g.cos[-1])[:, None]
    cS = np.insert(g.cos[:-1], 0, g.cos[0])[:, None]
    sl, st, gr, a, dt = g.sig_lon, g.sig_lat, g.gravity, g.radius, g.dt
    uE, uW, vE, vW, hE, hW = _east(u), _west(u), _east(v), _west(v), _east(h), _west(h)
    uN, uS, vN, vS = _north(u, -1.0), _south(u, -1.0), _north(v, -1.0), _south(v, -1.0)
    hN, hS = _north(h, 1.0), _south(h, 1.0)
    duE, duW, dvE, dvW, dhE, dhW = _east(du), _west(du), _east(dv), _west(dv), _east(dh), _west(dh)
    duN, duS, dvN, dvS = _north(du, -1.0), _south(du, -1.0), _north(dv, -1.0), _south(dv, -1.0)
    dhN, dhS = _north(dh, 1.0), _south(dh, 1.0)
    cor = f + u * t / a
    dcor = du * t / a
    dU = (-sl / c * (du * (uE - uW) + u * (duE - duW))
          - st * (dv * (uN - uS) + v * (duN - duS))
          - sl * (gr / c) * (dhE - dhW)
          + 2.0 * dt * (dcor * v + cor * dv))
    dV = (-sl / c * (du * (vE - vW) + u * (dvE - dvW))
          - st * (dv * (vN - vS) + v * (dvN - dvS))
          - st * gr * (dhN - dhS)
          - 2.0 * dt * (dcor * u + cor * du))
    dH = (-(sl / c) * (dhE * uE + hE * duE - dhW * uW - hW * duW)
          - (st / c) * ((dhN * vN + hN * dvN) * cN - (dhS * vS + hS * dvS) * cS))
    return np.stack([dH, dU, dV])


def increment_ad(g: Grid, Z, lam):
    """Adjoint of ``increment_tl`` at Z: returns the transpose applied to lam.

    lam = (lamH, lamU, lamV) are the weights on the (H, U, V) outputs.  Each
    term of the tangent linear code is transposed in turn (scatter form).
    """
    if g.tz is not None:
        return tz.increment_ad(g, Z, lam, *g.tz)
    h, u, v = Z
    lH, lU, lV = lam
    c = g.cos[:, None]
    t = g.tan[:, None]
    f = g.fcor[:, None]
    cN = np.append(g.cos[1:], g.cos[-1])[:, None]
    cS = np.insert(g.cos[:-1], 0, g.cos[0])[:, None]
    sl, st, gr, a, dt = g.sig_lon, g.sig_lat, g.gravity, g.radius, g.dt
    uE, uW, vE, vW, hE, hW = _east(u), _west(u), _east(v), _west(v), _east(h), _west(h)
    uN, uS, vN, vS = _north(u, -1.0), _south(u, -1.0), _north(v, -1.0), _south(v, -1.0)
    hN, hS = _north(h, 1.0), _south(h, 1.0)
    cor = f + u * t / a
    ah = np.zeros_like(h)
    au = np.zeros_like(u)
    av = np.zeros_like(v)
    # dU terms
    w = lU * (-sl / c)
    au += w * (uE - uW)
    au += _east_T(w * u) - _west_T(w * u)
    w = lU * (-st)
    av += w * (uN - uS)
    au += _north_T(w * v, -1.0) - _south_T(w * v, -1.0)
    w = lU * (-sl * gr / c)
    ah += _east_T(w) - _west_T(w)
    w = lU * 2.0 * dt
    au += w * v * t / a
    av += w * cor
    # dV terms
    w = lV * (-sl / c)
    au += w * (vE - vW)
    av += _east_T(w * u) - _west_T(w * u)
    w = lV * (-st)
    av += w * (vN - vS)
    av += _north_T(w * v, -1.0) - _south_T(w * v, -1.0)
    w = lV * (-st * gr)
    ah += _north_T(w, 1.0) - _south_T(w, 1.0)
    w = lV * (-2.0 * dt)
    au += w * u * t / a
    au += w * cor
    # dH terms
    w = lH * (-sl / c)
    ah += _east_T(w * uE) - _west_T(w * uW)
    au += _east_T(w * hE) - _west_T(w * hW)
    w = lH * (-st / c)
    ah += _north_T(w * vN * cN, 1.0) - _south_T(w * vS * cS, 1.0)
    av += _north_T(w * hN * cN, -1.0) - _south_T(w * hS * cS, -1.0)
    return np.stack([ah, au, av])


# --- time stepping ------------------------------------------------------------
def forward(g: Grid, x0, nsteps):
    """Leapfrog trajectory from x0; returns [nsteps+1][3][nlat][nlon]."""
    traj = np.empty((nsteps + 1,) + x0.shape, dtype=x0.dtype)
    traj[0] = x0
    if nsteps >= 1:
        traj[1] = x0 + 0.5 * increment(g, x0)
    for n in range(1, nsteps):
        traj[n + 1] = traj[n - 1] + increment(g, traj[n])
    return traj


def forward_at(g: Grid, x0, steps):
    """Model states at the requested steps (streams, keeps two levels)."""
    steps = sorted(steps)
    want = set(steps)
    out = {}
    last = steps[-1] if steps else 0
    prev, cur = None, x0.copy()
    if 0 in want:
        out[0] = cur.copy()
    for n in range(0, last):
        if n == 0:
            nxt = cur + 0.5 * increment(g, cur)
        else:
            nxt = prev + increment(g, cur)
        prev, cur = cur, nxt
        if n + 1 in want:
            out[n + 1] = cur.copy()
    return np.stack([out[k] for k in steps])


def tlm(g: Grid, traj, dx0):
    """Tangent linear trajectory about ``traj`` from dx0 (all levels)."""
    L = traj.shape[0] - 1
    d = np.empty_like(traj)
    d[0] = dx0
    if L >= 1:
        d[1] = dx0 + 0.5 * increment_tl(g, traj[0], dx0)
    for n in range(1, L):
        d[n + 1] = d[n - 1] + increment_tl(g, traj[n], d[n])
    return d


def adjoint(g: Grid, traj, forcing):
    """Transpose of ``tlm``: sum_n M'_n^T forcing[n], returned at level 0.

    The tangent linear recursion is transposed step by step in reverse order
    (the adjoint-of-a-product rule, eq. adjProd).
    """
    L = traj.shape[0] - 1
    a = forcing.copy()
    for n in range(L - 1, 0, -1):
        # transpose of d[n+1] = d[n-1] + F'(Z^n) d[n]
        a[n - 1] += a[n + 1]
        a[n] += increment_ad(g, traj[n], a[n + 1])
    if L >= 1:
        a[0] += a[1] + 0.5 * increment_ad(g, traj[0], a[1])
    return a[0]


# --- global 4D-Var functional (Def. "4D-Var DA problem", eq. min3sec) --------
def cost_grad(prob, x, with_grad=True, dtype=np.float64):
    """J(x) = 1/2 ||x - xb||^2_{B^-1} + lambda/2 sum_k ||H_k M_k(x) - v_k||^2_{R^-1}.

    Reading: both norms are squared and J carries a factor 1/2 (the Gauss-
    Newton footnote of Sec. 4 uses J = 1/2 F^T F); B and R are diagonal.
    ``dtype`` np.longdouble evaluates the same function of the same FP64
    inputs in extended precision.
    """
    g = Grid.of(prob, dtype)
    x = np.asarray(x, dtype)
    sb2 = prob.sigma_b[:, None, None] ** 2
    dxb = x - np.asarray(prob.xb0, dtype)
    Jb = 0.5 * np.sum(dxb * dxb / sb2)
    traj = forward(g, x, prob.nsteps)
    flat = traj.reshape(prob.nsteps + 1, 3, -1)
    st = prob.obs_step.astype(np.int64)
    fi = prob.obs_field.astype(np.int64)
    ce = prob.obs_cell.astype(np.int64)
    r = flat[st, fi, ce] - prob.obs_value
    wo = prob.lambda_obs / prob.obs_sigma ** 2
    Jo = 0.5 * np.sum(wo * r * r)
    if not with_grad:
        return Jb + Jo
    forcing = np.zeros_like(flat)
    np.add.at(forcing, (st, fi, ce), wo * r)
    grad = dxb / sb2 + adjoint(g, traj, forcing.reshape(traj.shape))
    return Jb + Jo, grad


def mass(g: Grid, Z):
    """Discrete mass sum_ij cos(theta_j) h_ij (conserved by the flux form)."""
    return float(np.sum(g.cos[:, None] * Z[0]))
