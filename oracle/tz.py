"""Turkel-Zwas variant of the discrete SWE (Sec. 7, discrete U, V, H with
coarse offsets p, q and averaging alpha), its TLM and its adjoint (FP64).

Test infrastructure only (see the package docstring).

The pressure-gradient terms of U and V, the divergence terms of H and the
Coriolis terms are taken over p columns and q rows; advection keeps offset
one.  Readings of the printed scheme:

* H carries the leading factor -sigma (sigma_lon on the longitude terms,
  sigma_lat on the latitude ones) and the latitude divergence the factor
  h / cos(theta) that the longitude one has; H is the advective form as
  printed, so it conserves no discrete mass (the flux form of the plain
  scheme has no counterpart with the wide divergence offsets);
* U and V read as in the plain scheme (2 dt on the Coriolis bracket, v
  differences for the meridional advection of v, a minus sign on the
  Coriolis term of V); the alpha-averaged Coriolis terms take u, v, f and
  tan(theta) at the neighbour: (i +- p, j) in U, (i, j +- q) in V;
* the alpha terms of H average the divergence over the corners
  (i +- p, j +- q);
* a row k beyond a pole (k = 1 .. q) is the k-th row from the pole on the
  other side of it: the same latitude, shifted by half a circle, u and v
  negated, with that row's cos, f and tan.

h is the full height here.  Field order (h, u, v); arrays [3][nlat][nlon].
"""
from __future__ import annotations

import numpy as np


def shift_lon(x, k):
    """Value at column i + k (periodic)."""
    return np.roll(x, -k, axis=-1)


def shift_lon_T(y, k):
    return np.roll(y, k, axis=-1)


def _src_rows(nlat, k):
    """Source row of every row j + k, and whether it lies across a pole (the
    row at the same depth on the other side)."""
    s = np.arange(nlat) + k
    across = (s >= nlat) | (s < 0)
    return np.where(s >= nlat, 2 * nlat - 1 - s, np.where(s < 0, -1 - s, s)), across


def shift_lat(x, k, sign):
    """Value at row j + k; rows beyond a pole come from across it, shifted by
    half a circle and multiplied by ``sign`` (-1 for u, v)."""
    nlat, nlon = x.shape[-2], x.shape[-1]
    src, across = _src_rows(nlat, k)
    out = x[src].copy()
    out[across] = sign * np.roll(out[across], -(nlon // 2), axis=-1)
    return out


def shift_lat_T(y, k, sign):
    """Transpose of ``shift_lat``."""
    nlat, nlon = y.shape[-2], y.shape[-1]
    src, across = _src_rows(nlat, k)
    contrib = y.copy()
    contrib[across] = sign * np.roll(y[across], nlon // 2, axis=-1)
    out = np.zeros_like(y)
    np.add.at(out, src, contrib)
    return out


def row_at(a, k):
    """Per-row table at row j + k (the source row's value beyond a pole)."""
    return a[_src_rows(a.shape[0], k)[0]][:, None]


class _Nbrs:
    """The state at the 13 points the scheme reads, and the row tables."""

    def __init__(self, g, Z, p, q):
        h, u, v = Z
        self.h, self.u, self.v = h, u, v
        L = lambda x, k: shift_lon(x, k)
        N = lambda x, k, s: shift_lat(x, k, s)
        self.uE, self.uW, self.vE, self.vW = L(u, 1), L(u, -1), L(v, 1), L(v, -1)
        self.hE, self.hW = L(h, 1), L(h, -1)
        self.uN, self.uS, self.vN, self.vS = N(u, 1, -1), N(u, -1, -1), N(v, 1, -1), N(v, -1, -1)
        self.hN, self.hS = N(h, 1, 1), N(h, -1, 1)
        self.hEp, self.hWp = L(h, p), L(h, -p)
        self.uEp, self.uWp, self.vEp, self.vWp = L(u, p), L(u, -p), L(v, p), L(v, -p)
        self.hNq, self.hSq = N(h, q, 1), N(h, -q, 1)
        self.uNq, self.uSq = N(u, q, -1), N(u, -q, -1)
        self.vNq, self.vSq = N(v, q, -1), N(v, -q, -1)
        # corners: across the pole first (half-circle shift), then p columns
        self.uEN, self.uWN = L(self.uNq, p), L(self.uNq, -p)
        self.uES, self.uWS = L(self.uSq, p), L(self.uSq, -p)
        self.vEN, self.vWN = L(self.vNq, p), L(self.vNq, -p)
        self.vES, self.vWS = L(self.vSq, p), L(self.vSq, -p)
        self.c, self.t, self.f = g.cos[:, None], g.tan[:, None], g.fcor[:, None]
        self.cNq, self.cSq = row_at(g.cos, q), row_at(g.cos, -q)
        self.tNq, self.tSq = row_at(g.tan, q), row_at(g.tan, -q)
        self.fNq, self.fSq = row_at(g.fcor, q), row_at(g.fcor, -q)


def increment(g, Z, p, q, alpha):
    """(H, U, V) increments over 2 dt of the Turkel-Zwas scheme."""
    n = _Nbrs(g, Z, p, q)
    h, u, v = n.h, n.u, n.v
    sl, st, gr, a, dt = g.sig_lon, g.sig_lat, g.gravity, g.radius, g.dt
    al = alpha
    c, t, f = n.c, n.t, n.f
    U = (-sl * (u / c) * (n.uE - n.uW) - st * v * (n.uN - n.uS)
         - sl * gr / (p * c) * (n.hEp - n.hWp)
         + 2.0 * dt * ((1 - al) * (f + u * t / a) * v
                       + 0.5 * al * (f + n.uEp * t / a) * n.vEp
                       + 0.5 * al * (f + n.uWp * t / a) * n.vWp))
    V = (-sl * (u / c) * (n.vE - n.vW) - st * v * (n.vN - n.vS)
         - st * gr / q * (n.hNq - n.hSq)
         - 2.0 * dt * ((1 - al) * (f + u * t / a) * u
                       + 0.5 * al * (n.fNq + n.uNq * n.tNq / a) * n.uNq
                       + 0.5 * al * (n.fSq + n.uSq * n.tSq / a) * n.uSq))
    Dl = ((1 - al) * (n.uEp - n.uWp) + 0.5 * al * (n.uEN - n.uWN + n.uES - n.uWS)) / p
    Dt = ((1 - al) * (n.vNq * n.cNq - n.vSq * n.cSq)
          + 0.5 * al * (n.vEN * n.cNq - n.vES * n.cSq)
          + 0.5 * al * (n.vWN * n.cNq - n.vWS * n.cSq)) / q
    H = (-(sl / c) * (u * (n.hE - n.hW) + h * Dl)
         - st * (v * (n.hN - n.hS) + (h / c) * Dt))
    return np.stack([H, U, V])


def increment_tl(g, Z, dZ, p, q, alpha):
    """Tangent linear of ``increment`` at Z applied to dZ."""
    n = _Nbrs(g, Z, p, q)
    d = _Nbrs(g, dZ, p, q)
    h, u, v = n.h, n.u, n.v
    dh, du, dv = d.h, d.u, d.v
    sl, st, gr, a, dt = g.sig_lon, g.sig_lat, g.gravity, g.radius, g.dt
    al = alpha
    c, t, f = n.c, n.t, n.f
    dU = (-sl / c * (du * (n.uE - n.uW) + u * (d.uE - d.uW))
          - st * (dv * (n.uN - n.uS) + v * (d.uN - d.uS))
          - sl * gr / (p * c) * (d.hEp - d.hWp)
          + 2.0 * dt * ((1 - al) * ((du * t / a) * v + (f + u * t / a) * dv)
                        + 0.5 * al * ((d.uEp * t / a) * n.vEp + (f + n.uEp * t / a) * d.vEp)
                        + 0.5 * al * ((d.uWp * t / a) * n.vWp + (f + n.uWp * t / a) * d.vWp)))
    dV = (-sl / c * (du * (n.vE - n.vW) + u * (d.vE - d.vW))
          - st * (dv * (n.vN - n.vS) + v * (d.vN - d.vS))
          - st * gr / q * (d.hNq - d.hSq)
          - 2.0 * dt * ((1 - al) * (f + 2.0 * u * t / a) * du
                        + 0.5 * al * (n.fNq + 2.0 * n.uNq * n.tNq / a) * d.uNq
                        + 0.5 * al * (n.fSq + 2.0 * n.uSq * n.tSq / a) * d.uSq))
    Dl = ((1 - al) * (n.uEp - n.uWp) + 0.5 * al * (n.uEN - n.uWN + n.uES - n.uWS)) / p
    dDl = ((1 - al) * (d.uEp - d.uWp) + 0.5 * al * (d.uEN - d.uWN + d.uES - d.uWS)) / p
    Dt = ((1 - al) * (n.vNq * n.cNq - n.vSq * n.cSq)
          + 0.5 * al * (n.vEN * n.cNq - n.vES * n.cSq)
          + 0.5 * al * (n.vWN * n.cNq - n.vWS * n.cSq)) / q
    dDt = ((1 - al) * (d.vNq * n.cNq - d.vSq * n.cSq)
           + 0.5 * al * (d.vEN * n.cNq - d.vES * n.cSq)
           + 0.5 * al * (d.vWN * n.cNq - d.vWS * n.cSq)) / q
    dH = (-(sl / c) * (du * (n.hE - n.hW) + u * (d.hE - d.hW) + dh * Dl + h * dDl)
          - st * (dv * (n.hN - n.hS) + v * (d.hN - d.hS) + (dh / c) * Dt + (h / c) * dDt))
    return np.stack([dH, dU, dV])


def increment_ad(g, Z, lam, p, q, alpha):
    """Transpose of ``increment_tl`` at Z applied to lam = (lamH, lamU, lamV),
    each term of the tangent linear code transposed in turn (scatter form)."""
    n = _Nbrs(g, Z, p, q)
    h, u, v = n.h, n.u, n.v
    lH, lU, lV = lam
    sl, st, gr, a, dt = g.sig_lon, g.sig_lat, g.gravity, g.radius, g.dt
    al = alpha
    c, t, f = n.c, n.t, n.f
    ah, au, av = np.zeros_like(h), np.zeros_like(u), np.zeros_like(v)
    LT, NT = shift_lon_T, shift_lat_T

    def corner_T(w, kl, kq):
        # transpose of x -> shift_lon(shift_lat(x, kq, -1), kl)
        return NT(LT(w, kl), kq, -1.0)

    # dU
    w = lU * (-sl / c)
    au += w * (n.uE - n.uW)
    au += LT(w * u, 1) - LT(w * u, -1)
    w = lU * (-st)
    av += w * (n.uN - n.uS)
    au += NT(w * v, 1, -1.0) - NT(w * v, -1, -1.0)
    w = lU * (-sl * gr / (p * c))
    ah += LT(w, p) - LT(w, -p)
    w = lU * 2.0 * dt
    au += w * (1 - al) * (t / a) * v
    av += w * (1 - al) * (f + u * t / a)
    au += LT(w * 0.5 * al * (t / a) * n.vEp, p) + LT(w * 0.5 * al * (t / a) * n.vWp, -p)
    av += LT(w * 0.5 * al * (f + n.uEp * t / a), p) + LT(w * 0.5 * al * (f + n.uWp * t / a), -p)
    # dV
    w = lV * (-sl / c)
    au += w * (n.vE - n.vW)
    av += LT(w * u, 1) - LT(w * u, -1)
    w = lV * (-st)
    av += w * (n.vN - n.vS)
    av += NT(w * v, 1, -1.0) - NT(w * v, -1, -1.0)
    w = lV * (-st * gr / q)
    ah += NT(w, q, 1.0) - NT(w, -q, 1.0)
    w = lV * (-2.0 * dt)
    au += w * (1 - al) * (f + 2.0 * u * t / a)
    au += NT(w * 0.5 * al * (n.fNq + 2.0 * n.uNq * n.tNq / a), q, -1.0)
    au += NT(w * 0.5 * al * (n.fSq + 2.0 * n.uSq * n.tSq / a), -q, -1.0)
    # dH
    Dl = ((1 - al) * (n.uEp - n.uWp) + 0.5 * al * (n.uEN - n.uWN + n.uES - n.uWS)) / p
    Dt = ((1 - al) * (n.vNq * n.cNq - n.vSq * n.cSq)
          + 0.5 * al * (n.vEN * n.cNq - n.vES * n.cSq)
          + 0.5 * al * (n.vWN * n.cNq - n.vWS * n.cSq)) / q
    w = lH * (-sl / c)
    au += w * (n.hE - n.hW)
    ah += LT(w * u, 1) - LT(w * u, -1)
    ah += w * Dl
    wl = w * h / p                                  # weight of dDl * p
    au += (1 - al) * (LT(wl, p) - LT(wl, -p))
    au += 0.5 * al * (corner_T(wl, p, q) - corner_T(wl, -p, q)
                      + corner_T(wl, p, -q) - corner_T(wl, -p, -q))
    w = lH * (-st)
    av += w * (n.hN - n.hS)
    ah += NT(w * v, 1, 1.0) - NT(w * v, -1, 1.0)
    ah += w * Dt / c
    wt = w * h / (c * q)                            # weight of dDt * q
    av += (1 - al) * (NT(wt * n.cNq, q, -1.0) - NT(wt * n.cSq, -q, -1.0))
    av += 0.5 * al * (corner_T(wt * n.cNq, p, q) - corner_T(wt * n.cSq, p, -q)
                      + corner_T(wt * n.cNq, -p, q) - corner_T(wt * n.cSq, -p, -q))
    return np.stack([ah, au, av])
