"""Turkel-Zwas variant on one box: the restricted model with a frozen pad q
rows and p columns wide (corners included), its TLM and adjoint.

Test infrastructure only (see the package docstring).

The increments of ``tz`` (Sec. 7 discrete U, V, H with offsets p, q and
averaging alpha, same readings) are evaluated on the box interior of a padded
frame [3][ny+2q][nx+2p] that holds the box, the frozen pad values of the
level (signs applied, see ``ddmaps``), the pad positions that map into the
box itself (spanning boxes: across a pole) and, for a box spanning the
circle, its own columns wrapped onto the east and west frame columns.  The
value at offset (dr, dc) of box cell (r, c) is the frame entry
(q + r + dr, p + c + dc); row tables (cos, tan, f) of a frame row are those
of the global row it maps to.  The adjoint is the transpose of the tangent
linear code, term by term: each term is added into a frame-shaped adjoint at
the offset it was read from, then the frame is folded back onto the box
(wrapped columns and internal pad positions into their cells, frozen
positions dropped).
"""
from __future__ import annotations

import numpy as np

from . import ddmaps


class TzGeometry:
    """Frame bookkeeping and row tables of one box under the variant."""

    def __init__(self, g, maps, s):
        b = maps.boxes[s]
        self.box, self.g = b, g
        self.p, self.q, self.alpha = g.tz
        p, q = self.p, self.q
        if (b.pad_p, b.pad_q) != (p, q):
            raise ValueError("the maps were not built for these offsets")
        ny, nx, nlat = b.ny, b.nx, g.nlat
        self.FX = nx + 2 * p
        grow = b.row0 + np.arange(-q, ny + q)
        mrow = np.where(grow < 0, -1 - grow, np.where(grow >= nlat, 2 * nlat - 1 - grow, grow))
        self.cos_f, self.tan_f, self.f_f = g.cos[mrow], g.tan[mrow], g.fcor[mrow]
        rr, cc = ddmaps.ring_coords(b)
        self.frame_flat = (rr + q) * self.FX + (cc + p)
        src = maps.halo_src[s]
        self.frozen = np.nonzero(src >= 0)[0]
        self.internal = np.nonzero(src < 0)[0]
        self.int_cell = maps.halo_off[s][self.internal].astype(np.int64)
        self.int_sign = maps.halo_sign[s][self.internal].astype(np.float64)

    # -- frame ----------------------------------------------------------------
    def pad(self, Zb, ring_level):
        b, p, q = self.box, self.p, self.q
        ny, nx = b.ny, b.nx
        P = np.zeros((3, ny + 2 * q, nx + 2 * p), dtype=Zb.dtype)
        P[:, q:q + ny, p:p + nx] = Zb
        Pf = P.reshape(3, -1)
        Zf = Zb.reshape(3, -1)
        ip = self.frame_flat[self.internal]
        Pf[0, ip] = Zf[0, self.int_cell]
        Pf[1, ip] = self.int_sign * Zf[1, self.int_cell]
        Pf[2, ip] = self.int_sign * Zf[2, self.int_cell]
        if ring_level is not None and self.frozen.size:
            Pf[:, self.frame_flat[self.frozen]] = ring_level[:, self.frozen]
        if b.span:
            P[:, :, :p] = P[:, :, nx:nx + p]
            P[:, :, p + nx:] = P[:, :, p:2 * p]
        return P

    def fold(self, A):
        """Transpose of ``pad`` with a zero (frozen) pad."""
        b, p, q = self.box, self.p, self.q
        ny, nx = b.ny, b.nx
        A = A.copy()
        if b.span:
            A[:, :, nx:nx + p] += A[:, :, :p]
            A[:, :, p:2 * p] += A[:, :, p + nx:]
        out = A[:, q:q + ny, p:p + nx].copy().reshape(3, -1)
        Af = A.reshape(3, -1)
        ip = self.frame_flat[self.internal]
        np.add.at(out[0], self.int_cell, Af[0, ip])
        np.add.at(out[1], self.int_cell, self.int_sign * Af[1, ip])
        np.add.at(out[2], self.int_cell, self.int_sign * Af[2, ip])
        return out.reshape(3, ny, nx)

    # -- views ----------------------------------------------------------------
    def at(self, P, f, dr, dc):
        """Field f at offset (dr, dc) of every box cell."""
        ny, nx, p, q = self.box.ny, self.box.nx, self.p, self.q
        return P[f, q + dr:q + dr + ny, p + dc:p + dc + nx]

    def rows(self, tab, dr):
        """Row table at row offset dr, as a column."""
        return tab[self.q + dr:self.q + dr + self.box.ny][:, None]

    def add(self, A, f, dr, dc, w):
        """Transpose of ``at``: w added where (dr, dc) was read."""
        ny, nx, p, q = self.box.ny, self.box.nx, self.p, self.q
        A[f, q + dr:q + dr + ny, p + dc:p + dc + nx] += w


def _consts(geo):
    g = geo.g
    return g.sig_lon, g.sig_lat, g.gravity, g.radius, g.dt


def _div(geo, P):
    """The averaged divergences (Dl, Dt) of H at P."""
    at, p, q, al = geo.at, geo.p, geo.q, geo.alpha
    cN, cS = geo.rows(geo.cos_f, q), geo.rows(geo.cos_f, -q)
    Dl = ((1 - al) * (at(P, 1, 0, p) - at(P, 1, 0, -p))
          + 0.5 * al * (at(P, 1, q, p) - at(P, 1, q, -p) + at(P, 1, -q, p) - at(P, 1, -q, -p))) / p
    Dt = ((1 - al) * (at(P, 2, q, 0) * cN - at(P, 2, -q, 0) * cS)
          + 0.5 * al * (at(P, 2, q, p) * cN - at(P, 2, -q, p) * cS)
          + 0.5 * al * (at(P, 2, q, -p) * cN - at(P, 2, -q, -p) * cS)) / q
    return Dl, Dt


def increment(geo: TzGeometry, P):
    """(H, U, V) increments over 2 dt on the box interior of frame P."""
    sl, st, gr, a, dt = _consts(geo)
    at, p, q, al = geo.at, geo.p, geo.q, geo.alpha
    c, t, f = geo.rows(geo.cos_f, 0), geo.rows(geo.tan_f, 0), geo.rows(geo.f_f, 0)
    tN, tS = geo.rows(geo.tan_f, q), geo.rows(geo.tan_f, -q)
    fN, fS = geo.rows(geo.f_f, q), geo.rows(geo.f_f, -q)
    h, u, v = at(P, 0, 0, 0), at(P, 1, 0, 0), at(P, 2, 0, 0)
    uEp, uWp, vEp, vWp = at(P, 1, 0, p), at(P, 1, 0, -p), at(P, 2, 0, p), at(P, 2, 0, -p)
    uNq, uSq = at(P, 1, q, 0), at(P, 1, -q, 0)
    U = (-sl * (u / c) * (at(P, 1, 0, 1) - at(P, 1, 0, -1)) - st * v * (at(P, 1, 1, 0) - at(P, 1, -1, 0))
         - sl * gr / (p * c) * (at(P, 0, 0, p) - at(P, 0, 0, -p))
         + 2.0 * dt * ((1 - al) * (f + u * t / a) * v
                       + 0.5 * al * (f + uEp * t / a) * vEp
                       + 0.5 * al * (f + uWp * t / a) * vWp))
    V = (-sl * (u / c) * (at(P, 2, 0, 1) - at(P, 2, 0, -1)) - st * v * (at(P, 2, 1, 0) - at(P, 2, -1, 0))
         - st * gr / q * (at(P, 0, q, 0) - at(P, 0, -q, 0))
         - 2.0 * dt * ((1 - al) * (f + u * t / a) * u
                       + 0.5 * al * (fN + uNq * tN / a) * uNq
                       + 0.5 * al * (fS + uSq * tS / a) * uSq))
    Dl, Dt = _div(geo, P)
    H = (-(sl / c) * (u * (at(P, 0, 0, 1) - at(P, 0, 0, -1)) + h * Dl)
         - st * (v * (at(P, 0, 1, 0) - at(P, 0, -1, 0)) + (h / c) * Dt))
    return np.stack([H, U, V])


def increment_tl(geo: TzGeometry, P, dP):
    """Tangent linear of ``increment`` at frame P applied to frame dP."""
    sl, st, gr, a, dt = _consts(geo)
    at, p, q, al = geo.at, geo.p, geo.q, geo.alpha
    c, t, f = geo.rows(geo.cos_f, 0), geo.rows(geo.tan_f, 0), geo.rows(geo.f_f, 0)
    tN, tS = geo.rows(geo.tan_f, q), geo.rows(geo.tan_f, -q)
    fN, fS = geo.rows(geo.f_f, q), geo.rows(geo.f_f, -q)
    h, u, v = at(P, 0, 0, 0), at(P, 1, 0, 0), at(P, 2, 0, 0)
    dh, du, dv = at(dP, 0, 0, 0), at(dP, 1, 0, 0), at(dP, 2, 0, 0)
    uEp, uWp, vEp, vWp = at(P, 1, 0, p), at(P, 1, 0, -p), at(P, 2, 0, p), at(P, 2, 0, -p)
    uNq, uSq = at(P, 1, q, 0), at(P, 1, -q, 0)
    dU = (-sl / c * (du * (at(P, 1, 0, 1) - at(P, 1, 0, -1)) + u * (at(dP, 1, 0, 1) - at(dP, 1, 0, -1)))
          - st * (dv * (at(P, 1, 1, 0) - at(P, 1, -1, 0)) + v * (at(dP, 1, 1, 0) - at(dP, 1, -1, 0)))
          - sl * gr / (p * c) * (at(dP, 0, 0, p) - at(dP, 0, 0, -p))
          + 2.0 * dt * ((1 - al) * ((du * t / a) * v + (f + u * t / a) * dv)
                        + 0.5 * al * ((at(dP, 1, 0, p) * t / a) * vEp + (f + uEp * t / a) * at(dP, 2, 0, p))
                        + 0.5 * al * ((at(dP, 1, 0, -p) * t / a) * vWp
                                      + (f + uWp * t / a) * at(dP, 2, 0, -p))))
    dV = (-sl / c * (du * (at(P, 2, 0, 1) - at(P, 2, 0, -1)) + u * (at(dP, 2, 0, 1) - at(dP, 2, 0, -1)))
          - st * (dv * (at(P, 2, 1, 0) - at(P, 2, -1, 0)) + v * (at(dP, 2, 1, 0) - at(dP, 2, -1, 0)))
          - st * gr / q * (at(dP, 0, q, 0) - at(dP, 0, -q, 0))
          - 2.0 * dt * ((1 - al) * (f + 2.0 * u * t / a) * du
                        + 0.5 * al * (fN + 2.0 * uNq * tN / a) * at(dP, 1, q, 0)
                        + 0.5 * al * (fS + 2.0 * uSq * tS / a) * at(dP, 1, -q, 0)))
    Dl, Dt = _div(geo, P)
    dDl, dDt = _div(geo, dP)
    dH = (-(sl / c) * (du * (at(P, 0, 0, 1) - at(P, 0, 0, -1)) + u * (at(dP, 0, 0, 1) - at(dP, 0, 0, -1))
                       + dh * Dl + h * dDl)
          - st * (dv * (at(P, 0, 1, 0) - at(P, 0, -1, 0)) + v * (at(dP, 0, 1, 0) - at(dP, 0, -1, 0))
                  + (dh / c) * Dt + (h / c) * dDt))
    return np.stack([dH, dU, dV])


def increment_ad(geo: TzGeometry, P, lam):
    """Transpose of ``increment_tl`` at frame P applied to lam = (lamH, lamU,
    lamV) on the box; returns the frame-shaped adjoint (fold it with
    ``geo.fold``)."""
    sl, st, gr, a, dt = _consts(geo)
    at, add, p, q, al = geo.at, geo.add, geo.p, geo.q, geo.alpha
    c, t, f = geo.rows(geo.cos_f, 0), geo.rows(geo.tan_f, 0), geo.rows(geo.f_f, 0)
    cN, cS = geo.rows(geo.cos_f, q), geo.rows(geo.cos_f, -q)
    tN, tS = geo.rows(geo.tan_f, q), geo.rows(geo.tan_f, -q)
    fN, fS = geo.rows(geo.f_f, q), geo.rows(geo.f_f, -q)
    h, u, v = at(P, 0, 0, 0), at(P, 1, 0, 0), at(P, 2, 0, 0)
    uEp, uWp, vEp, vWp = at(P, 1, 0, p), at(P, 1, 0, -p), at(P, 2, 0, p), at(P, 2, 0, -p)
    uNq, uSq = at(P, 1, q, 0), at(P, 1, -q, 0)
    lH, lU, lV = lam
    A = np.zeros_like(P)
    H, U, V = 0, 1, 2
    # dU
    w = lU * (-sl / c)
    add(A, U, 0, 0, w * (at(P, 1, 0, 1) - at(P, 1, 0, -1)))
    add(A, U, 0, 1, w * u)
    add(A, U, 0, -1, -w * u)
    w = lU * (-st)
    add(A, V, 0, 0, w * (at(P, 1, 1, 0) - at(P, 1, -1, 0)))
    add(A, U, 1, 0, w * v)
    add(A, U, -1, 0, -w * v)
    w = lU * (-sl * gr / (p * c))
    add(A, H, 0, p, w)
    add(A, H, 0, -p, -w)
    w = lU * 2.0 * dt
    add(A, U, 0, 0, w * (1 - al) * (t / a) * v)
    add(A, V, 0, 0, w * (1 - al) * (f + u * t / a))
    add(A, U, 0, p, w * 0.5 * al * (t / a) * vEp)
    add(A, V, 0, p, w * 0.5 * al * (f + uEp * t / a))
    add(A, U, 0, -p, w * 0.5 * al * (t / a) * vWp)
    add(A, V, 0, -p, w * 0.5 * al * (f + uWp * t / a))
    # dV
    w = lV * (-sl / c)
    add(A, U, 0, 0, w * (at(P, 2, 0, 1) - at(P, 2, 0, -1)))
    add(A, V, 0, 1, w * u)
    add(A, V, 0, -1, -w * u)
    w = lV * (-st)
    add(A, V, 0, 0, w * (at(P, 2, 1, 0) - at(P, 2, -1, 0)))
    add(A, V, 1, 0, w * v)
    add(A, V, -1, 0, -w * v)
    w = lV * (-st * gr / q)
    add(A, H, q, 0, w)
    add(A, H, -q, 0, -w)
    w = lV * (-2.0 * dt)
    add(A, U, 0, 0, w * (1 - al) * (f + 2.0 * u * t / a))
    add(A, U, q, 0, w * 0.5 * al * (fN + 2.0 * uNq * tN / a))
    add(A, U, -q, 0, w * 0.5 * al * (fS + 2.0 * uSq * tS / a))
    # dH
    Dl, Dt = _div(geo, P)
    w = lH * (-sl / c)
    add(A, U, 0, 0, w * (at(P, 0, 0, 1) - at(P, 0, 0, -1)))
    add(A, H, 0, 1, w * u)
    add(A, H, 0, -1, -w * u)
    add(A, H, 0, 0, w * Dl)
    wl = w * h / p                                   # weight of dDl * p
    add(A, U, 0, p, (1 - al) * wl)
    add(A, U, 0, -p, -(1 - al) * wl)
    add(A, U, q, p, 0.5 * al * wl)
    add(A, U, q, -p, -0.5 * al * wl)
    add(A, U, -q, p, 0.5 * al * wl)
    add(A, U, -q, -p, -0.5 * al * wl)
    w = lH * (-st)
    add(A, V, 0, 0, w * (at(P, 0, 1, 0) - at(P, 0, -1, 0)))
    add(A, H, 1, 0, w * v)
    add(A, H, -1, 0, -w * v)
    add(A, H, 0, 0, w * Dt / c)
    wt = w * h / (c * q)                             # weight of dDt * q
    add(A, V, q, 0, (1 - al) * wt * cN)
    add(A, V, -q, 0, -(1 - al) * wt * cS)
    add(A, V, q, p, 0.5 * al * wt * cN)
    add(A, V, -q, p, -0.5 * al * wt * cS)
    add(A, V, q, -p, 0.5 * al * wt * cN)
    add(A, V, -q, -p, -0.5 * al * wt * cS)
    return A


# -- restricted model on the box ------------------------------------------------
def forward(geo: TzGeometry, x, ring):
    """Local trajectory [nlev][3][ny][nx] from control x and frozen pad values
    ``ring`` [nlev][3][nring] (or None)."""
    L = geo.box.nlev - 1
    traj = np.empty((L + 1,) + x.shape, dtype=x.dtype)
    traj[0] = x

    def rl(n):
        return None if ring is None else ring[n]

    if L >= 1:
        traj[1] = x + 0.5 * increment(geo, geo.pad(x, rl(0)))
    for n in range(1, L):
        traj[n + 1] = traj[n - 1] + increment(geo, geo.pad(traj[n], rl(n)))
    return traj


def tlm(geo: TzGeometry, traj, ring, dx):
    L = traj.shape[0] - 1
    d = np.empty_like(traj)
    d[0] = dx

    def rl(n):
        return None if ring is None else ring[n]

    if L >= 1:
        d[1] = dx + 0.5 * increment_tl(geo, geo.pad(traj[0], rl(0)), geo.pad(dx, None))
    for n in range(1, L):
        d[n + 1] = d[n - 1] + increment_tl(geo, geo.pad(traj[n], rl(n)), geo.pad(d[n], None))
    return d


def adjoint(geo: TzGeometry, traj, ring, forcing):
    """Transpose of ``tlm`` applied to per-level forcing; returns level 0."""
    L = traj.shape[0] - 1
    a = forcing.copy()

    def rl(n):
        return None if ring is None else ring[n]

    def jt(n, lam):
        return geo.fold(increment_ad(geo, geo.pad(traj[n], rl(n)), lam))

    for n in range(L - 1, 0, -1):
        a[n - 1] += a[n + 1]
        a[n] += jt(n, a[n + 1])
    if L >= 1:
        a[0] += a[1] + 0.5 * jt(0, a[1])
    return a[0]
