"""Restricted model on one box, its TLM and adjoint, and the local functional.

Test infrastructure only (see the package docstring).

The restricted model (eq. restricted) is the discrete SWE of ``model`` run on
the extended box of one subdomain, started from the control at its first level
S_j, with the lateral boundary read from a halo ring frozen in time (values
supplied per level) except where the box wraps onto itself.  The stencil is
evaluated on a padded copy of the box whose one-cell frame holds the ring and
the internal wraps; the adjoint is the literal transpose of that code, written
by scattering each tangent-linear term into the padded frame and folding the
internal-wrap frame entries back into the box (ring entries get nothing).

Local functional (eq. eq:cost:parallel1), readings: every norm is squared and
J carries 1/2; the background term sits at the first level S_j and uses the
global background run restricted to the box; the observation term uses the
local trajectory at the observation level; restriction weights of Def.
defrestrfun are applied to squared terms as 1/(number of boxes covering the
point) (spatial count for the background, space-time count for observations;
``weight_mode`` 1 sets them to one); the overlap term is summed over every
intersecting neighbour subdomain s' on the shared levels and cells,
mu/2 sum_f (Z_f - T_{s',f})^2 / sigma_{b,f}^2, with T_{s'} the neighbour's
trajectory, frozen during a local evaluation.
"""
from __future__ import annotations

import numpy as np

from . import model, tz_local
from .model import Grid


class LocalGeometry:
    """Row tables and padded-frame bookkeeping for one box."""

    def __init__(self, g: Grid, maps, s):
        b = maps.boxes[s]
        self.box = b
        self.g = g
        # the Turkel-Zwas variant reads a wider frame (see tz_local)
        self.tz = tz_local.TzGeometry(g, maps, s) if g.tz is not None else None
        if self.tz is not None:
            return
        ny, nx = b.ny, b.nx
        rows = b.row0 + np.arange(ny)
        cos_ext = np.concatenate([[g.cos[0]], g.cos, [g.cos[-1]]])
        self.c = g.cos[rows][:, None]
        self.t = g.tan[rows][:, None]
        self.f = g.fcor[rows][:, None]
        self.cN = cos_ext[rows + 2][:, None]
        self.cS = cos_ext[rows][:, None]
        # padded-frame coordinates of each ring position
        pr = np.concatenate([np.zeros(nx, int), np.full(nx, ny + 1), np.arange(ny) + 1,
                             np.arange(ny) + 1])
        pc = np.concatenate([np.arange(nx) + 1, np.arange(nx) + 1, np.zeros(ny, int),
                             np.full(ny, nx + 1)])
        self.frame_flat = pr * (nx + 2) + pc
        src = maps.halo_src[s]
        self.internal = np.nonzero(src < 0)[0]
        self.ring = np.nonzero(src >= 0)[0]
        self.int_cell = maps.halo_off[s][self.internal].astype(np.int64)
        self.int_sign = maps.halo_sign[s][self.internal].astype(np.float64)

    def pad(self, Zb, ring_level):
        """Padded (3, ny+2, nx+2) array: box + ring (already signed) + wraps."""
        b = self.box
        P = np.zeros((3, b.ny + 2, b.nx + 2), dtype=Zb.dtype)
        P[:, 1:-1, 1:-1] = Zb
        Pf = P.reshape(3, -1)
        Zf = Zb.reshape(3, -1)
        ip = self.frame_flat[self.internal]
        Pf[0, ip] = Zf[0, self.int_cell]
        Pf[1, ip] = self.int_sign * Zf[1, self.int_cell]
        Pf[2, ip] = self.int_sign * Zf[2, self.int_cell]
        if ring_level is not None and self.ring.size:
            rp = self.frame_flat[self.ring]
            Pf[:, rp] = ring_level[:, self.ring]
        return P

    def fold(self, A):
        """Transpose of ``pad`` with a zero (frozen) ring."""
        out = A[:, 1:-1, 1:-1].copy().reshape(3, -1)
        Af = A.reshape(3, -1)
        ip = self.frame_flat[self.internal]
        np.add.at(out[0], self.int_cell, Af[0, ip])
        np.add.at(out[1], self.int_cell, self.int_sign * Af[1, ip])
        np.add.at(out[2], self.int_cell, self.int_sign * Af[2, ip])
        return out.reshape(3, self.box.ny, self.box.nx)


def _views(P):
    C = P[:, 1:-1, 1:-1]
    E = P[:, 1:-1, 2:]
    W = P[:, 1:-1, :-2]
    N = P[:, 2:, 1:-1]
    S = P[:, :-2, 1:-1]
    return C, E, W, N, S


def increment(geo: LocalGeometry, P):
    """(H, U, V) increments on the box interior from a padded state."""
    g = geo.g
    C, E, W, N, S = _views(P)
    h, u, v = C
    hE, uE, vE = E
    hW, uW, vW = W
    hN, uN, vN = N
    hS, uS, vS = S
    c, t, f, cN, cS = geo.c, geo.t, geo.f, geo.cN, geo.cS
    sl, st, gr, a, dt = g.sig_lon, g.sig_lat, g.gravity, g.radius, g.dt
    cor = f + u * t / a
    U = (-sl * (u / c) * (uE - uW) - st * v * (uN - uS)
         - sl * (gr / c) * (hE - hW) + 2.0 * dt * cor * v)
    V = (-sl * (u / c) * (vE - vW) - st * v * (vN - vS)
         - st * gr * (hN - hS) - 2.0 * dt * cor * u)
    H = -(sl / c) * (hE * uE - hW * uW) - (st / c) * (hN * vN * cN - hS * vS * cS)
    return np.stack([H, U, V])


def increment_tl(geo: LocalGeometry, P, dP):
    g = geo.g
    C, E, W, N, S = _views(P)
    dC, dE, dW, dN, dS = _views(dP)
    h, u, v = C
    hE, uE, vE = E
    hW, uW, vW = W
    hN, uN, vN = N
    hS, uS, vS = S
    dh, du, dv = dC
    dhE, duE, dvE = dE
    dhW, duW, dvW = dW
    dhN, duN, dvN = dN
    dhS, duS, dvS = dS
    c, t, f, cN, cS = geo.c, geo.t, geo.f, geo.cN, geo.cS
    sl, st, gr, a, dt = g.sig_lon, g.sig_lat, g.gravity, g.radius, g.dt
    cor = f + u * t / a
    dU = (-sl / c * (du * (uE - uW) + u * (duE - duW))
          - st * (dv * (uN - uS) + v * (duN - duS))
          - sl * gr / c * (dhE - dhW)
          + 2.0 * dt * (du * t / a * v + cor * dv))
    dV = (-sl / c * (du * (vE - vW) + u * (dvE - dvW))
          - st * (dv * (vN - vS) + v * (dvN - dvS))
          - st * gr * (dhN - dhS)
          - 2.0 * dt * (du * t / a * u + cor * du))
    dH = (-(sl / c) * (dhE * uE + hE * duE - dhW * uW - hW * duW)
          - (st / c) * ((dhN * vN + hN * dvN) * cN - (dhS * vS + hS * dvS) * cS))
    return np.stack([dH, dU, dV])


def increment_ad(geo: LocalGeometry, P, lam):
    """Transpose of ``increment_tl``: scatter into a padded adjoint array."""
    g = geo.g
    C, E, W, N, S = _views(P)
    h, u, v = C
    hE, uE, vE = E
    hW, uW, vW = W
    hN, uN, vN = N
    hS, uS, vS = S
    lH, lU, lV = lam
    c, t, f, cN, cS = geo.c, geo.t, geo.f, geo.cN, geo.cS
    sl, st, gr, a, dt = g.sig_lon, g.sig_lat, g.gravity, g.radius, g.dt
    cor = f + u * t / a
    A = np.zeros_like(P)
    aC, aE, aW, aN, aS = _views(A)      # views: in-place adds land in A
    # U row
    w = lU * (-sl / c)
    aC[1] += w * (uE - uW)
    aE[1] += w * u
    aW[1] -= w * u
    w = lU * (-st)
    aC[2] += w * (uN - uS)
    aN[1] += w * v
    aS[1] -= w * v
    w = lU * (-sl * gr / c)
    aE[0] += w
    aW[0] -= w
    w = lU * (2.0 * dt)
    aC[1] += w * t / a * v
    aC[2] += w * cor
    # V row
    w = lV * (-sl / c)
    aC[1] += w * (vE - vW)
    aE[2] += w * u
    aW[2] -= w * u
    w = lV * (-st)
    aC[2] += w * (vN - vS)
    aN[2] += w * v
    aS[2] -= w * v
    w = lV * (-st * gr)
    aN[0] += w
    aS[0] -= w
    w = lV * (-2.0 * dt)
    aC[1] += w * (t / a * u + cor)
    # H row
    w = lH * (-sl / c)
    aE[0] += w * uE
    aE[1] += w * hE
    aW[0] -= w * uW
    aW[1] -= w * hW
    w = lH * (-st / c)
    aN[0] += w * vN * cN
    aN[2] += w * hN * cN
    aS[0] -= w * vS * cS
    aS[2] -= w * hS * cS
    return geo.fold(A)


def forward(geo: LocalGeometry, x, ring):
    """Local trajectory [nlev][3][ny][nx] from control x and frozen ring.

    ``ring`` is [nlev][3][nring] (values as seen by the stencil, signs
    applied) or None when the box has no frozen positions.
    """
    if geo.tz is not None:
        return tz_local.forward(geo.tz, x, ring)
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


def tlm(geo: LocalGeometry, traj, ring, dx):
    if geo.tz is not None:
        return tz_local.tlm(geo.tz, traj, ring, dx)
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


def adjoint(geo: LocalGeometry, traj, ring, forcing):
    """Transpose of ``tlm`` applied to per-level forcing; returns level 0."""
    if geo.tz is not None:
        return tz_local.adjoint(geo.tz, traj, ring, forcing)
    L = traj.shape[0] - 1
    a = forcing.copy()

    def rl(n):
        return None if ring is None else ring[n]

    for n in range(L - 1, 0, -1):
        a[n - 1] += a[n + 1]
        a[n] += increment_ad(geo, geo.pad(traj[n], rl(n)), a[n + 1])
    if L >= 1:
        a[0] += a[1] + 0.5 * increment_ad(geo, geo.pad(traj[0], rl(0)), a[1])
    return a[0]


# --- frozen inputs from trajectories -----------------------------------------
def restrict_global(maps, s, gtraj):
    """Box trajectory of subdomain s cut from a global trajectory [N+1][3][nlat][nlon]."""
    b = maps.boxes[s]
    rows = b.row0 + np.arange(b.ny)
    cols = (b.col0 + np.arange(b.nx)) % maps.nlon
    return gtraj[b.lev0:b.lev0 + b.nlev][:, :, rows][:, :, :, cols]


def ring_from_trajs(maps, s, trajs):
    """Frozen ring of s [nlev][3][nring] from the owners' box trajectories.

    ``trajs`` maps subdomain index -> box trajectory [nlev][3][ny][nx]; owners
    share the interval of s, so local level indices coincide.
    """
    b = maps.boxes[s]
    src = maps.halo_src[s]
    off = maps.halo_off[s]
    sgn = maps.halo_sign[s].astype(np.float64)
    ring = np.zeros((b.nlev, 3, b.nring), dtype=next(iter(trajs.values())).dtype)
    for k in np.nonzero(src >= 0)[0]:
        t = trajs[int(src[k])].reshape(b.nlev, 3, -1)
        ring[:, 0, k] = t[:, 0, off[k]]
        ring[:, 1, k] = sgn[k] * t[:, 1, off[k]]
        ring[:, 2, k] = sgn[k] * t[:, 2, off[k]]
    return ring


def weights(prob, maps, s):
    """Background weight per box cell and the space-time count function."""
    b = maps.boxes[s]
    gr, gc = maps.box_cells_global(b)
    csp = maps.cover_sp[gr, gc].astype(np.float64)
    if prob.weight_mode == 1:
        return np.ones_like(csp), csp
    return 1.0 / csp, csp


def cost_grad(prob, maps, s, x, xb, ring, nbr_trajs, with_grad=True, parts=False,
              dtype=np.float64):
    """Local functional J_s(x) and its gradient (eq. eq:cost:parallel1).

    x, xb      : [3][ny][nx] control and background at level S_j
    ring       : [nlev][3][nring] frozen halo values (or None)
    nbr_trajs  : dict s' -> box trajectory of every overlap neighbour s'
                 (levels from the neighbour's first level on; only the levels
                 it shares with s are read)
    dtype      : arithmetic type; np.longdouble evaluates the same function
                 of the same FP64 inputs in extended precision
    """
    if dtype is not np.float64:
        x, xb = np.asarray(x, dtype), np.asarray(xb, dtype)
        ring = None if ring is None else np.asarray(ring, dtype)
        nbr_trajs = {k: np.asarray(v, dtype) for k, v in nbr_trajs.items()}
    g = Grid.of(prob, dtype)
    geo = LocalGeometry(g, maps, s)
    b = maps.boxes[s]
    sb2 = prob.sigma_b[:, None, None] ** 2
    wb, csp = weights(prob, maps, s)
    wb = wb.reshape(b.ny, b.nx)
    dxb = x - xb
    Jb = 0.5 * np.sum(wb * dxb * dxb / sb2)

    traj = forward(geo, x, ring)
    flat = traj.reshape(b.nlev, 3, -1)
    forcing = np.zeros_like(flat)

    # observation term
    idx = maps.obs_bin[s]
    Jo = 0.0
    if idx.size:
        st = prob.obs_step[idx].astype(np.int64)
        cell = prob.obs_cell[idx].astype(np.int64)
        fld = prob.obs_field[idx].astype(np.int64)
        loc = maps.box_index(b, cell // prob.nlon, cell % prob.nlon)
        assert (loc >= 0).all()
        n = st - b.lev0
        if prob.weight_mode == 1:
            wo = np.ones(idx.size)
        else:
            wo = 1.0 / (csp[loc] * maps.time_count[st])
        r = flat[n, fld, loc] - prob.obs_value[idx]
        q = prob.lambda_obs * wo / prob.obs_sigma[idx] ** 2
        Jo = 0.5 * np.sum(q * r * r)
        np.add.at(forcing, (n, fld, loc), q * r)

    # overlap term, neighbour by neighbour
    Jov = 0.0
    mu = prob.mu_overlap
    gr, gc = maps.box_cells_global(b)
    sb2f = (prob.sigma_b ** 2)[:, None]
    for sp in maps.neighbors[s]:
        bp = maps.boxes[int(sp)]
        lo = max(b.lev0, bp.lev0)
        hi = min(b.lev0 + b.nlev, bp.lev0 + bp.nlev)
        if lo >= hi:
            continue
        idxp = maps.box_index(bp, gr, gc)
        mine = np.nonzero(idxp >= 0)[0]
        if mine.size == 0:
            continue
        theirs = idxp[mine]
        T = nbr_trajs[int(sp)].reshape(-1, 3, bp.ny * bp.nx)
        for lev in range(lo, hi):
            e = flat[lev - b.lev0][:, mine] - T[lev - bp.lev0][:, theirs]
            Jov += 0.5 * mu * np.sum(e * e / sb2f)
            forcing[lev - b.lev0][:, mine] += mu * e / sb2f

    J = Jb + Jo + Jov
    if not with_grad:
        return (J, (Jb, Jo, Jov)) if parts else J
    grad = wb * dxb / sb2 + adjoint(geo, traj, ring, forcing.reshape(traj.shape))
    if parts:
        return J, grad, (Jb, Jo, Jov)
    return J, grad
