"""Gauss-Newton local solver (Alg. 5 / Alg. 6) on the CPU, FP64.

Test infrastructure only (see the package docstring).

The local functional J_s of ``local.cost_grad`` is a sum of weighted squares
of residuals that are affine in the control (background) or in the local
trajectory (observations, overlap penalty), so J_s = 1/2 |F(x)|^2 and the
Gauss-Newton normal matrix at x (eqs. line5and7, line6and7 with the
restrictions of B and R) is

    A(x) = B_w^{-1} + M'(x)^T W M'(x),

where M'(x) is the tangent linear model of the local sweep about the
trajectory of x (control -> every local level), B_w^{-1} the diagonal
background weight w^b / sigma_b^2 of each control entry and W the diagonal
weight of each local trajectory entry: lambda w_o / sigma_o^2 summed over
the observations of that entry and mu / sigma_b^2 once per overlap
neighbour sharing it.  The right-hand side is -grad J_s(x), which at
x = x^b reduces to G^T R^{-1} d of eq. line6and7 (d the misfit of Alg. 6)
and in general carries the overlap and background terms as well.

Readings (the paper names the solver of the normal equations, a
B-preconditioned Krylov method, Alg. 7, but gives only its citation):

* preconditioning by the diagonal square root V = diag(sigma_b) of B
  (eqs. EqV, Eq_matrixAV): the system is solved for xi = delta x / sigma_b,
  (V A V) xi = -V grad J_s, whose background block is diag(w^b), the
  identity of eq. Eq_matrixAV:1 when every restriction weight is one;
* the Krylov method is textbook conjugate gradients from xi = 0, stopped
  after ``cg_max_iter`` iterations, when |r| <= cg_rtol |r_0|, or when the
  curvature p^T A p is not positive; or, as Alg. 7 names, the Lanczos
  method on the same B-preconditioned system (``krylov="lanczos"``): the
  Lanczos basis v_1 = r_0 / |r_0|, ..., the tridiagonal T_j of its
  recurrence coefficients, x_j = V_j y_j with T_j y_j = |r_0| e_1, whose
  residual norm is beta_{j+1} |e_j^T y_j|; same caps and stop tests (T_j
  not positive definite ends it at x_{j-1}).  It reaches the CG iterates in
  exact arithmetic and also yields the Ritz values (eigenvalues of T_j) of
  the preconditioned normal matrix;
* the Gauss-Newton update u^{l+1} = u^l + delta u^l of Alg. 5 is taken in
  full (no line search), and the iteration stops after ``max_iter`` updates
  or when |V grad J_s| <= grad_rtol |V grad J_s(u^0)|, tested before each
  update.
"""
from __future__ import annotations

import numpy as np

from . import local
from .model import Grid


def residual_weights(prob, maps, s):
    """Diagonal W over the local trajectory [nlev][3][ny][nx] of subdomain s."""
    b = maps.boxes[s]
    W = np.zeros((b.nlev, 3, b.ny * b.nx))
    _, csp = local.weights(prob, maps, s)
    idx = maps.obs_bin[s]
    if idx.size:
        st = prob.obs_step[idx].astype(np.int64)
        cell = prob.obs_cell[idx].astype(np.int64)
        fld = prob.obs_field[idx].astype(np.int64)
        loc = maps.box_index(b, cell // prob.nlon, cell % prob.nlon)
        if prob.weight_mode == 1:
            wo = np.ones(idx.size)
        else:
            wo = 1.0 / (csp[loc] * maps.time_count[st])
        np.add.at(W, (st - b.lev0, fld, loc), prob.lambda_obs * wo / prob.obs_sigma[idx] ** 2)
    gr, gc = maps.box_cells_global(b)
    isb2 = 1.0 / prob.sigma_b ** 2
    for sp in maps.neighbors[s]:
        bp = maps.boxes[int(sp)]
        lo = max(b.lev0, bp.lev0)
        hi = min(b.lev0 + b.nlev, bp.lev0 + bp.nlev)
        mine = np.nonzero(maps.box_index(bp, gr, gc) >= 0)[0]
        if lo >= hi or mine.size == 0:
            continue
        W[lo - b.lev0:hi - b.lev0, :, mine] += (prob.mu_overlap * isb2)[None, :, None]
    return W.reshape(b.nlev, 3, b.ny, b.nx)


def background_weight(prob, maps, s):
    """Diagonal B_w^{-1} over the control [3][ny][nx]."""
    b = maps.boxes[s]
    wb, _ = local.weights(prob, maps, s)
    return wb.reshape(1, b.ny, b.nx) / (prob.sigma_b ** 2)[:, None, None]


def hessvec(prob, maps, s, traj, ring, dx, W=None, dtype=np.float64):
    """A(x) dx with A the Gauss-Newton normal matrix about the local
    trajectory ``traj`` of x (eq. line5and7).  ``dtype`` np.longdouble runs
    the same steps in extended precision."""
    g = Grid.of(prob, dtype)
    geo = local.LocalGeometry(g, maps, s)
    if W is None:
        W = residual_weights(prob, maps, s)
    dz = local.tlm(geo, traj, ring, dx)
    return background_weight(prob, maps, s) * dx + local.adjoint(geo, traj, ring, W * dz)


def cg(apply, b, max_iter, rtol):
    """Conjugate gradients for apply(x) = b from x = 0.  Returns (x, iters)."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(np.dot(r, r))
    r0 = np.sqrt(rr)
    k = 0
    while k < max_iter and np.sqrt(rr) > rtol * r0:
        q = apply(p)
        pq = float(np.dot(p, q))
        if not pq > 0.0:
            break
        a = rr / pq
        x = x + a * p
        r = r - a * q
        rn = float(np.dot(r, r))
        p = r + (rn / rr) * p
        rr = rn
        k += 1
    return x, k


def _tridiag_solve(a, b, rhs):
    """Solve the symmetric tridiagonal system (diagonal a, off-diagonal b) by
    its LDL^T factorization; None if a pivot is not positive."""
    n = len(a)
    d = np.empty(n)
    lo = np.empty(max(n - 1, 0))
    z = np.empty(n)
    for i in range(n):
        d[i] = a[i] - (lo[i - 1] ** 2 * d[i - 1] if i > 0 else 0.0)
        if not d[i] > 0.0:
            return None
        if i < n - 1:
            lo[i] = b[i] / d[i]
        z[i] = rhs[i] - (lo[i - 1] * z[i - 1] if i > 0 else 0.0)
    y = np.empty(n)
    for i in range(n - 1, -1, -1):
        y[i] = z[i] / d[i] - (lo[i] * y[i + 1] if i < n - 1 else 0.0)
    return y


def lanczos(apply, b, max_iter, rtol):
    """Lanczos method for apply(x) = b (symmetric positive definite) from
    x = 0.  Returns (x, iters, alpha, beta): x = V_j y_j after j = iters
    products, and the recurrence coefficients of T_j (diagonal alpha[:j],
    off-diagonal beta[1:j]; beta[0] = |b|)."""
    beta0 = float(np.linalg.norm(b))
    alpha, beta = [], [beta0]
    if max_iter <= 0 or not beta0 > 0.0 or not beta0 > rtol * beta0:
        return np.zeros_like(b), 0, np.array(alpha), np.array(beta)
    V = [b / beta0]
    y = None
    j = 0
    while j < max_iter:
        w = apply(V[j])
        if j > 0:
            w = w - beta[j] * V[j - 1]
        a = float(np.dot(w, V[j]))
        w = w - a * V[j]
        bn = float(np.linalg.norm(w))
        yn = _tridiag_solve(alpha + [a], beta[1:j + 1], np.eye(j + 1)[0] * beta0)
        if yn is None:
            break
        alpha.append(a)
        beta.append(bn)
        y = yn
        j += 1
        if bn * abs(y[-1]) <= rtol * beta0 or not bn > 0.0:
            break
        V.append(w / bn)
    x = np.zeros_like(b) if y is None else sum(yi * vi for yi, vi in zip(y, V))
    return x, j, np.array(alpha), np.array(beta)


def ritz_values(alpha, beta):
    """Eigenvalues of T_j (the Ritz values of the Lanczos run)."""
    j = len(alpha)
    T = np.diag(alpha) + np.diag(beta[1:j], 1) + np.diag(beta[1:j], -1)
    return np.linalg.eigvalsh(T)


def minimize(prob, maps, s, x0, xb, ring, nbr_trajs, max_iter=5, grad_rtol=0.0,
             cg_max_iter=50, cg_rtol=1e-6, krylov="cg"):
    """Gauss-Newton iterations on J_s from x0 (Alg. 5 with the normal
    equations solved as above).  Returns a dict like ``lbfgs.minimize``."""
    g = Grid.of(prob)
    geo = local.LocalGeometry(g, maps, s)
    sb = prob.sigma_b[:, None, None] * np.ones_like(x0)
    W = residual_weights(prob, maps, s)
    # iterate held in xi = (x - x^b) / sigma_b, as the normal equations are
    xi_it = (np.asarray(x0, dtype=np.float64) - xb) / sb
    x = xb + sb * xi_it
    J, gr = local.cost_grad(prob, maps, s, x, xb, ring, nbr_trajs)
    g0 = float(np.linalg.norm(sb * gr))
    gn = g0
    hist = [J]
    it = 0
    cg_total = 0
    ritz = np.zeros(0)     # Ritz values of the last Lanczos run with a product
    status = "max_iter"
    while it < max_iter:
        if gn <= grad_rtol * g0:
            status = "converged"
            break
        traj = local.forward(geo, x, ring)

        def apply(v):
            return (sb * hessvec(prob, maps, s, traj, ring, (sb * v.reshape(x.shape)), W)).ravel()

        if krylov == "lanczos":
            xi, k, al, be = lanczos(apply, -(sb * gr).ravel(), cg_max_iter, cg_rtol)
            if k:
                ritz = ritz_values(al, be)
        else:
            xi, k = cg(apply, -(sb * gr).ravel(), cg_max_iter, cg_rtol)
        cg_total += k
        xi_it = xi_it + xi.reshape(x.shape)
        x = xb + sb * xi_it
        J, gr = local.cost_grad(prob, maps, s, x, xb, ring, nbr_trajs)
        gn = float(np.linalg.norm(sb * gr))
        hist.append(J)
        it += 1
    return dict(x=x, xi=xi_it, J=J, grad=gr, iters=it, cg_iters=cg_total, nfev=it + 1, status=status,
                history=hist, g0norm=g0, gnorm=gn, ritz=ritz)
