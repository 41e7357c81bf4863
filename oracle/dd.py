"""Alg. 1 (DD-4DVar) on the CPU: background run, local solves, exchange, gather.

Test infrastructure only (see the package docstring).

Steps, in the order of Alg. 1:

1. run the model from the background initial state over the whole window
   (the global background trajectory u^b);
2. set every local control to the background at its first level S_j and take
   the halo rings and overlap targets from the background trajectory;
3. repeat: minimize every local functional independently (L-BFGS in the
   variables xi = (x - x^b_s) / sigma_b, i.e. the diagonal special case of the
   B = V V^T preconditioning of eqs. EqV, Eq_matrixAV), integrate each new
   control over its interval, then exchange: rings and targets are refreshed
   from the new local trajectories; stop when max_s |xi_s^l - xi_s^{l-1}|_inf
   is below ``outer_tol`` or after ``max_outer`` sweeps;
4. gather (reading of the garbled last line of Alg. 1): the partition of
   unity of eq. rest, A^n(cell) = sum_s Z_s^n(cell) / c(n, cell); the analysis
   is the level-0 field.
"""
from __future__ import annotations

import numpy as np

from . import ddmaps as ddm
from . import gn
from . import lbfgs
from . import local
from . import model


def background(prob, maps, dtype=np.float64):
    """Global background run from x_b0 and every box's restriction of it.

    ``dtype`` np.longdouble runs the same steps in extended precision from the
    same FP64 initial state (a reference for FP64 evaluations: the observation
    and overlap residuals are differences of nearly equal depths, so the
    rounding of an FP64 run reaches the gradient amplified)."""
    g = model.Grid.of(prob, dtype)
    bg = model.forward(g, np.asarray(prob.xb0, dtype), prob.nsteps)
    trajs = {b.sub: local.restrict_global(maps, b.sub, bg) for b in maps.boxes}
    return bg, trajs


def local_forward_all(prob, maps, xs, rings):
    g = model.Grid.of(prob)
    out = {}
    for b in maps.boxes:
        geo = local.LocalGeometry(g, maps, b.sub)
        out[b.sub] = local.forward(geo, xs[b.sub], rings[b.sub])
    return out


def exchange(maps, trajs):
    """Rings and targets for every subdomain from the current trajectories."""
    rings = {b.sub: local.ring_from_trajs(maps, b.sub, trajs) for b in maps.boxes}
    return rings, trajs


def gather(prob, maps, trajs, level=0):
    """Partition-of-unity assembly of the local fields at one global level."""
    acc = np.zeros((3, prob.nlat, prob.nlon))
    cnt = np.zeros((prob.nlat, prob.nlon))
    for b in maps.boxes:
        if not (b.lev0 <= level <= b.lev0 + b.nlev - 1):
            continue
        rows = b.row0 + np.arange(b.ny)
        cols = (b.col0 + np.arange(b.nx)) % prob.nlon
        Z = trajs[b.sub][level - b.lev0]
        acc[:, rows[:, None], cols[None, :]] += Z
        cnt[rows[:, None], cols[None, :]] += 1.0
    return acc / cnt


def solve(prob, maps=None, max_outer=5, outer_tol=1e-6, lbfgs_m=8, max_iter=50,
          grad_rtol=0.0, max_ls=30, c1=1e-4, verbose=False, local_solver="lbfgs",
          cg_max_iter=50, cg_rtol=1e-6, krylov="cg"):
    """Alg. 1.  ``local_solver`` "lbfgs" (the default) or "gn": Gauss-Newton
    (Alg. 5 / Alg. 6, see ``gn``) with ``max_iter`` updates per local solve and
    ``krylov`` "cg" (conjugate gradients) or "lanczos" (Alg. 7) runs of at most
    ``cg_max_iter`` products."""
    if maps is None:
        maps = ddm.build(prob)
    bg, trajs = background(prob, maps)
    xb = {s: trajs[s][0].copy() for s in trajs}
    xs = {s: trajs[s][0].copy() for s in trajs}
    rings, targets = exchange(maps, trajs)
    sb = prob.sigma_b[:, None, None]
    report = dict(outer=0, evals=0, history=[])
    ritz_last = {}     # per subdomain: extreme Ritz values of its last Lanczos run
    for outer in range(1, max_outer + 1):
        new_xs = {}
        step = 0.0
        for b in maps.boxes:
            s = b.sub
            shape = xs[s].shape

            def fun(xi, s=s, shape=shape):
                xx = xb[s] + sb * xi.reshape(shape)
                J, gr = local.cost_grad(prob, maps, s, xx, xb[s], rings[s],
                                        {k: targets[k] for k in maps.neighbors[s]})
                return J, (sb * gr).ravel()

            xi0 = ((xs[s] - xb[s]) / sb).ravel()
            if local_solver == "gn":
                res = gn.minimize(prob, maps, s, xs[s], xb[s], rings[s],
                                  {k: targets[k] for k in maps.neighbors[s]}, max_iter=max_iter,
                                  grad_rtol=grad_rtol, cg_max_iter=cg_max_iter, cg_rtol=cg_rtol,
                                  krylov=krylov)
                res["x"] = res["xi"].ravel()
                report["cg_iters"] = report.get("cg_iters", 0) + res["cg_iters"]
                if res["ritz"].size:
                    ritz_last[s] = (float(res["ritz"].min()), float(res["ritz"].max()))
            else:
                res = lbfgs.minimize(fun, xi0, m=lbfgs_m, max_iter=max_iter,
                                     grad_rtol=grad_rtol, c1=c1, max_ls=max_ls)
            report["evals"] += res["nfev"]
            new_xs[s] = xb[s] + sb * res["x"].reshape(shape)
            step = max(step, float(np.max(np.abs(res["x"] - xi0))))
            report["history"].append((outer, s, res["J"], res["iters"], res["status"]))
        xs = new_xs
        trajs = local_forward_all(prob, maps, xs, rings)
        rings, targets = exchange(maps, trajs)
        report["outer"] = outer
        if verbose:
            print(f"outer {outer}: max |dxi| = {step:.3e}")
        if step < outer_tol:
            break
    xa = gather(prob, maps, trajs, 0)
    if ritz_last:
        report["ritz_min"] = min(v[0] for v in ritz_last.values())
        report["ritz_max"] = max(v[1] for v in ritz_last.values())
    return xa, dict(report, controls=xs, trajs=trajs, background=bg)
