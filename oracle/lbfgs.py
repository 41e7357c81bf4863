"""Limited-memory BFGS with Armijo backtracking (FP64).

Test infrastructure only (see the package docstring).

The paper names L-BFGS as the quasi-Newton variant of the local Newton step
(remark after Alg. 5: the Hessian is updated by low-rank corrections at every
iteration) and runs the local minimizations with L-BFGS codes on both of its
platforms.  Readings: m stored pairs with the initial inverse Hessian gamma*I,
gamma = s^T y / y^T y of the newest pair (1 before any pair exists); the
search direction comes from the standard two-loop recursion; the step starts
at 1 and is halved until the Armijo condition J(x + a d) <= J(x) + c1 a g^T d
holds (at most ``max_ls`` trials); a pair is skipped when
s^T y <= 1e-12 |s| |y|; iteration stops at ``max_iter`` accepted steps or when
|g| <= grad_rtol |g_0|.
"""
from __future__ import annotations

import numpy as np


def two_loop(g, pairs):
    q = g.copy()
    alphas = []
    for s, y in reversed(pairs):
        rho = 1.0 / np.dot(y, s)
        a = rho * np.dot(s, q)
        q -= a * y
        alphas.append(a)
    if pairs:
        s, y = pairs[-1]
        gamma = np.dot(s, y) / np.dot(y, y)
    else:
        gamma = 1.0
    r = gamma * q
    for (s, y), a in zip(pairs, reversed(alphas)):
        rho = 1.0 / np.dot(y, s)
        b = rho * np.dot(y, r)
        r += s * (a - b)
    return -r


def minimize(fun, x0, m=8, max_iter=50, grad_rtol=0.0, c1=1e-4, max_ls=30):
    """Minimize fun(x) -> (J, grad) from x0 (1-D arrays).  Returns a dict."""
    x = np.array(x0, dtype=np.float64, copy=True)
    J, g = fun(x)
    g0 = float(np.linalg.norm(g))
    pairs = []
    hist = [J]
    nfev = 1
    status = "max_iter"
    it = 0
    while it < max_iter:
        if np.linalg.norm(g) <= grad_rtol * g0:
            status = "converged"
            break
        d = two_loop(g, pairs)
        gd = float(np.dot(g, d))
        if not gd < 0.0:
            d = -g
            gd = -float(np.dot(g, g))
        alpha = 1.0
        ok = False
        for _ in range(max_ls):
            xn = x + alpha * d
            Jn, gn = fun(xn)
            nfev += 1
            if Jn <= J + c1 * alpha * gd:
                ok = True
                break
            alpha *= 0.5
        if not ok:
            status = "line_search_failed"
            break
        s = xn - x
        y = gn - g
        sy = float(np.dot(s, y))
        if sy > 1e-12 * np.linalg.norm(s) * np.linalg.norm(y):
            pairs.append((s, y))
            if len(pairs) > m:
                pairs.pop(0)
        x, J, g = xn, Jn, gn
        hist.append(J)
        it += 1
    else:
        if np.linalg.norm(g) <= grad_rtol * g0:
            status = "converged"
    return dict(x=x, J=J, grad=g, iters=it, nfev=nfev, status=status,
                gnorm0=g0, gnorm=float(np.linalg.norm(g)), history=hist)
