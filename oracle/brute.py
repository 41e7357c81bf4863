"""Per-cell pure-Python evaluation of the discrete SWE increment (tiny grids).

Test infrastructure only (see the package docstring).

A second, loop-by-loop transcription of the discrete U, V, H of Sec. 7
(p = q = 1, alpha = 0, same readings as ``model``), indexing neighbours
explicitly.  It exists only to pin the vectorised code.
"""
from __future__ import annotations

import math


def increment_cell(prob, Z, j, i):
    nlat, nlon = prob.nlat, prob.nlon
    a, g, om, dt = prob.radius, prob.gravity, prob.omega, prob.dt
    dth = math.pi / nlat
    dla = 2 * math.pi / nlon
    sl = dt / (a * dla)
    st = dt / (a * dth)

    def lat(jj):
        return -math.pi / 2 + (jj + 0.5) * dth

    def val(f, jj, ii):
        """Field f at row jj (may be -1 or nlat), column ii (any integer)."""
        sign = 1.0
        if jj < 0:
            jj, ii, sign = 0, ii + nlon // 2, -1.0
        elif jj >= nlat:
            jj, ii, sign = nlat - 1, ii + nlon // 2, -1.0
        x = Z[f][jj][ii % nlon]
        return x if f == 0 else sign * x

    def cosrow(jj):
        jj = min(max(jj, 0), nlat - 1)
        return math.cos(lat(jj))

    th = lat(j)
    c = math.cos(th)
    t = math.tan(th)
    fc = 2 * om * math.sin(th)
    h, u, v = val(0, j, i), val(1, j, i), val(2, j, i)
    cor = fc + u * t / a
    U = (-sl * u / c * (val(1, j, i + 1) - val(1, j, i - 1))
         - st * v * (val(1, j + 1, i) - val(1, j - 1, i))
         - sl * g / c * (val(0, j, i + 1) - val(0, j, i - 1))
         + 2 * dt * cor * v)
    V = (-sl * u / c * (val(2, j, i + 1) - val(2, j, i - 1))
         - st * v * (val(2, j + 1, i) - val(2, j - 1, i))
         - st * g * (val(0, j + 1, i) - val(0, j - 1, i))
         - 2 * dt * cor * u)
    H = (-sl / c * (val(0, j, i + 1) * val(1, j, i + 1) - val(0, j, i - 1) * val(1, j, i - 1))
         - st / c * (val(0, j + 1, i) * val(2, j + 1, i) * cosrow(j + 1)
                     - val(0, j - 1, i) * val(2, j - 1, i) * cosrow(j - 1)))
    return H, U, V


def increment(prob, Z):
    out = [[[0.0] * prob.nlon for _ in range(prob.nlat)] for _ in range(3)]
    for j in range(prob.nlat):
        for i in range(prob.nlon):
            H, U, V = increment_cell(prob, Z, j, i)
            out[0][j][i], out[1][j][i], out[2][j][i] = H, U, V
    return out
