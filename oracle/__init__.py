"""Plain FP64 CPU oracle for the space-time DD 4D-Var local cost/gradient.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the CPU-baseline leg of the benchmark may import or call anything here; the
GPU library never does, and shares no code, tables or helpers with it.

Written from the paper (D'Amore, Constantinescu, Carracciuolo, "A scalable
space-time domain decomposition approach for solving large-scale nonlinear
regularized inverse ill-posed problems in 4D variational data assimilation"):

* ``model``   -- SWE on the sphere (Sec. 7, eqs. EquU/EquV/EquH and the
                 unstaggered discrete U, V, H with p = q = 1, alpha = 0) on the
                 global grid, its tangent linear model and its adjoint (the
                 adjoint definition of the DA setup, Sec. 2), and the global
                 4D-Var functional (Def. of the 4D-Var DA problem, eq. min3sec).
* ``ddmaps``  -- the space-time decomposition DD(Delta x Omega) (Def.
                 domdecom), extended boxes with a per-side overlap (eqs. Eq-r,
                 nlocx), frozen halo sources, coverage counts (restriction
                 weights, Def. defrestrfun), overlap neighbour sets (eqs. overl,
                 ospatial, otime) and observation bins.
* ``local``   -- the restricted model on one box with a frozen halo ring
                 (eq. restricted), its TLM and its adjoint in scatter form,
                 and the local functional with overlap regularization
                 (eq. eq:cost:parallel1) and its gradient.
* ``lbfgs``   -- limited-memory BFGS with Armijo backtracking (the L-BFGS
                 variant named in the remark after Alg. 5).
* ``gn``      -- the Gauss-Newton local solver (Alg. 5 / Alg. 6): normal
                 matrix products (eq. line5and7) from the TLM and the adjoint,
                 conjugate gradients in the B^{1/2}-preconditioned variables.
* ``dd``      -- Alg. 1 (DD-4DVar): background run, local solves, exchange,
                 gather.
* ``brute``   -- per-cell pure-Python loops for tiny grids (a pin).

Readings of points the paper leaves open are stated where they are used.
"""
from . import model, ddmaps, local, lbfgs, gn, dd, brute  # noqa: F401
