"""Device context wrapper: torch tensors for device memory and streams.

Thin layer over the C ABI (argument marshalling only).  torch provides the
device buffers and the current HIP stream; every computation runs in
libdd4dvar.so.
"""
from __future__ import annotations

import numpy as np

from . import _lib as L
from .descriptors import Descriptors

PRECISIONS = {"fp64": L.DD4DVAR_FP64, "fp32": L.DD4DVAR_FP32_STATE}


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the dd4dvar engine needs a HIP device")
    return torch


class Context:
    def __init__(self, prob, precision="fp64", device="cuda:0"):
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device)
        self.prob = prob
        self.precision = precision
        torch.cuda.set_device(self.device)
        self.desc = Descriptors(prob, PRECISIONS[precision])
        self.handle = L.dd4dvar_create(self.desc.model, self.desc.part, self.desc.data,
                                       self._stream())
        self.plan = L.dd4dvar_ctx_plan(self.handle)
        self.nsub, self.ctrl_len, self.traj_len = L.dd4dvar_plan_sizes(self.plan)
        self.info = [L.dd4dvar_plan_subdomain_info(self.plan, s) for s in range(self.nsub)]
        # bumped by every call that integrates the local models and so
        # replaces the stored trajectories the adjoint linearizes around
        self.traj_generation = 0
        # bumped by every call that replaces the frozen halo rings and overlap
        # targets (exchange, solve), which the local model itself depends on
        self.ring_generation = 0

    # -- plumbing -----------------------------------------------------------
    def _stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def close(self):
        if getattr(self, "handle", None):
            L.dd4dvar_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self, n):
        return self.torch.empty(int(n), dtype=self.torch.float64, device=self.device)

    @staticmethod
    def ptr(t):
        return None if t is None else t.data_ptr()

    def set_exec_mode(self, mode):
        L.dd4dvar_set_exec_mode(self.handle, mode)

    def set_exec_plan(self, mode, passes=0):
        L.dd4dvar_set_exec_plan(self.handle, mode, passes)

    def exec_plan(self):
        """{mode, passes, strip_rows, persistent} of the plan in use."""
        return L.dd4dvar_get_exec_plan(self.handle)

    def set_tz_kernels(self, kind):
        """Turkel-Zwas forward and adjoint step kernels: 0 gather form,
        1 column walk (q = 2, p <= 8; the default where it applies), 2 the
        column walk with the persistent FP32 forward sweep (no box spanning
        the circle)."""
        L.dd4dvar_set_tz_kernels(self.handle, kind)

    def tz_kernels(self):
        """{kind, column_walk_applies, max_kind} of the Turkel-Zwas step
        kernels (max_kind: the highest kind that applies)."""
        return L.dd4dvar_get_tz_kernels(self.handle)

    def set_solver_parts(self, entries):
        """Entries per part of the local solvers' vector work (default 16384)."""
        L.dd4dvar_set_solver_parts(self.handle, entries)

    def solver_parts(self):
        """{entries, parts} of the local solvers' part map."""
        return L.dd4dvar_get_solver_parts(self.handle)

    def synchronize(self):
        """Wait for the queued work; raises DD4DVarError (E_NONFINITE) if a
        cost or gradient computed since the last check was NaN or Inf."""
        L.dd4dvar_synchronize(self.handle, self._stream())

    def set_checkpointing(self, stride):
        """0: keep every level; stride >= 3: keep checkpoint pairs every
        stride levels and recompute segments in the adjoint.  Returns the
        bytes of the state arena."""
        nbytes = L.dd4dvar_set_checkpointing(self.handle, int(stride))
        self.traj_generation += 1
        return nbytes

    def set_graph(self, on):
        L.dd4dvar_set_graph(self.handle, on)

    def autotune(self, x, reps=5, J=None, grad=None):
        """Time the execution plans of local_cost_grad at x and keep the
        fastest; returns the report (every candidate and the choice)."""
        if J is None:
            J = self.torch.empty(self.nsub, dtype=self.torch.float64, device=self.device)
        if grad is None:
            grad = self.empty(self.ctrl_len)
        rep = L.dd4dvar_autotune(self.handle, x.data_ptr(), J.data_ptr(), grad.data_ptr(), reps,
                                 self._stream())
        self.traj_generation += 1
        return rep

    def set_timing(self, on):
        L.dd4dvar_set_timing(self.handle, on)

    def get_timing(self):
        return L.dd4dvar_get_timing(self.handle)

    # -- C ABI calls --------------------------------------------------------
    def background_controls(self):
        x = self.empty(self.ctrl_len)
        L.dd4dvar_background_controls(self.handle, x.data_ptr(), self._stream())
        return x

    def cost_grad(self, x, J=None, grad=None, sub_ids=None):
        if J is None:
            J = self.torch.full((self.nsub,), float("nan"), dtype=self.torch.float64,
                                device=self.device)
        if grad is None:
            grad = self.torch.zeros(self.ctrl_len, dtype=self.torch.float64, device=self.device)
        L.dd4dvar_local_cost_grad(self.handle, x.data_ptr(), J.data_ptr(), grad.data_ptr(),
                                  self._stream(), sub_ids=sub_ids)
        self.traj_generation += 1
        return J, grad

    def forward(self, x, with_traj=True):
        traj = self.empty(self.traj_len) if with_traj else None
        L.dd4dvar_forward_integrate(self.handle, 1, x.data_ptr(), self.ptr(traj), self._stream())
        self.traj_generation += 1
        return traj

    def forward_global(self, x0):
        p = self.prob
        traj = self.empty((p.nsteps + 1) * 3 * p.nlat * p.nlon)
        L.dd4dvar_forward_integrate(self.handle, 0, x0.data_ptr(), traj.data_ptr(), self._stream())
        return traj.view(p.nsteps + 1, 3, p.nlat, p.nlon)

    def adjoint(self, forcing=None):
        out = self.empty(self.ctrl_len)
        L.dd4dvar_adjoint_integrate(self.handle, 1, self.ptr(forcing), out.data_ptr(),
                                    self._stream())
        return out

    def tangent_linear(self, dx, with_traj=True):
        """dZ = M' dx about the trajectories of the last forward (packed
        FP64 perturbation trajectories, or None)."""
        out = self.empty(self.traj_len) if with_traj else None
        L.dd4dvar_tangent_linear(self.handle, dx.data_ptr(), self.ptr(out), self._stream())
        return out

    def gn_hessvec(self, dx, out=None):
        """(B_w^{-1} + M'^T W M') dx about the trajectories of the last forward."""
        if out is None:
            out = self.empty(self.ctrl_len)
        L.dd4dvar_gn_hessvec(self.handle, dx.data_ptr(), out.data_ptr(), self._stream())
        return out

    def exchange(self, x):
        L.dd4dvar_exchange(self.handle, x.data_ptr(), self._stream())
        self.traj_generation += 1
        self.ring_generation += 1

    def gather(self, level):
        p = self.prob
        out = self.empty(3 * p.nlat * p.nlon)
        L.dd4dvar_gather(self.handle, level, out.data_ptr(), self._stream())
        return out.view(3, p.nlat, p.nlon)

    # noise floor of J used by default: FP32 state sweeps leave ~1e-7
    # relative rounding noise in J; FP64 runs the plain Armijo search
    J_NOISE_RTOL = {"fp64": 0.0, "fp32": 1e-6}

    LOCAL_SOLVERS = {"lbfgs": 0, "gn": 1}
    KRYLOV = {"cg": 0, "lanczos": 1}

    def solve(self, lbfgs_m=8, max_iter=50, max_outer=5, max_ls=30, grad_rtol=0.0,
              outer_tol=1e-6, armijo_c1=1e-4, x_init=None, want_controls=False,
              j_noise_rtol=None, local_solver="lbfgs", cg_max_iter=50, cg_rtol=1e-6,
              products=None, krylov="cg"):
        """Alg. 1.  products: an FP32-state Context of the same problem whose
        sweeps supply the Gauss-Newton normal-matrix products while this
        (FP64) context evaluates J and the gradients (dd4dvar_solve_mixed).
        krylov: "cg" or "lanczos" (Alg. 7) for the Gauss-Newton normal
        equations; the report carries the Lanczos runs' extreme Ritz values."""
        p = self.prob
        if j_noise_rtol is None:
            j_noise_rtol = self.J_NOISE_RTOL[self.precision]
        opts = L.dd4dvar_solve_opts(lbfgs_m=lbfgs_m, max_iter=max_iter, max_outer=max_outer,
                                    max_ls=max_ls, grad_rtol=grad_rtol, outer_tol=outer_tol,
                                    armijo_c1=armijo_c1, j_noise_rtol=j_noise_rtol,
                                    local_solver=self.LOCAL_SOLVERS[local_solver],
                                    cg_max_iter=cg_max_iter, cg_rtol=cg_rtol,
                                    krylov=self.KRYLOV[krylov])
        xa = np.empty((3, p.nlat, p.nlon))
        xo = self.empty(self.ctrl_len) if want_controls else None
        if products is None:
            st, rep = L.dd4dvar_solve(self.handle, opts, self.ptr(x_init), self.ptr(xo), xa)
        else:
            st, rep = L.dd4dvar_solve_mixed(self.handle, products.handle, opts, self.ptr(x_init),
                                            self.ptr(xo), xa)
            products.traj_generation += 1
            products.ring_generation += 1
        self.traj_generation += 1
        self.ring_generation += 1
        return xa, rep, st, xo

    # -- layout helpers (host side) -----------------------------------------
    def unpack_ctrl(self, x):
        a = x.detach().cpu().numpy() if hasattr(x, "detach") else np.asarray(x)
        out = []
        for inf in self.info:
            ny, nx, off = int(inf[1]), int(inf[3]), int(inf[6])
            out.append(a[off:off + 3 * ny * nx].reshape(3, ny, nx))
        return out

    def pack_ctrl(self, parts):
        a = np.empty(self.ctrl_len)
        for inf, v in zip(self.info, parts):
            ny, nx, off = int(inf[1]), int(inf[3]), int(inf[6])
            a[off:off + 3 * ny * nx] = np.asarray(v).ravel()
        return self.torch.from_numpy(a).to(self.device)

    def unpack_traj(self, t):
        a = t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)
        out = []
        for inf in self.info:
            ny, nx, nlev, off = int(inf[1]), int(inf[3]), int(inf[5]), int(inf[7])
            out.append(a[off:off + nlev * 3 * ny * nx].reshape(nlev, 3, ny, nx))
        return out

    def pack_traj(self, parts):
        a = np.empty(self.traj_len)
        for inf, v in zip(self.info, parts):
            ny, nx, nlev, off = int(inf[1]), int(inf[3]), int(inf[5]), int(inf[7])
            a[off:off + nlev * 3 * ny * nx] = np.asarray(v).ravel()
        return self.torch.from_numpy(a).to(self.device)
