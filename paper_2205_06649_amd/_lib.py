"""ctypes binding of libdd4dvar.so: the C ABI of include/dd4dvar.h, same names.

Argument marshalling only; every step of the computation runs in the
library's HIP kernels.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdd4dvar.so")

DD4DVAR_OK = 0
DD4DVAR_E_INVALID = 1
DD4DVAR_E_NOMEM = 2
DD4DVAR_E_DEVICE = 3
DD4DVAR_E_NONFINITE = 4
DD4DVAR_E_NOTCONVERGED = 5
DD4DVAR_E_STATE = 6
STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_NOMEM", 3: "E_DEVICE", 4: "E_NONFINITE",
                5: "E_NOTCONVERGED", 6: "E_STATE"}

DD4DVAR_FP64 = 0
DD4DVAR_FP32_STATE = 1

MAP_HALO_SRC, MAP_HALO_OFF, MAP_HALO_SIGN, MAP_COVER, MAP_TIME_COUNT, MAP_NEIGHBORS, \
    MAP_OBS_BIN, MAP_HALO_GCELL = range(8)


class dd4dvar_model_desc(C.Structure):
    _fields_ = [("nlat", C.c_int32), ("nlon", C.c_int32), ("nsteps", C.c_int32),
                ("dt", C.c_double), ("radius", C.c_double), ("gravity", C.c_double),
                ("omega", C.c_double), ("h_ref", C.c_double),
                ("lambda_obs", C.c_double), ("mu_overlap", C.c_double),
                ("precision", C.c_int32), ("weight_mode", C.c_int32),
                ("tz_p", C.c_int32), ("tz_q", C.c_int32), ("tz_alpha", C.c_double)]


class dd4dvar_partition_desc(C.Structure):
    _fields_ = [("n_bands", C.c_int32), ("band_lat_edges", C.POINTER(C.c_int32)),
                ("band_npieces", C.POINTER(C.c_int32)),
                ("piece_lon_edges", C.POINTER(C.c_int32)),
                ("n_time", C.c_int32), ("time_edges", C.POINTER(C.c_int32)),
                ("overlap_cells", C.c_int32), ("overlap_steps", C.c_int32)]


class dd4dvar_data_desc(C.Structure):
    _fields_ = [("xb0", C.POINTER(C.c_double)), ("sigma_b", C.POINTER(C.c_double)),
                ("nobs", C.c_int64), ("obs_step", C.POINTER(C.c_int32)),
                ("obs_cell", C.POINTER(C.c_int32)), ("obs_field", C.POINTER(C.c_int8)),
                ("obs_value", C.POINTER(C.c_double)), ("obs_sigma", C.POINTER(C.c_double))]


class dd4dvar_solve_opts(C.Structure):
    _fields_ = [("lbfgs_m", C.c_int32), ("max_iter", C.c_int32), ("max_outer", C.c_int32),
                ("max_ls", C.c_int32), ("grad_rtol", C.c_double), ("outer_tol", C.c_double),
                ("armijo_c1", C.c_double), ("j_noise_rtol", C.c_double),
                ("local_solver", C.c_int32), ("cg_max_iter", C.c_int32), ("cg_rtol", C.c_double),
                ("krylov", C.c_int32)]


class dd4dvar_solve_report(C.Structure):
    _fields_ = [("outer_iters", C.c_int32), ("total_evals", C.c_int32),
                ("lbfgs_iters", C.c_int32), ("gn_products", C.c_int32), ("J_final", C.c_double),
                ("gnorm_ratio_max", C.c_double), ("seconds", C.c_double),
                ("ritz_min", C.c_double), ("ritz_max", C.c_double)]


class dd4dvar_tune_report(C.Structure):
    _fields_ = [("ncand", C.c_int32), ("mode", C.c_int32 * 8), ("passes", C.c_int32 * 8),
                ("ms", C.c_double * 8), ("chosen", C.c_int32)]


_VP = C.c_void_p
_SIGS = {
    "dd4dvar_plan_create": (C.c_int, [C.POINTER(dd4dvar_model_desc), C.POINTER(dd4dvar_partition_desc),
                                      C.POINTER(dd4dvar_data_desc), C.POINTER(_VP)]),
    "dd4dvar_plan_destroy": (None, [_VP]),
    "dd4dvar_plan_sizes": (C.c_int, [_VP, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64)]),
    "dd4dvar_plan_subdomain_info": (C.c_int, [_VP, C.c_int32, C.POINTER(C.c_int64)]),
    "dd4dvar_plan_get_map": (C.c_int, [_VP, C.c_int32, C.c_int32, C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int32)]),
    "dd4dvar_last_error": (C.c_char_p, [_VP]),
    "dd4dvar_create": (C.c_int, [C.POINTER(dd4dvar_model_desc), C.POINTER(dd4dvar_partition_desc),
                                 C.POINTER(dd4dvar_data_desc), _VP, C.POINTER(_VP)]),
    "dd4dvar_destroy": (None, [_VP]),
    "dd4dvar_ctx_plan": (_VP, [_VP]),
    "dd4dvar_background_controls": (C.c_int, [_VP, _VP, _VP]),
    "dd4dvar_local_cost_grad": (C.c_int, [_VP, C.c_int32, C.POINTER(C.c_int32), _VP, _VP, _VP, _VP]),
    "dd4dvar_local_cost_grad_noalloc": (C.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "dd4dvar_forward_integrate": (C.c_int, [_VP, C.c_int32, _VP, _VP, _VP]),
    "dd4dvar_adjoint_integrate": (C.c_int, [_VP, C.c_int32, _VP, _VP, _VP]),
    "dd4dvar_tangent_linear": (C.c_int, [_VP, _VP, _VP, _VP]),
    "dd4dvar_gn_hessvec": (C.c_int, [_VP, _VP, _VP, _VP]),
    "dd4dvar_exchange": (C.c_int, [_VP, _VP, _VP]),
    "dd4dvar_gather": (C.c_int, [_VP, C.c_int32, _VP, _VP]),
    "dd4dvar_set_exec_mode": (C.c_int, [_VP, C.c_int32]),
    "dd4dvar_set_exec_plan": (C.c_int, [_VP, C.c_int32, C.c_int32]),
    "dd4dvar_get_exec_plan": (C.c_int, [_VP, C.POINTER(C.c_int32)]),
    "dd4dvar_set_tz_kernels": (C.c_int, [_VP, C.c_int32]),
    "dd4dvar_get_tz_kernels": (C.c_int, [_VP, C.POINTER(C.c_int32)]),
    "dd4dvar_set_solver_parts": (C.c_int, [_VP, C.c_int32]),
    "dd4dvar_get_solver_parts": (C.c_int, [_VP, C.POINTER(C.c_int32)]),
    "dd4dvar_synchronize": (C.c_int, [_VP, _VP]),
    "dd4dvar_set_timing": (C.c_int, [_VP, C.c_int32]),
    "dd4dvar_set_graph": (C.c_int, [_VP, C.c_int32]),
    "dd4dvar_set_checkpointing": (C.c_int, [_VP, C.c_int32, C.POINTER(C.c_int64)]),
    "dd4dvar_autotune": (C.c_int, [_VP, _VP, _VP, _VP, C.c_int32, _VP, C.POINTER(dd4dvar_tune_report)]),
    "dd4dvar_get_timing": (C.c_int, [_VP, C.POINTER(C.c_double)]),
    "dd4dvar_solve": (C.c_int, [_VP, C.POINTER(dd4dvar_solve_opts), _VP, _VP, _VP,
                                C.POINTER(dd4dvar_solve_report)]),
    "dd4dvar_solve_mixed": (C.c_int, [_VP, _VP, C.POINTER(dd4dvar_solve_opts), _VP, _VP, _VP,
                                      C.POINTER(dd4dvar_solve_report)]),
}

_lib = None


def lib():
    """Load libdd4dvar.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built: run python -m paper_2205_06649_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_names():
    return list(_SIGS)


class DD4DVarError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status, ctx=None):
    if status != DD4DVAR_OK:
        m = lib().dd4dvar_last_error(ctx)
        raise DD4DVarError(status, m.decode() if m else "")
    return status


def _ptr(arr, ctype):
    return arr.ctypes.data_as(C.POINTER(ctype))


# ---- same-name wrappers -------------------------------------------------------
def dd4dvar_plan_create(model, part, data):
    out = _VP()
    st = lib().dd4dvar_plan_create(C.byref(model), C.byref(part), C.byref(data), C.byref(out))
    check(st)
    return out


def dd4dvar_plan_destroy(plan):
    lib().dd4dvar_plan_destroy(plan)


def dd4dvar_plan_sizes(plan):
    n = C.c_int32()
    a = C.c_int64()
    b = C.c_int64()
    check(lib().dd4dvar_plan_sizes(plan, C.byref(n), C.byref(a), C.byref(b)))
    return n.value, a.value, b.value


def dd4dvar_plan_subdomain_info(plan, s):
    out = (C.c_int64 * 10)()
    check(lib().dd4dvar_plan_subdomain_info(plan, s, out))
    return list(out)


def dd4dvar_plan_get_map(plan, kind, s):
    import numpy as np
    n = C.c_int64(0)
    check(lib().dd4dvar_plan_get_map(plan, kind, s, C.byref(n), None))
    buf = np.empty(n.value, dtype=np.int32)
    check(lib().dd4dvar_plan_get_map(plan, kind, s, C.byref(n), _ptr(buf, C.c_int32)))
    return buf


def dd4dvar_last_error(ctx=None):
    m = lib().dd4dvar_last_error(ctx)
    return m.decode() if m else ""


def dd4dvar_create(model, part, data, stream=None):
    out = _VP()
    st = lib().dd4dvar_create(C.byref(model), C.byref(part), C.byref(data), stream, C.byref(out))
    check(st)
    return out


def dd4dvar_destroy(ctx):
    lib().dd4dvar_destroy(ctx)


def dd4dvar_ctx_plan(ctx):
    return lib().dd4dvar_ctx_plan(ctx)


def dd4dvar_background_controls(ctx, x_dev, stream=None):
    check(lib().dd4dvar_background_controls(ctx, x_dev, stream), ctx)


def dd4dvar_local_cost_grad(ctx, x_dev, J_dev, grad_dev, stream=None, sub_ids=None):
    if sub_ids is None:
        st = lib().dd4dvar_local_cost_grad(ctx, 0, None, x_dev, J_dev, grad_dev, stream)
    else:
        import numpy as np
        ids = np.ascontiguousarray(sub_ids, dtype=np.int32)
        st = lib().dd4dvar_local_cost_grad(ctx, int(ids.size), _ptr(ids, C.c_int32), x_dev, J_dev,
                                           grad_dev, stream)
    check(st, ctx)


def dd4dvar_local_cost_grad_noalloc(ctx, x_dev, J_dev, grad_dev, stream=None):
    check(lib().dd4dvar_local_cost_grad_noalloc(ctx, x_dev, J_dev, grad_dev, stream), ctx)


def dd4dvar_forward_integrate(ctx, scope, x_dev, traj_dev, stream=None):
    check(lib().dd4dvar_forward_integrate(ctx, scope, x_dev, traj_dev, stream), ctx)


def dd4dvar_adjoint_integrate(ctx, scope, forcing_dev, adj0_dev, stream=None):
    check(lib().dd4dvar_adjoint_integrate(ctx, scope, forcing_dev, adj0_dev, stream), ctx)


def dd4dvar_tangent_linear(ctx, dx_dev, dtraj_dev, stream=None):
    check(lib().dd4dvar_tangent_linear(ctx, dx_dev, dtraj_dev, stream), ctx)


def dd4dvar_gn_hessvec(ctx, dx_dev, out_dev, stream=None):
    check(lib().dd4dvar_gn_hessvec(ctx, dx_dev, out_dev, stream), ctx)


def dd4dvar_exchange(ctx, x_dev, stream=None):
    check(lib().dd4dvar_exchange(ctx, x_dev, stream), ctx)


def dd4dvar_gather(ctx, level, out_dev, stream=None):
    check(lib().dd4dvar_gather(ctx, level, out_dev, stream), ctx)


def dd4dvar_set_exec_mode(ctx, mode):
    check(lib().dd4dvar_set_exec_mode(ctx, mode), ctx)


def dd4dvar_set_exec_plan(ctx, mode, passes):
    check(lib().dd4dvar_set_exec_plan(ctx, mode, passes), ctx)


def dd4dvar_get_exec_plan(ctx):
    out = (C.c_int32 * 4)()
    check(lib().dd4dvar_get_exec_plan(ctx, out), ctx)
    return {"mode": out[0], "passes": out[1], "strip_rows": out[2], "persistent": bool(out[3])}


def dd4dvar_set_tz_kernels(ctx, kind):
    check(lib().dd4dvar_set_tz_kernels(ctx, kind), ctx)


def dd4dvar_get_tz_kernels(ctx):
    out = (C.c_int32 * 2)()
    check(lib().dd4dvar_get_tz_kernels(ctx, out), ctx)
    return {"kind": out[0], "column_walk_applies": out[1] >= 1, "max_kind": out[1]}


def dd4dvar_set_solver_parts(ctx, entries):
    check(lib().dd4dvar_set_solver_parts(ctx, entries), ctx)


def dd4dvar_get_solver_parts(ctx):
    out = (C.c_int32 * 2)()
    check(lib().dd4dvar_get_solver_parts(ctx, out), ctx)
    return {"entries": out[0], "parts": out[1]}


def dd4dvar_synchronize(ctx, stream=None):
    check(lib().dd4dvar_synchronize(ctx, stream), ctx)


def dd4dvar_set_timing(ctx, on):
    check(lib().dd4dvar_set_timing(ctx, int(bool(on))), ctx)


def dd4dvar_set_checkpointing(ctx, stride):
    nbytes = C.c_int64(0)
    check(lib().dd4dvar_set_checkpointing(ctx, stride, C.byref(nbytes)), ctx)
    return nbytes.value


def dd4dvar_set_graph(ctx, on):
    check(lib().dd4dvar_set_graph(ctx, int(bool(on))), ctx)


def dd4dvar_autotune(ctx, x_dev, J_dev, grad_dev, reps, stream=None):
    rep = dd4dvar_tune_report()
    check(lib().dd4dvar_autotune(ctx, x_dev, J_dev, grad_dev, reps, stream, C.byref(rep)), ctx)
    n = rep.ncand
    return {"candidates": [{"mode": rep.mode[i], "passes": rep.passes[i], "ms": rep.ms[i]}
                           for i in range(n)],
            "chosen": rep.chosen}


def dd4dvar_get_timing(ctx):
    out = (C.c_double * 6)()
    check(lib().dd4dvar_get_timing(ctx, out), ctx)
    keys = ("fwd_ms", "adj_ms", "reduce_ms", "fwd_launches", "adj_launches", "calls")
    return dict(zip(keys, list(out)))


def dd4dvar_solve(ctx, opts, x_init_dev, x_out_dev, xa_host):
    rep = dd4dvar_solve_report()
    st = lib().dd4dvar_solve(ctx, C.byref(opts), x_init_dev, x_out_dev,
                             _ptr(xa_host, C.c_double), C.byref(rep))
    if st not in (DD4DVAR_OK, DD4DVAR_E_NOTCONVERGED):
        check(st, ctx)
    return st, rep


def dd4dvar_solve_mixed(ctx, ctx_lo, opts, x_init_dev, x_out_dev, xa_host):
    rep = dd4dvar_solve_report()
    st = lib().dd4dvar_solve_mixed(ctx, ctx_lo, C.byref(opts), x_init_dev, x_out_dev,
                                   _ptr(xa_host, C.c_double), C.byref(rep))
    if st not in (DD4DVAR_OK, DD4DVAR_E_NOTCONVERGED):
        check(st, ctx)
    return st, rep
