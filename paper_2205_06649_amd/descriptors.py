"""Marshal a problem description into the C ABI descriptor structs.

The problem object needs the attributes of the model, partition and data
descriptors of include/dd4dvar.h (as produced by the ``synth`` generator).
The returned holder keeps the NumPy buffers alive while the structs are used.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


class Descriptors:
    def __init__(self, prob, precision=L.DD4DVAR_FP64):
        self._keep = []

        def arr(a, dtype):
            a = np.ascontiguousarray(a, dtype=dtype)
            self._keep.append(a)
            return a

        self.model = L.dd4dvar_model_desc(
            nlat=prob.nlat, nlon=prob.nlon, nsteps=prob.nsteps, dt=prob.dt,
            radius=prob.radius, gravity=prob.gravity, omega=prob.omega, h_ref=prob.h_ref,
            lambda_obs=prob.lambda_obs, mu_overlap=prob.mu_overlap,
            precision=int(precision), weight_mode=int(prob.weight_mode),
            tz_p=int(getattr(prob, "tz_p", 0)), tz_q=int(getattr(prob, "tz_q", 1)),
            tz_alpha=float(getattr(prob, "tz_alpha", 0.0)))
        be = arr(prob.band_lat_edges, np.int32)
        bn = arr(prob.band_npieces, np.int32)
        pe = arr(prob.piece_lon_edges, np.int32)
        te = arr(prob.time_edges, np.int32)
        self.part = L.dd4dvar_partition_desc(
            n_bands=int(bn.size), band_lat_edges=be.ctypes.data_as(C.POINTER(C.c_int32)),
            band_npieces=bn.ctypes.data_as(C.POINTER(C.c_int32)),
            piece_lon_edges=pe.ctypes.data_as(C.POINTER(C.c_int32)),
            n_time=int(te.size - 1), time_edges=te.ctypes.data_as(C.POINTER(C.c_int32)),
            overlap_cells=int(prob.overlap_cells), overlap_steps=int(prob.overlap_steps))
        xb = arr(prob.xb0, np.float64)
        sb = arr(prob.sigma_b, np.float64)
        st = arr(prob.obs_step, np.int32)
        ce = arr(prob.obs_cell, np.int32)
        fi = arr(prob.obs_field, np.int8)
        va = arr(prob.obs_value, np.float64)
        si = arr(prob.obs_sigma, np.float64)
        self.data = L.dd4dvar_data_desc(
            xb0=xb.ctypes.data_as(C.POINTER(C.c_double)),
            sigma_b=sb.ctypes.data_as(C.POINTER(C.c_double)), nobs=int(st.size),
            obs_step=st.ctypes.data_as(C.POINTER(C.c_int32)),
            obs_cell=ce.ctypes.data_as(C.POINTER(C.c_int32)),
            obs_field=fi.ctypes.data_as(C.POINTER(C.c_int8)),
            obs_value=va.ctypes.data_as(C.POINTER(C.c_double)),
            obs_sigma=si.ctypes.data_as(C.POINTER(C.c_double)))


class Plan:
    """Host-only plan (maps) of a problem; no GPU needed."""

    def __init__(self, prob, precision=L.DD4DVAR_FP64):
        self.desc = Descriptors(prob, precision)
        self.handle = L.dd4dvar_plan_create(self.desc.model, self.desc.part, self.desc.data)

    def close(self):
        if self.handle:
            L.dd4dvar_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sizes(self):
        return L.dd4dvar_plan_sizes(self.handle)

    def info(self, s):
        return L.dd4dvar_plan_subdomain_info(self.handle, s)

    def map(self, kind, s=0):
        return L.dd4dvar_plan_get_map(self.handle, kind, s)
