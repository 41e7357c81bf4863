"""Host-side checks of the C ABI library (no GPU): symbols, maps, validation.

The planner's integer maps must equal the oracle's maps bit for bit (partition
and halo index maps of the decomposition, Def. domdecom, eqs. Eq-r, nlocx).
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from oracle import ddmaps
from paper_2205_06649_amd import _lib as L
from paper_2205_06649_amd.descriptors import Descriptors, Plan
from test_oracle_pins import MIXED_CFG, SPAN_CFG, TZ_SPACE_CFGS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "dd4dvar.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dd4dvar_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = _header_functions()
    assert len(names) >= 15
    lib = C.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    # the binding wraps every declared entry point under the same name
    assert set(names) == set(L.exported_names())


def _spec(which):
    if which.startswith("tz_"):
        # Turkel-Zwas pads: pieces, spanning bands, bricks, pole-crossing pads
        name, tzv = {"tz_c1": ("c1", (2, 2, 0.5)), "tz_span": ("span", (1, 3, 1.0)),
                     "tz_mixed": ("mixed", (3, 2, 0.25)), "tz_deep": ("deep", (1, 3, 0.5)),
                     "tz_time": ("time", (2, 2, 0.5))}[which]
        cfg = (dict(synth.CONFIGS["c1"], bands=1, pieces=1, overlap_cells=0, index=146)
               if name == "time" else TZ_SPACE_CFGS[name])
        return synth.make_spec(dict(cfg, tz=tzv))
    if which == "span":
        return synth.make_spec(SPAN_CFG)
    if which == "mixed":
        return synth.make_spec(MIXED_CFG)
    return synth.make_spec(which)


def _with_values(p):
    # map checks need no real observation values
    return p.replace(obs_value=np.zeros(p.nobs))


@pytest.mark.parametrize("which", ["tiny1", "tiny2", "small", "c1", "c2", "span", "mixed", "c3",
                                   "tz_c1", "tz_span", "tz_mixed", "tz_deep", "tz_time"])
def test_plan_maps_match_oracle_bitwise(which):
    p = _with_values(_spec(which))
    om = ddmaps.build(p)
    plan = Plan(p)
    nsub, ctrl_len, traj_len = plan.sizes()
    assert nsub == len(om.boxes)
    ctrl = 0
    traj = 0
    for b in om.boxes:
        s = b.sub
        info = plan.info(s)
        assert info == [b.row0, b.ny, b.col0, b.nx, b.lev0, b.nlev, ctrl, traj, int(b.span), b.nring]
        ctrl += 3 * b.ny * b.nx
        traj += b.nlev * 3 * b.ny * b.nx
        assert np.array_equal(plan.map(L.MAP_HALO_SRC, s), om.halo_src[s])
        assert np.array_equal(plan.map(L.MAP_HALO_OFF, s), om.halo_off[s])
        assert np.array_equal(plan.map(L.MAP_HALO_SIGN, s), om.halo_sign[s])
        gr, gc = om.box_cells_global(b)
        assert np.array_equal(plan.map(L.MAP_COVER, s), om.cover_sp[gr, gc])
        assert np.array_equal(plan.map(L.MAP_NEIGHBORS, s), om.neighbors[s])
        assert np.array_equal(plan.map(L.MAP_OBS_BIN, s), om.obs_bin[s])
    assert ctrl == ctrl_len and traj == traj_len
    assert np.array_equal(plan.map(L.MAP_TIME_COUNT), om.time_count)
    plan.close()


def test_plan_c5_shapes():
    p = _with_values(synth.make_spec("c5"))
    plan = Plan(p)
    nsub, ctrl_len, traj_len = plan.sizes()
    assert nsub == 2048
    infos = [plan.info(s) for s in (0, 17, 2047)]
    assert infos[0][1] == 68 and infos[0][3] == 136 and infos[0][5] == 30
    assert infos[1][1] == 72 and infos[1][5] == 30
    assert infos[2][5] == 30
    assert plan.info(300)[5] == 34
    plan.close()


def _bad(p, **kw):
    return p.replace(**kw)


def _time_decomposition(p):
    """The same problem on one band of one piece (boxes covering the sphere)."""
    return p.replace(band_lat_edges=np.array([0, p.nlat], dtype=np.int32),
                     band_npieces=np.array([1], dtype=np.int32),
                     piece_lon_edges=np.array([0, p.nlon], dtype=np.int32), overlap_cells=0)


def test_turkel_zwas_limits_accepted():
    """The largest offsets (nlon/2, nlat/2) and alpha in {0, 1} plan on a time
    decomposition; the plain scheme (tz_p = 0) ignores tz_q and tz_alpha."""
    t = _time_decomposition(_with_values(synth.make_spec("c1")))
    for kw in (dict(tz_p=32, tz_q=16, tz_alpha=1.0), dict(tz_p=1, tz_q=1, tz_alpha=0.0),
               dict(tz_p=0, tz_q=-5, tz_alpha=7.0)):
        Plan(t.replace(**kw)).close()


@pytest.mark.parametrize("case", [
    "odd_nlon", "edges_not_tiling", "overlap_too_big", "sigma_nonpositive", "obs_cell_range",
    "obs_step_range", "duplicate_obs", "nan_obs", "bad_field", "piece_wraps", "time_overlap",
    "tz_pad_wraps", "tz_p_range", "tz_q_range", "tz_q_zero", "tz_alpha_range", "tz_alpha_nan"])
def test_invalid_descriptors_rejected(case):
    p = _with_values(synth.make_spec("c1"))
    if case == "odd_nlon":
        q = p.replace(nlon=63, xb0=p.xb0[:, :, :63])
    elif case == "edges_not_tiling":
        q = p.replace(band_lat_edges=np.array([0, 10, 30], dtype=np.int32))
    elif case == "overlap_too_big":
        q = p.replace(overlap_cells=17)
    elif case == "sigma_nonpositive":
        q = p.replace(sigma_b=np.array([1.0, 0.0, 1.0]))
    elif case == "obs_cell_range":
        c = p.obs_cell.copy()
        c[5] = p.nlat * p.nlon
        q = p.replace(obs_cell=c)
    elif case == "obs_step_range":
        s = p.obs_step.copy()
        s[0] = p.nsteps + 1
        q = p.replace(obs_step=s)
    elif case == "duplicate_obs":
        q = p.replace(obs_step=np.concatenate([p.obs_step, p.obs_step[:1]]),
                      obs_cell=np.concatenate([p.obs_cell, p.obs_cell[:1]]),
                      obs_field=np.concatenate([p.obs_field, p.obs_field[:1]]),
                      obs_value=np.concatenate([p.obs_value, p.obs_value[:1]]),
                      obs_sigma=np.concatenate([p.obs_sigma, p.obs_sigma[:1]]))
    elif case == "nan_obs":
        v = p.obs_value.copy()
        v[3] = np.nan
        q = p.replace(obs_value=v)
    elif case == "bad_field":
        f = p.obs_field.copy()
        f[2] = 3
        q = p.replace(obs_field=f)
    elif case == "piece_wraps":
        q = p.replace(band_npieces=np.array([2, 2], dtype=np.int32),
                      piece_lon_edges=np.array([0, 60, 64, 0, 32, 64], dtype=np.int32),
                      overlap_cells=2)
    elif case == "time_overlap":
        q = p.replace(overlap_steps=11)
    elif case == "tz_pad_wraps":
        q = p.replace(tz_p=15, tz_q=1, tz_alpha=0.5)
    else:
        t = _time_decomposition(p)
        q = {"tz_p_range": dict(tz_p=33, tz_q=1), "tz_q_range": dict(tz_p=1, tz_q=17),
             "tz_q_zero": dict(tz_p=1, tz_q=0), "tz_alpha_range": dict(tz_p=1, tz_q=1, tz_alpha=1.5),
             "tz_alpha_nan": dict(tz_p=1, tz_q=1, tz_alpha=np.nan)}[case]
        q = t.replace(**q)
    with pytest.raises(L.DD4DVarError) as e:
        Plan(q)
    assert e.value.status == L.DD4DVAR_E_INVALID
    assert L.dd4dvar_last_error(None)


def test_map_query_errors():
    p = _with_values(synth.make_spec("tiny2"))
    plan = Plan(p)
    n = C.c_int64(0)
    assert L.lib().dd4dvar_plan_get_map(plan.handle, 99, 0, C.byref(n), None) == L.DD4DVAR_E_INVALID
    assert L.lib().dd4dvar_plan_get_map(plan.handle, 0, 10_000, C.byref(n), None) == L.DD4DVAR_E_INVALID
    assert L.lib().dd4dvar_plan_get_map(plan.handle, 0, 0, C.byref(n), None) == L.DD4DVAR_OK
    small = (C.c_int32 * 1)()
    cap = C.c_int64(0)
    assert L.lib().dd4dvar_plan_get_map(plan.handle, 0, 0, C.byref(cap), small) == L.DD4DVAR_E_INVALID
    plan.close()


def test_descriptors_roundtrip():
    p = _with_values(synth.make_spec("c1"))
    d = Descriptors(p, L.DD4DVAR_FP32_STATE)
    assert d.model.precision == 1 and d.model.nlat == 32 and d.data.nobs == p.nobs
