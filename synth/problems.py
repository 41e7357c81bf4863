"""Seeded synthetic twin-experiment problems for space-time DD 4D-Var.

What is drawn here (and nothing else):

* a truth snapshot on a cell-centred lat-lon grid: eight Gaussian bumps of
  height anomaly around a mean depth, with winds in geostrophic balance for a
  constant mid-latitude Coriolis parameter (twin experiment, Sec. 7);
* the time step, fixed once from a CFL number on the truth snapshot;
* the background initial state (truth + white Gaussian noise per field) and
  the diagonal background / observation standard deviations;
* observation positions (grid points drawn without replacement at every
  observation step; h, u and v are observed at each point) and observation
  noise.  Observation values need the truth trajectory, which the caller
  supplies (``finish_spec``), so this module runs no model;
* the space-time partition edges: uniform bands x pieces x intervals, or an
  irregular "brick" layout with seeded piece sizes.

Field order everywhere is (h, u, v); arrays are [field][lat][lon] with
longitude fastest, latitude running south to north.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional, Sequence

import numpy as np

DEFAULT_CONSTANTS = dict(radius=6.37122e6, gravity=9.80616, omega=7.292e-5,
                         h_ref=1.0e4)

SEED_BASE = 2205066490
# independent random streams spawned from one SeedSequence per problem
_STREAMS = ("truth", "background", "obs_positions", "obs_noise", "partition",
            "directions")

# The five benchmark configurations (index = seed offset) and small test cases.
CONFIGS = {
    "c1": dict(index=0, nlat=32, nlon=64, nsteps=20, bands=2, pieces=2,
               ntime=2, overlap_cells=2, overlap_steps=2, obs_frac=0.05,
               obs_every=5),
    "c2": dict(index=1, nlat=128, nlon=256, nsteps=100, bands=4, pieces=4,
               ntime=4, overlap_cells=4, overlap_steps=4, obs_frac=0.02,
               obs_every=4),
    "c3": dict(index=2, nlat=256, nlon=512, nsteps=200, brick=(8, 8, 24, 96),
               ntime=8, overlap_cells=3, overlap_steps=3, obs_frac=0.02,
               obs_every=4),
    "c4": dict(index=3, nlat=512, nlon=1024, nsteps=1000, bands=8, pieces=8,
               ntime=10, overlap_cells=3, overlap_steps=3, obs_frac=0.02,
               obs_every=4),
    "c5": dict(index=4, nlat=1024, nlon=2048, nsteps=200, bands=16, pieces=16,
               ntime=8, overlap_cells=4, overlap_steps=4, obs_points=15873,
               obs_every=10),
    # small cases used by the tests
    "tiny1": dict(index=100, nlat=8, nlon=16, nsteps=4, bands=1, pieces=1,
                  ntime=1, overlap_cells=0, overlap_steps=0, obs_frac=0.25,
                  obs_every=2),
    "tiny2": dict(index=101, nlat=8, nlon=16, nsteps=4, bands=2, pieces=2,
                  ntime=2, overlap_cells=1, overlap_steps=1, obs_frac=0.25,
                  obs_every=2),
    "small": dict(index=102, nlat=16, nlon=32, nsteps=12, bands=2, pieces=3,
                  ntime=3, overlap_cells=2, overlap_steps=2, obs_frac=0.1,
                  obs_every=3),
}


@dataclasses.dataclass
class Problem:
    """A complete DD 4D-Var problem: model, partition, background, obs."""
    name: str
    nlat: int
    nlon: int
    nsteps: int
    dt: float
    radius: float
    gravity: float
    omega: float
    h_ref: float
    lambda_obs: float
    mu_overlap: float
    weight_mode: int
    band_lat_edges: np.ndarray      # int32 [n_bands+1]
    band_npieces: np.ndarray        # int32 [n_bands]
    piece_lon_edges: np.ndarray     # int32, npieces+1 per band, concatenated
    time_edges: np.ndarray          # int32 [n_time+1]
    overlap_cells: int
    overlap_steps: int
    truth0: np.ndarray              # f64 [3][nlat][nlon]
    xb0: np.ndarray                 # f64 [3][nlat][nlon]
    sigma_b: np.ndarray             # f64 [3]
    obs_step: np.ndarray            # int32 [nobs]
    obs_cell: np.ndarray            # int32 [nobs]  (= lat*nlon + lon)
    obs_field: np.ndarray           # int8  [nobs]
    obs_value: Optional[np.ndarray]  # f64  [nobs]
    obs_sigma: np.ndarray           # f64  [nobs]
    obs_noise: np.ndarray           # f64  [nobs] standard-normal draws
    seed: int
    # discretization: tz_p = 0 the plain centred scheme; tz_p >= 1 the
    # Turkel-Zwas variant with offsets (tz_p, tz_q) and averaging tz_alpha
    tz_p: int = 0
    tz_q: int = 1
    tz_alpha: float = 0.0

    @property
    def nobs(self) -> int:
        return int(self.obs_step.shape[0])

    def rng(self, stream: str) -> np.random.Generator:
        """A fresh generator for one of the named independent streams."""
        children = np.random.SeedSequence(self.seed).spawn(len(_STREAMS))
        return np.random.Generator(np.random.PCG64(children[_STREAMS.index(stream)]))

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def composition(rng: np.random.Generator, total: int, parts: int, lo: int,
                hi: int) -> np.ndarray:
    """Seeded bounded composition of ``total`` into ``parts`` sizes in [lo, hi].

    Sizes are drawn one at a time, uniformly between the bounds that keep the
    remainder feasible, then shuffled.
    """
    if not (parts * lo <= total <= parts * hi):
        raise ValueError("infeasible composition")
    sizes = []
    rem = total
    for k in range(parts, 0, -1):
        a = max(lo, rem - hi * (k - 1))
        b = min(hi, rem - lo * (k - 1))
        x = int(rng.integers(a, b + 1))
        sizes.append(x)
        rem -= x
    sizes = np.array(sizes, dtype=np.int64)
    rng.shuffle(sizes)
    return sizes


def _uniform_edges(n: int, parts: int) -> np.ndarray:
    return np.array([(k * n) // parts for k in range(parts + 1)], dtype=np.int32)


def _truth_snapshot(rng, nlat, nlon, radius, gravity, omega, h_ref,
                    nbumps=8, amplitude=100.0):
    """Bump-sum height field and geostrophic winds at the cell centres."""
    dlat = math.pi / nlat
    dlon = 2 * math.pi / nlon
    theta = -math.pi / 2 + (np.arange(nlat) + 0.5) * dlat
    lam = np.arange(nlon) * dlon
    th = theta[:, None]
    la = lam[None, :]
    x = np.cos(th) * np.cos(la)
    y = np.cos(th) * np.sin(la)
    z = np.sin(th) * np.ones_like(la)
    dx_dth = -np.sin(th) * np.cos(la)
    dy_dth = -np.sin(th) * np.sin(la)
    dz_dth = np.cos(th) * np.ones_like(la)
    # d(r)/d(lambda) divided by cos(theta)
    dx_dla_c = -np.sin(la) * np.ones_like(th)
    dy_dla_c = np.cos(la) * np.ones_like(th)

    zc = rng.uniform(-1.0, 1.0, nbumps)
    phic = rng.uniform(0.0, 2 * math.pi, nbumps)
    amp = rng.uniform(-1.0, 1.0, nbumps)
    width = rng.uniform(500e3, 1500e3, nbumps)
    rc = np.sqrt(1.0 - zc ** 2)
    hb = np.zeros((nlat, nlon))
    dh_dth = np.zeros((nlat, nlon))
    dh_dla_c = np.zeros((nlat, nlon))
    for k in range(nbumps):
        xk, yk, zk = rc[k] * math.cos(phic[k]), rc[k] * math.sin(phic[k]), zc[k]
        dot = x * xk + y * yk + z * zk
        kappa = radius ** 2 / width[k] ** 2
        gk = amp[k] * np.exp(-kappa * (1.0 - dot))     # chordal^2 = 2 - 2 dot
        hb += gk
        dh_dth += gk * kappa * (dx_dth * xk + dy_dth * yk + dz_dth * zk)
        dh_dla_c += gk * kappa * (dx_dla_c * xk + dy_dla_c * yk)
    scale = amplitude / np.max(np.abs(hb))
    f0 = 2 * omega * math.sin(math.pi / 4)
    h = h_ref + scale * hb
    u = -(gravity / (f0 * radius)) * scale * dh_dth
    v = (gravity / (f0 * radius)) * scale * dh_dla_c
    return np.stack([h, u, v]).astype(np.float64)


def cfl_dt(x0, nlat, nlon, radius, gravity, cfl=0.5):
    """Time step from a CFL number on the narrowest (polar) zonal spacing."""
    dlat = math.pi / nlat
    dlon = 2 * math.pi / nlon
    c0 = math.cos(-math.pi / 2 + 0.5 * dlat)
    h, u, v = x0
    speed = np.sqrt(gravity * h) + np.sqrt(u * u + v * v)
    return cfl * radius * c0 * dlon / float(np.max(speed))


def make_spec(cfg, *, seed: Optional[int] = None, dt: Optional[float] = None,
              lambda_obs=1.0, mu_overlap=1.0, weight_mode=0,
              constants=None) -> Problem:
    """Draw everything except observation values (which need the truth run)."""
    if isinstance(cfg, str):
        name = cfg
        cfg = CONFIGS[cfg]
    else:
        name = cfg.get("name", "custom")
    const = dict(DEFAULT_CONSTANTS)
    if constants:
        const.update(constants)
    nlat, nlon, nsteps = cfg["nlat"], cfg["nlon"], cfg["nsteps"]
    if seed is None:
        seed = SEED_BASE + int(cfg.get("index", 0))
    children = np.random.SeedSequence(seed).spawn(len(_STREAMS))
    rngs = {n: np.random.Generator(np.random.PCG64(c)) for n, c in zip(_STREAMS, children)}

    truth0 = _truth_snapshot(rngs["truth"], nlat, nlon, const["radius"],
                             const["gravity"], const["omega"], const["h_ref"])
    if dt is None:
        dt = cfl_dt(truth0, nlat, nlon, const["radius"], const["gravity"]) * float(
            cfg.get("dt_scale", 1.0))
    std = truth0.reshape(3, -1).std(axis=1)
    sigma_b = 0.05 * std
    sigma_o = 0.01 * std
    xb0 = truth0 + sigma_b[:, None, None] * rngs["background"].standard_normal(truth0.shape)

    # partition
    if "brick" in cfg:
        nb, npc, lo, hi = cfg["brick"]
        prng = rngs["partition"]
        bsz = composition(prng, nlat, nb, lo, hi)
        band_edges = np.concatenate([[0], np.cumsum(bsz)]).astype(np.int32)
        band_np = np.full(nb, npc, dtype=np.int32)
        pieces = []
        for _ in range(nb):
            psz = composition(prng, nlon, npc, lo, hi)
            pieces.append(np.concatenate([[0], np.cumsum(psz)]))
        piece_edges = np.concatenate(pieces).astype(np.int32)
    else:
        nb, npc = cfg["bands"], cfg["pieces"]
        band_edges = _uniform_edges(nlat, nb)
        band_np = np.full(nb, npc, dtype=np.int32)
        piece_edges = np.concatenate([_uniform_edges(nlon, npc)] * nb).astype(np.int32)
    time_edges = _uniform_edges(nsteps, cfg["ntime"])

    # observation positions and noise
    ncell = nlat * nlon
    if "obs_points" in cfg:
        npts = int(cfg["obs_points"])
    else:
        npts = int(math.floor(cfg["obs_frac"] * ncell + 1e-9))
    every = int(cfg["obs_every"])
    steps, cells, fields = [], [], []
    for k in range(0, nsteps + 1, every):
        pts = np.sort(rngs["obs_positions"].choice(ncell, npts, replace=False))
        steps.append(np.full(3 * npts, k))
        cells.append(np.repeat(pts, 3))
        fields.append(np.tile(np.arange(3), npts))
    obs_step = np.concatenate(steps).astype(np.int32)
    obs_cell = np.concatenate(cells).astype(np.int32)
    obs_field = np.concatenate(fields).astype(np.int8)
    obs_noise = rngs["obs_noise"].standard_normal(obs_step.shape[0])
    obs_sigma = sigma_o[obs_field.astype(np.int64)].astype(np.float64)

    return Problem(
        name=name, nlat=nlat, nlon=nlon, nsteps=nsteps, dt=float(dt),
        radius=const["radius"], gravity=const["gravity"], omega=const["omega"],
        h_ref=const["h_ref"], lambda_obs=float(lambda_obs),
        mu_overlap=float(mu_overlap), weight_mode=int(weight_mode),
        band_lat_edges=band_edges, band_npieces=band_np,
        piece_lon_edges=piece_edges, time_edges=time_edges,
        overlap_cells=int(cfg["overlap_cells"]),
        overlap_steps=int(cfg["overlap_steps"]),
        truth0=truth0, xb0=xb0, sigma_b=sigma_b.astype(np.float64),
        obs_step=obs_step, obs_cell=obs_cell, obs_field=obs_field,
        obs_value=None, obs_sigma=obs_sigma, obs_noise=obs_noise, seed=seed,
        tz_p=int(cfg.get("tz", (0, 1, 0.0))[0]), tz_q=int(cfg.get("tz", (0, 1, 0.0))[1]),
        tz_alpha=float(cfg.get("tz", (0, 1, 0.0))[2]))


TruthForward = Callable[[Problem, np.ndarray, Sequence[int]], np.ndarray]


def finish_spec(spec: Problem, truth_forward: TruthForward) -> Problem:
    """Sample the truth trajectory at the observation points and add noise.

    ``truth_forward(spec, x0, steps)`` must return the model states at the
    requested steps, shape [len(steps)][3][nlat][nlon], from initial state x0.
    """
    steps = sorted(set(int(k) for k in spec.obs_step))
    traj = np.asarray(truth_forward(spec, spec.truth0, steps), dtype=np.float64)
    pos = {k: i for i, k in enumerate(steps)}
    idx = np.array([pos[int(k)] for k in spec.obs_step], dtype=np.int64)
    flat = traj.reshape(len(steps), 3, -1)
    truth_vals = flat[idx, spec.obs_field.astype(np.int64), spec.obs_cell.astype(np.int64)]
    return spec.replace(obs_value=truth_vals + spec.obs_sigma * spec.obs_noise)


def make_problem(cfg, truth_forward: TruthForward, **kw) -> Problem:
    return finish_spec(make_spec(cfg, **kw), truth_forward)
