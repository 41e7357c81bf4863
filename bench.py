#!/usr/bin/env python3
"""Benchmark: batched local cost + gradient of space-time DD 4D-Var on one GPU.

One step = one evaluation of every subdomain's regularized local functional
and its gradient (background term, forward sweep, observation and overlap
misfits, adjoint sweep, FP64 reductions) through dd4dvar_local_cost_grad.

Default workload: SWE on a 1024 x 2048 lat-lon grid, 200 steps, 16 x 16
spatial pieces x 8 time intervals (2048 subdomains), overlap 4 cells / 4
steps, 999,999 observations every 10 steps; FP32 state sweeps with FP64
costs and gradients.  Inputs are seeded and synthetic (twin experiment); the
truth run that produces the observation values runs on the GPU library.

The library's autotuner picks the execution plan (step kernels, or
persistent per-box sweeps with one launch per sweep or fused), timing HIP
graph replays; the timed steps are graph replays of that plan.

Prints one JSON line.  Extra fields: the autotuner's candidates, the same
plan launched eagerly, the plain per-subdomain FP64 path (one launch per
subdomain per step) and the batched FP64 path, the FP32 error against FP64,
phase timings, an FP32-vs-FP64 DD solve, the Gauss-Newton local solver, the
Turkel-Zwas variant on a time decomposition of the same grid, and the oracle
timed on host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gpu_truth_forward(spec, x0, steps):
    """Truth trajectory at the observation steps, run by the GPU library."""
    import torch
    from paper_2205_06649_amd.context import Context
    one = spec.replace(band_lat_edges=np.array([0, spec.nlat], np.int32),
                       band_npieces=np.array([1], np.int32),
                       piece_lon_edges=np.array([0, spec.nlon], np.int32),
                       time_edges=np.array([0, spec.nsteps], np.int32),
                       overlap_cells=0, overlap_steps=0, xb0=x0,
                       obs_step=spec.obs_step[:0], obs_cell=spec.obs_cell[:0],
                       obs_field=spec.obs_field[:0], obs_value=np.zeros(0),
                       obs_sigma=spec.obs_sigma[:0], obs_noise=spec.obs_noise[:0])
    ctx = Context(one, "fp64")
    traj = ctx.forward_global(torch.from_numpy(np.ascontiguousarray(x0)).cuda())
    out = traj[list(steps)].cpu().numpy()
    del traj
    ctx.close()
    torch.cuda.empty_cache()
    return out


def algorithmic_bytes(ctx, prec_bytes, persistent=False):
    """Compulsory HBM bytes of one evaluation, per sweep (no re-reads).

    Step kernels (one launch per level): the forward launch at level n reads
    Z^n and Z^{n-1} and writes Z^{n+1} (3 fields each) plus the frozen ring
    values of level n; the adjoint launch at level n reads Z^n, lambda^{n+1},
    lambda^{n+2} and writes lambda^n (where they exist), reads the overlap
    target where covered, the coverage byte, the ring values and 20 B per
    observation entry; level 0 reads x, x_b (FP64) and writes the FP64
    gradient instead of lambda^0.

    Persistent sweeps (one workgroup per box for the whole window): the
    current level and the one before stay on chip, so the forward only writes
    each level once (and reads x and the ring) and the adjoint only reads
    each level once (plus targets, coverage, ring, observations and the
    level-0 control, background and gradient).
    """
    from paper_2205_06649_amd import _lib as L
    b = prec_bytes
    tcount = L.dd4dvar_plan_get_map(ctx.plan, L.MAP_TIME_COUNT, 0)
    fwd = adj = 0.0
    pts = 0
    for s, inf in enumerate(ctx.info):
        ny, nx, lev0, nlev = int(inf[1]), int(inf[3]), int(inf[4]), int(inf[5])
        ncell = ny * nx
        L_ = nlev - 1
        pts += ncell * L_
        nfrozen = int(np.count_nonzero(L.dd4dvar_plan_get_map(ctx.plan, L.MAP_HALO_SRC, s) >= 0))
        cover = L.dd4dvar_plan_get_map(ctx.plan, L.MAP_COVER, s).astype(np.int64)
        nobs = L.dd4dvar_plan_get_map(ctx.plan, L.MAP_OBS_BIN, s).size
        # forward: init + L steps
        fwd += ncell * (24 + 3 * b)
        for n in range(L_):
            nvec = 1 if persistent else (3 if n >= 1 else 2)
            fwd += ncell * 3 * b * nvec + nfrozen * 3 * b
        # adjoint: levels L..0
        for n in range(L_, -1, -1):
            if persistent:
                nvec = 1
            else:
                nvec = 1 + (n + 1 <= L_) + (n + 2 <= L_) + (n > 0)
            covered = int(np.count_nonzero(cover * tcount[lev0 + n] - 1 > 0))
            adj += ncell * (nvec * 3 * b + 1) + covered * 3 * b + nfrozen * 3 * b
            if n == 0:
                adj += ncell * 72
        adj += nobs * 20
    return fwd, adj, pts


def gn_product_bytes(ctx, prec_bytes, persistent=False):
    """Compulsory HBM bytes of one Gauss-Newton normal-matrix product: the
    tangent-linear sweep and the adjoint sweep with the Gauss-Newton forcing.

    Step kernels: the tangent-linear launch at level n reads Z^n, dZ^n,
    dZ^{n-1} and writes dZ^{n+1} (plus the ring of Z^n); the adjoint launch
    reads Z^n, lambda^{n+1}, lambda^{n+2}, dZ^n and writes lambda^n.
    Persistent sweeps: dZ^n and dZ^{n-1} (lambda^{n+1}, lambda^{n+2}) stay on
    chip, so the tangent-linear sweep reads Z^n and writes dZ^{n+1} once per
    level and the adjoint reads Z^n, and dZ^n only where another box covers
    the cell.  Both read dx (FP64) at level 0 and write the FP64 product
    there, and 20 B per observation entry.
    """
    from paper_2205_06649_amd import _lib as L
    b = prec_bytes
    tcount = L.dd4dvar_plan_get_map(ctx.plan, L.MAP_TIME_COUNT, 0)
    tlm = adj = 0.0
    for s, inf in enumerate(ctx.info):
        ny, nx, lev0, nlev = int(inf[1]), int(inf[3]), int(inf[4]), int(inf[5])
        ncell = ny * nx
        L_ = nlev - 1
        nfrozen = int(np.count_nonzero(L.dd4dvar_plan_get_map(ctx.plan, L.MAP_HALO_SRC, s) >= 0))
        cover = L.dd4dvar_plan_get_map(ctx.plan, L.MAP_COVER, s).astype(np.int64)
        nobs = L.dd4dvar_plan_get_map(ctx.plan, L.MAP_OBS_BIN, s).size
        tlm += ncell * (24 + 3 * b)
        for n in range(L_):
            nvec = 2 if persistent else (4 if n >= 1 else 3)
            tlm += ncell * 3 * b * nvec + nfrozen * 3 * b
        for n in range(L_, -1, -1):
            if persistent:
                nvec = 1
                dz = int(np.count_nonzero(cover * tcount[lev0 + n] - 1 > 0))
            else:
                nvec = 1 + (n + 1 <= L_) + (n + 2 <= L_) + (n > 0)
                dz = ncell
            adj += ncell * (nvec * 3 * b + 1) + dz * 3 * b + nfrozen * 3 * b
            if n == 0:
                adj += ncell * 24
        adj += nobs * 20
    return tlm, adj


# HBM bytes per launch of the dominant kernels on the default workload, from
# rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per dispatch, scaled by 2.0 and
# 1.0: what the two counters read for a plain 1 GiB device copy), keyed by a
# digest of the kernel sources they were measured on: a changed kernel (or
# another workload) reports null until it is measured again.
MEASURED_TRAFFIC = {
    "k_adj": ("sweep", "ff254c10224ff0ba", 1158229105),
    "k_adj_box/10": ("box", "d0a69a4840912446", 16093533656),
    "k_adj_box/11": ("box", "d0a69a4840912446", 16089092536),
    "k_adj_strip/11": ("box", "d0a69a4840912446", 16657258389),
    "k_eval_box/10": ("box", "d0a69a4840912446", 29856191456),
    # Gauss-Newton normal-matrix product: tangent-linear sweep (10 passes)
    # and the adjoint with the Gauss-Newton forcing (column strips, 11 rows)
    "k_tlm_box/10": ("box", "d0a69a4840912446", 16788000987),
    "k_adj_strip_gn/11": ("box", "d0a69a4840912446", 15650230395),
}
KERNEL_SOURCES = {"sweep": ("sweep.hip", "kernels.h", "stencil.h"),
                  "box": ("box.hip", "kernels.h", "stencil.h")}


def measured_traffic(kernel, config):
    import hashlib
    if config != "c5" or kernel not in MEASURED_TRAFFIC:
        return None
    unit, want, nbytes = MEASURED_TRAFFIC[kernel]
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[unit]:
        with open(os.path.join(ROOT, "paper_2205_06649_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return nbytes if h.hexdigest()[:16] == want else None


EXEC_MODES = {0: "step kernels, all boxes per launch",
              2: "persistent per-box forward and adjoint sweeps, one launch each",
              3: "persistent per-box sweeps, forward and adjoint fused in one launch",
              4: "persistent per-box sweeps, the adjoint in column strips"}

KERNEL_NAMES = {0: "k_adj", 2: "k_adj_box", 3: "k_eval_box", 4: "k_adj_strip"}

# Alg. 1 with L-BFGS local solves run to a 1e-6 relative reduction of every
# local gradient norm (the configuration's solve target), two outer sweeps
SOLVE_OPTS = dict(max_outer=2, max_iter=600, grad_rtol=1e-6, outer_tol=0.0)
SOLVE_TARGET = 1e-6


def solve_leg(prob, mode):
    """DD solve (Alg. 1) with L-BFGS local solves to a 1e-6 relative
    reduction of every local gradient, in FP64, and the same solve with FP32
    state sweeps (which stops at its rounding floor, reported): wall time,
    evaluations, iterations, the gradient reduction reached, and the FP32
    analysis error relative to the FP64 analysis (per field, relative to its
    spread; maximum over fields)."""
    import torch
    from paper_2205_06649_amd.context import Context
    out = {"options": dict(SOLVE_OPTS)}
    xa = {}
    for prec in ("fp64", "fp32"):
        ctx = Context(prob, prec)
        if prec == "fp32":
            ctx.set_exec_mode(mode)
        torch.cuda.synchronize()
        t = time.perf_counter()
        a, rep, st, _ = ctx.solve(**SOLVE_OPTS)
        sec = time.perf_counter() - t
        xa[prec] = a
        out[prec] = {"seconds": sec, "evaluations": int(rep.total_evals),
                     "lbfgs_iters": int(rep.lbfgs_iters), "J_final": float(rep.J_final),
                     "gnorm_ratio_max": float(rep.gnorm_ratio_max),
                     "target_met": bool(rep.gnorm_ratio_max <= SOLVE_TARGET)}
        log(f"{prec} solve: {sec:.2f} s, {rep.total_evals} evaluations, {rep.lbfgs_iters} "
            f"iterations, gradient ratio {rep.gnorm_ratio_max:.2e}")
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    ref = xa["fp64"]
    out["fp32_analysis_rel_err"] = float(max(
        np.linalg.norm(xa["fp32"][f] - ref[f]) / np.linalg.norm(ref[f] - ref[f].mean())
        for f in range(3)))
    out["speedup_fp32_vs_fp64"] = out["fp64"]["seconds"] / out["fp32"]["seconds"]
    return out


def few_boxes_solve_leg(spec, reps=3):
    """Local solves on a decomposition with few large boxes: the benchmark's
    grid, window and observations as a time decomposition into 8 intervals,
    each box the whole sphere (6.3 million control entries per box), FP32
    state sweeps.  One outer iteration of Alg. 1 with 10 L-BFGS iterations,
    and one with 2 Gauss-Newton updates of 6 CG products; the time of one
    evaluation beside them, so that what the solver's own vector work costs
    shows as the rest."""
    import torch
    import synth
    from paper_2205_06649_amd.context import Context
    tspec = spec.replace(band_lat_edges=np.array([0, spec.nlat], np.int32),
                         band_npieces=np.array([1], np.int32),
                         piece_lon_edges=np.array([0, spec.nlon], np.int32), overlap_cells=0)
    prob = synth.finish_spec(tspec, gpu_truth_forward)
    ctx = Context(prob, "fp32")
    out = {"workload": f"{prob.nlat}x{prob.nlon}, {prob.nsteps} steps, "
                       f"{len(prob.time_edges) - 1} intervals (boxes covering the sphere)",
           "solver_parts": ctx.solver_parts()}
    x = ctx.background_controls()
    ms, _, _ = time_evals(ctx, x, reps, 1)
    out["eval_ms"] = ms
    for name, kw in (("lbfgs", dict(max_iter=10)),
                     ("gauss_newton_cg", dict(max_iter=2, local_solver="gn", cg_max_iter=6))):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, rep, _, _ = ctx.solve(max_outer=1, outer_tol=0.0, **kw)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        out[name] = {"seconds": sec, "evaluations": int(rep.total_evals),
                     "products": int(rep.gn_products)}
        log(f"few-box {name} solve: {sec * 1e3:.0f} ms, {rep.total_evals} evaluations, "
            f"{rep.gn_products} products")
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return out


def differentiation_leg(config="c4"):
    """The local sweeps under torch.autograd on the 512 x 1024, 1000-step,
    8 x 8 x 10 decomposition (local windows of 103-106 steps): LocalSweep maps
    the packed FP64 controls to the packed trajectories of every box, and its
    backward is the library's adjoint sweep (Sec. 2 adjoint model).  A
    nonlinear loss of the trajectories, L = 1/2 sum ((Z - c) / sigma_b)^2
    with c the rest state, is differentiated with every level stored and with
    square-root checkpointing (pairs every ~sqrt(2 L) levels, segments
    recomputed in the adjoint): the two gradients must be equal bit for bit,
    and the gradient is checked against centred differences of L.  Reported:
    the state arena, the device memory in use after the forward and after
    the backward, and the time of forward + backward, for both."""
    import math
    import torch
    import synth
    from paper_2205_06649_amd.autograd import local_sweep
    from paper_2205_06649_amd.context import Context
    spec = synth.make_spec(config)
    prob = synth.finish_spec(spec, gpu_truth_forward)
    ctx = Context(prob, "fp64")
    nlev = max(int(i[5]) for i in ctx.info)
    stride = int(round(math.sqrt(2 * (nlev - 1))))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4)
    sb = torch.tensor(prob.sigma_b, dtype=torch.float64, device="cuda")
    scale = torch.cat([sb[f].expand(int(i[1]) * int(i[3])) for i in ctx.info for f in range(3)])
    x = ctx.background_controls() + 0.3 * scale * torch.randn(ctx.ctrl_len, generator=gen,
                                                              dtype=torch.float64, device="cuda")
    d = scale * torch.randn(ctx.ctrl_len, generator=gen, dtype=torch.float64, device="cuda")
    # the rest state and 1/sigma_b per field, applied box by box (views of
    # the packed trajectory, [nlev][3][ny*nx] each)
    c = torch.zeros(3, 1, dtype=torch.float64, device="cuda")
    c[0] = prob.h_ref
    isb = (1.0 / sb)[:, None]
    boxes = [(int(i[7]), int(i[5]), int(i[1]) * int(i[3])) for i in ctx.info]

    def loss(traj):
        return 0.5 * sum((((traj[o:o + n * 3 * m].view(n, 3, m) - c) * isb) ** 2).sum()
                         for o, n, m in boxes)

    def used():
        free, total = torch.cuda.mem_get_info()
        return total - free

    out = {"workload": f"SWE on the sphere {prob.nlat}x{prob.nlon}, {prob.nsteps} steps, "
                       f"{ctx.nsub} subdomains, local windows up to {nlev - 1} steps, FP64",
           "checkpoint_stride": stride, "runs": {}}
    grads = {}
    base = used()
    for ck in (0, stride):
        arena = ctx.set_checkpointing(ck)
        torch.cuda.synchronize()
        xr = x.clone().requires_grad_(True)
        t0 = time.perf_counter()
        traj = local_sweep(ctx, xr)
        L = loss(traj)
        torch.cuda.synchronize()
        after_fwd = used()
        L.backward()
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        after_bwd = used()
        ctx.synchronize()
        grads[ck] = xr.grad.clone()
        out["runs"]["every_level" if ck == 0 else "sqrt_checkpoints"] = {
            "stride": ck, "state_arena_bytes": int(arena),
            "device_bytes_in_use_after_forward": int(after_fwd),
            "device_bytes_in_use_after_backward": int(after_bwd),
            "device_bytes_added_by_forward": int(after_fwd - base),
            "seconds_forward_backward": sec}
        log(f"differentiation, stride {ck}: arena {arena / 1e9:.2f} GB, in use {after_fwd / 1e9:.1f} GB"
            f" after forward, {sec:.2f} s forward + backward")
        del xr, traj, L
        torch.cuda.empty_cache()
    out["device_bytes_in_use_before"] = int(base)
    out["checkpointed_gradient_bit_equal"] = bool(torch.equal(grads[0], grads[stride]))
    an = float(torch.dot(grads[stride], d))
    fd = {}
    with torch.no_grad():
        for eps in (1e-3, 1e-4):
            Lp = float(loss(local_sweep(ctx, x + eps * d)))
            Lm = float(loss(local_sweep(ctx, x - eps * d)))
            fd[eps] = (Lp - Lm) / (2 * eps)
    out["fd_check"] = {"directional_derivative": an,
                       "centred_differences": {str(k): v for k, v in fd.items()},
                       "rel_err": {str(k): abs(v - an) / abs(an) for k, v in fd.items()}}
    log(f"differentiation: <grad, d> {an:.6e}, centred differences rel err "
        f"{abs(fd[1e-4] - an) / abs(an):.2e}")
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return out


GN_OPTS = dict(max_outer=2, max_iter=3, cg_max_iter=20, cg_rtol=1e-4, grad_rtol=1e-6,
               outer_tol=0.0)


def gn_leg(prob, x, mode, passes, config, reps=10, solves=True):
    """Gauss-Newton local solver (Alg. 5 / Alg. 6).  The normal-matrix
    product (tangent-linear sweep, then the adjoint sweep forced by the
    residual weights applied to the perturbation) timed at x in FP32, and DD
    solves with Gauss-Newton local solves in FP32 and FP64: wall time,
    evaluations, products, and the FP32 analysis error relative to the FP64
    Gauss-Newton analysis (per field, relative to its spread)."""
    import torch
    from paper_2205_06649_amd.context import Context
    out = {"options": dict(GN_OPTS)}
    ctx = Context(prob, "fp32")
    ctx.set_exec_mode(mode)
    ctx.forward(x, with_traj=False)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    sb = torch.tensor(prob.sigma_b, dtype=torch.float64, device="cuda")
    scale = torch.cat([sb[f].expand(int(i[1]) * int(i[3])) for i in ctx.info for f in range(3)])
    dx = scale * torch.randn(ctx.ctrl_len, generator=gen, dtype=torch.float64, device="cuda")
    hv = torch.empty_like(dx)

    def timed(fn):
        for _ in range(2):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / reps

    ms_prod = timed(lambda: ctx.gn_hessvec(dx, hv))
    ms_tlm = timed(lambda: ctx.tangent_linear(dx, with_traj=False))
    tlm_b, adj_b = gn_product_bytes(ctx, 4, persistent=(mode >= 2))
    out["exec_mode"] = EXEC_MODES[mode]
    out["product_ms"] = ms_prod
    out["tlm_ms"] = ms_tlm
    out["adjoint_ms"] = ms_prod - ms_tlm
    out["tlm_algorithmic_bytes"] = tlm_b
    out["adjoint_algorithmic_bytes"] = adj_b
    out["product_algorithmic_GBs"] = (tlm_b + adj_b) / (ms_prod * 1e-3) / 1e9
    out["tlm_algorithmic_GBs"] = tlm_b / (ms_tlm * 1e-3) / 1e9
    out["adjoint_algorithmic_GBs"] = adj_b / ((ms_prod - ms_tlm) * 1e-3) / 1e9
    if mode >= 2:
        # HBM bytes the counters measured per launch (the context's first plan:
        # 10 passes of 1024 cells; the strip adjoint with the autotuned rows),
        # while the kernel sources are unchanged
        out["tlm_traffic"] = measured_traffic("k_tlm_box/10", config)
        out["adjoint_traffic"] = measured_traffic(
            f"k_adj_strip_gn/{passes}" if mode == 4 else "k_adj_box_gn/10", config)
    log(f"gauss-newton product {ms_prod:.2f} ms (tangent-linear {ms_tlm:.2f} ms)")
    ctx.close()
    del ctx, dx, hv
    torch.cuda.empty_cache()
    if not solves:
        return out
    xa = {}
    for prec in ("fp64", "fp32"):
        ctx = Context(prob, prec)
        if prec == "fp32":
            ctx.set_exec_mode(mode)
        torch.cuda.synchronize()
        t = time.perf_counter()
        a, rep, st, _ = ctx.solve(local_solver="gn", **GN_OPTS)
        sec = time.perf_counter() - t
        xa[prec] = a
        out[prec] = {"seconds": sec, "evaluations": int(rep.total_evals),
                     "gn_iters": int(rep.lbfgs_iters), "products": int(rep.gn_products),
                     "J_final": float(rep.J_final), "gnorm_ratio_max": float(rep.gnorm_ratio_max)}
        log(f"{prec} gauss-newton solve: {sec:.2f} s, {rep.total_evals} evaluations, "
            f"{rep.gn_products} products")
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    # mixed precision: FP64 evaluations, FP32 normal-matrix products
    ctx64 = Context(prob, "fp64")
    ctx32 = Context(prob, "fp32")
    ctx32.set_exec_mode(mode)
    torch.cuda.synchronize()
    t = time.perf_counter()
    a, rep, st, _ = ctx64.solve(local_solver="gn", products=ctx32, **GN_OPTS)
    sec = time.perf_counter() - t
    xa["mixed"] = a
    out["mixed"] = {"seconds": sec, "evaluations": int(rep.total_evals),
                    "gn_iters": int(rep.lbfgs_iters), "products": int(rep.gn_products),
                    "J_final": float(rep.J_final), "gnorm_ratio_max": float(rep.gnorm_ratio_max)}
    log(f"mixed gauss-newton solve: {sec:.2f} s, {rep.total_evals} evaluations, "
        f"{rep.gn_products} products, gradient ratio {rep.gnorm_ratio_max:.2e}")
    ctx64.close()
    ctx32.close()
    del ctx64, ctx32
    torch.cuda.empty_cache()
    # the Lanczos solver of the normal equations (Alg. 7), FP32 sweeps: same
    # products as CG, and the extreme Ritz values of the local preconditioned
    # normal matrices
    ctx = Context(prob, "fp32")
    ctx.set_exec_mode(mode)
    torch.cuda.synchronize()
    t = time.perf_counter()
    a, rep, st, _ = ctx.solve(local_solver="gn", krylov="lanczos", **GN_OPTS)
    sec = time.perf_counter() - t
    xa["lanczos_fp32"] = a
    out["lanczos_fp32"] = {"seconds": sec, "evaluations": int(rep.total_evals),
                           "gn_iters": int(rep.lbfgs_iters), "products": int(rep.gn_products),
                           "J_final": float(rep.J_final),
                           "gnorm_ratio_max": float(rep.gnorm_ratio_max),
                           "ritz_min": float(rep.ritz_min), "ritz_max": float(rep.ritz_max)}
    log(f"fp32 gauss-newton solve with lanczos: {sec:.2f} s, {rep.gn_products} products, "
        f"Ritz values {rep.ritz_min:.3e} .. {rep.ritz_max:.3e}")
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    ref = xa["fp64"]
    out["lanczos_fp32_vs_cg_fp32_rel_err"] = float(max(
        np.linalg.norm(xa["lanczos_fp32"][f] - xa["fp32"][f]) / np.linalg.norm(ref[f] - ref[f].mean())
        for f in range(3)))
    for k in ("fp32", "mixed", "lanczos_fp32"):
        out[f"{k}_analysis_rel_err"] = float(max(
            np.linalg.norm(xa[k][f] - ref[f]) / np.linalg.norm(ref[f] - ref[f].mean())
            for f in range(3)))
    out["speedup_fp32_vs_fp64"] = out["fp64"]["seconds"] / out["fp32"]["seconds"]
    out["speedup_mixed_vs_fp64"] = out["fp64"]["seconds"] / out["mixed"]["seconds"]
    return out


TZ_VARIANT = (2, 2, 0.5)


def tz_leg(spec, reps=5):
    """Turkel-Zwas variant (Sec. 7 discrete U, V, H with offsets p, q and
    averaging alpha) on a time decomposition of the benchmark's grid, window,
    intervals and observation network: one box per interval, each covering
    the sphere (the truth run that makes the observations uses the variant
    too).  FP32 and FP64 evaluations with the step kernels, the sweep phases,
    and the algorithmic rate of each sweep; then the benchmark's own space-time
    decomposition under the variant (frozen pads), FP32."""
    import torch

    import synth
    from paper_2205_06649_amd.context import Context
    p_, q_, a_ = TZ_VARIANT
    tspec = spec.replace(band_lat_edges=np.array([0, spec.nlat], np.int32),
                         band_npieces=np.array([1], np.int32),
                         piece_lon_edges=np.array([0, spec.nlon], np.int32),
                         overlap_cells=0, tz_p=p_, tz_q=q_, tz_alpha=a_)
    prob = synth.finish_spec(tspec, gpu_truth_forward)
    out = {"tz_p": p_, "tz_q": q_, "tz_alpha": a_,
           "workload": f"{prob.nlat}x{prob.nlon}, {prob.nsteps} steps, "
                       f"{len(prob.time_edges) - 1} intervals (boxes covering the sphere), "
                       f"overlap {prob.overlap_steps} steps, {prob.nobs} obs"}
    res = {}
    for prec, b in (("fp32", 4), ("fp64", 8)):
        ctx = Context(prob, prec)
        out[f"step_kernels_{prec}"] = {0: "gather", 1: "column walk",
                                       2: "column walk, persistent forward"}[ctx.tz_kernels()["kind"]]
        gen = torch.Generator(device="cuda")
        gen.manual_seed(2205)
        sb = torch.tensor(prob.sigma_b, dtype=torch.float64, device="cuda")
        scale = torch.cat([sb[f].expand(int(i[1]) * int(i[3])) for i in ctx.info for f in range(3)])
        x = ctx.background_controls() + 0.3 * scale * torch.randn(
            ctx.ctrl_len, generator=gen, dtype=torch.float64, device="cuda")
        ms, J, g = time_evals(ctx, x, reps, 2)
        ctx.set_timing(True)
        ctx.cost_grad(x, J, g)
        ctx.get_timing()
        for _ in range(reps):
            ctx.cost_grad(x, J, g)
        t = ctx.get_timing()
        ctx.set_timing(False)
        # compulsory bytes as for the plain step kernels: the 13-point
        # neighbourhoods are re-reads of the same levels through the caches
        fwd_b, adj_b, _ = algorithmic_bytes(ctx, b)
        fwd_ms, adj_ms = t["fwd_ms"] / t["calls"], t["adj_ms"] / t["calls"]
        pts = sum(int(i[1]) * int(i[3]) * (int(i[5]) - 1) for i in ctx.info)
        res[prec] = (J.cpu().numpy(), g.cpu().numpy())
        out[prec] = {"ms_per_eval": ms, "local_point_steps_per_s": pts / (ms * 1e-3),
                     "forward_ms": fwd_ms, "adjoint_ms": adj_ms,
                     "forward_GBs": fwd_b / (fwd_ms * 1e-3) / 1e9,
                     "adjoint_GBs": adj_b / (adj_ms * 1e-3) / 1e9,
                     "adjoint_frac_of_hbm_peak": adj_b / (adj_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        log(f"turkel-zwas {prec}: {ms:.2f} ms/eval (forward {fwd_ms:.2f} ms, "
            f"{out[prec]['forward_GBs']:.0f} GB/s; adjoint {adj_ms:.2f} ms, "
            f"{out[prec]['adjoint_GBs']:.0f} GB/s)")
        ctx.close()
        del ctx, x, J, g
        torch.cuda.empty_cache()
    (J32, g32), (J64, g64) = res["fp32"], res["fp64"]
    out["fp32_vs_fp64_rel_err"] = {
        "J_max": float(np.max(np.abs(J32 - J64) / np.abs(J64))),
        "grad_norm": float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))}
    # the benchmark's own space-time decomposition (2048 boxes) under the
    # variant: every box reads a frozen pad q rows and p columns wide, which
    # the exchange refreshes; FP32 step kernels
    sspec = spec.replace(tz_p=p_, tz_q=q_, tz_alpha=a_)
    sprob = synth.finish_spec(sspec, gpu_truth_forward)
    ctx = Context(sprob, "fp32")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2205)
    sb = torch.tensor(sprob.sigma_b, dtype=torch.float64, device="cuda")
    scale = torch.cat([sb[f].expand(int(i[1]) * int(i[3])) for i in ctx.info for f in range(3)])
    x = ctx.background_controls() + 0.3 * scale * torch.randn(
        ctx.ctrl_len, generator=gen, dtype=torch.float64, device="cuda")
    ms, J, g = time_evals(ctx, x, reps, 2)
    for _ in range(2):
        ctx.exchange(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.exchange(x)
    e1.record()
    e1.synchronize()
    pts = sum(int(i[1]) * int(i[3]) * (int(i[5]) - 1) for i in ctx.info)
    out["spatial_fp32"] = {"subdomains": ctx.nsub, "ms_per_eval": ms,
                           "local_point_steps_per_s": pts / (ms * 1e-3),
                           "pad_positions_per_box": int(ctx.info[0][9]),
                           "exchange_ms": e0.elapsed_time(e1) / reps,
                           "step_kernels": {0: "gather", 1: "column walk",
                                            2: "column walk, persistent forward"}[
                                                ctx.tz_kernels()["kind"]]}
    log(f"turkel-zwas on {ctx.nsub} boxes, fp32: {ms:.2f} ms/eval, exchange "
        f"{out['spatial_fp32']['exchange_ms']:.2f} ms")
    ctx.close()
    del ctx, x, J, g
    torch.cuda.empty_cache()
    return out


def time_evals(ctx, x, steps, warmup):
    import torch
    J = torch.empty(ctx.nsub, dtype=torch.float64, device="cuda")
    g = torch.empty(ctx.ctrl_len, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        ctx.cost_grad(x, J, g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.cost_grad(x, J, g)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, J, g


def step_distribution(ctx, x, steps):
    """Per-evaluation durations from HIP events on the launch stream (one
    pair per evaluation, after the timed run): median, p10, p90 in ms."""
    import torch
    J = torch.empty(ctx.nsub, dtype=torch.float64, device="cuda")
    g = torch.empty(ctx.ctrl_len, dtype=torch.float64, device="cuda")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for a, b in ev:
        a.record()
        ctx.cost_grad(x, J, g)
        b.record()
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    return {"median": float(np.median(t)), "p10": float(np.percentile(t, 10)),
            "p90": float(np.percentile(t, 90)), "n": int(steps)}


_POOL = {}


def _pool_eval(s):
    """One local cost+gradient evaluation in a forked worker (inputs inherited
    from the parent); returns (local point-steps, seconds)."""
    from oracle import local
    d = _POOL
    b = d["maps"].boxes[s]
    t0 = time.perf_counter()
    local.cost_grad(d["prob"], d["maps"], s, d["x"][s], d["trajs"][s][0], d["rings"][s],
                    {k: d["trajs"][k] for k in d["maps"].neighbors[s]})
    return b.ny * b.nx * (b.nlev - 1), time.perf_counter() - t0


def cpu_baseline(spec, budget_s=20.0):
    """The FP64 oracle timed on host cores over a bounded sample: whole local
    cost+gradient evaluations of first-interval subdomains of the workload,
    first in one process, then in a pool of forked processes (one per host
    core, at most 16) over further subdomains of the same sample.  Runs before
    the GPU is touched, so the workers inherit no device state."""
    import multiprocessing as mp
    from oracle import ddmaps, local, model
    g = model.Grid.of(spec)
    maps = ddmaps.build(spec.replace(obs_value=np.zeros(spec.nobs)))
    sample = [b.sub for b in maps.boxes if b.interval == 0 and b.ny == max(bb.ny for bb in maps.boxes)]
    lmax = max(maps.boxes[s].nlev for s in sample) - 1
    steps = sorted({int(k) for k in spec.obs_step if k <= lmax})
    truth = model.forward_at(g, spec.truth0, steps)
    pos = {k: i for i, k in enumerate(steps)}
    vals = np.full(spec.nobs, np.nan)
    sel = spec.obs_step <= lmax
    idx = np.array([pos[int(k)] for k in spec.obs_step[sel]])
    vals[sel] = (truth.reshape(len(steps), 3, -1)[idx, spec.obs_field[sel].astype(int),
                                                     spec.obs_cell[sel]]
                 + spec.obs_sigma[sel] * spec.obs_noise[sel])
    prob = spec.replace(obs_value=vals)   # later steps are never read by the sample
    bg = model.forward(g, spec.xb0, lmax)
    log(f"cpu baseline: oracle inputs ready ({len(sample)} candidate subdomains)")
    trajs, rings, xs = {}, {}, {}
    rng = np.random.default_rng(1)
    for s in sample:
        need = set(maps.neighbors[s].tolist()) | set(int(k) for k in maps.halo_src[s] if k >= 0)
        for k in need | {s}:
            if k not in trajs:
                trajs[k] = local.restrict_global(maps, k, bg)
        rings[s] = local.ring_from_trajs(maps, s, trajs)
        xs[s] = trajs[s][0] + 0.3 * spec.sigma_b[:, None, None] * rng.standard_normal(trajs[s][0].shape)
    _POOL.update(prob=prob, maps=maps, trajs=trajs, rings=rings, x=xs)
    # one process
    done = pts = 0
    t_total = 0.0
    for s in sample * 4:
        n, dt = _pool_eval(s)
        pts += n
        t_total += dt
        done += 1
        if t_total >= budget_s / 2:
            break
    single = pts / t_total
    log(f"cpu baseline: one process {single:.3e} local point-steps/s ({done} evaluations)")
    # a pool of forked processes over the subdomains of the sample, taken in
    # turn (again from the first when the sample is exhausted); the GPU machine
    # allots 16 host cores to its one GPU, whatever os.cpu_count() shows, so
    # the pool has at most 16 workers
    ncores = max(1, min(16, os.cpu_count() or 1))
    per_eval = t_total / done
    nwork = int(max(ncores, ncores * round(budget_s / 2 / per_eval))) if ncores > 1 else 0
    work = [sample[(done + i) % len(sample)] for i in range(nwork)]
    pool_rate, pool_wall = None, None
    if work:
        ctx = mp.get_context("fork")
        t0 = time.perf_counter()
        with ctx.Pool(ncores) as pool:
            res = pool.map(_pool_eval, work, chunksize=1)
        pool_wall = time.perf_counter() - t0
        pool_rate = sum(r[0] for r in res) / pool_wall
        log(f"cpu baseline: {ncores} processes {pool_rate:.3e} local point-steps/s "
            f"({len(work)} evaluations, {pool_wall:.1f} s)")
    box = maps.boxes[sample[0]]
    shape = f"{box.ny}x{box.nx}x{box.nlev - 1}-step"
    if pool_rate is not None:
        return dict(value=pool_rate, unit="local grid-point-steps/s", cores=ncores, kind="oracle",
                    sample=f"{len(work)} full local cost+gradient evaluations of first-interval "
                           f"{shape} subdomains of the same workload in {ncores} forked processes "
                           f"(NumPy FP64, {pool_wall:.1f} s wall)",
                    seconds=pool_wall,
                    single_process={"value": single, "cores": 1, "evaluations": done,
                                    "seconds": t_total})
    return dict(value=single, unit="local grid-point-steps/s", cores=1, kind="oracle",
                sample=f"{done} full local cost+gradient evaluations of first-interval {shape} "
                       f"subdomains of the same workload (NumPy FP64, one process, {t_total:.1f} s)",
                seconds=t_total)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c5")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the FP32-vs-FP64 DD solve (analysis error) leg")
    ap.add_argument("--no-gn", action="store_true",
                    help="skip the Gauss-Newton leg (normal-matrix product, GN solves)")
    ap.add_argument("--no-gn-solve", action="store_true",
                    help="time the Gauss-Newton normal-matrix product only")
    ap.add_argument("--no-tz", action="store_true",
                    help="skip the Turkel-Zwas leg (time decomposition of the same grid)")
    ap.add_argument("--no-diff", action="store_true",
                    help="skip the differentiation leg (autograd with checkpointing, config 4)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the whole path runs in-device on a single MI355X; "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        return 2

    import synth

    t0 = time.perf_counter()
    spec = synth.make_spec(args.config)
    cpu = None
    if not args.no_cpu:
        # before any device work: the worker processes are forked from here
        log("timing the oracle on host cores")
        cpu = cpu_baseline(spec, args.cpu_budget)
        cpu["host_cpu"] = _cpu_model()

    import torch
    from paper_2205_06649_amd.context import Context

    log(f"spec {args.config}: {spec.nlat}x{spec.nlon}x{spec.nsteps}, nobs={spec.nobs} "
        f"({time.perf_counter() - t0:.1f}s)")
    prob = synth.finish_spec(spec, gpu_truth_forward)
    log(f"truth run + observations done ({time.perf_counter() - t0:.1f}s)")

    ctx = Context(prob, "fp32")
    log(f"fp32 context: {ctx.nsub} subdomains ({time.perf_counter() - t0:.1f}s)")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2205)
    xb = ctx.background_controls()
    sb = torch.tensor(prob.sigma_b, dtype=torch.float64, device="cuda")
    scale = torch.cat([sb[f].expand(int(inf[1]) * int(inf[3])) for inf in ctx.info for f in range(3)])
    x = xb + 0.3 * scale * torch.randn(ctx.ctrl_len, generator=gen, dtype=torch.float64, device="cuda")

    # step kernels over all boxes per launch (mode 0), then the persistent
    # per-box sweeps (mode 2) when every box fits a workgroup: the faster
    # one is the headline
    # the library's autotuner times every execution plan that applies (HIP
    # graph replays) and keeps the fastest; the headline times K replays of
    # that plan, and the same plan launched eagerly is reported beside it
    ctx.set_graph(True)
    tune = ctx.autotune(x, reps=3)
    for i, c in enumerate(tune["candidates"]):
        log(f"autotune: mode {c['mode']} ({EXEC_MODES[c['mode']]}), passes {c['passes']}: "
            f"{c['ms']:.3f} ms/eval{'  <- chosen' if i == tune['chosen'] else ''}")
    mode = tune["candidates"][tune["chosen"]]["mode"]
    passes = tune["candidates"][tune["chosen"]]["passes"]
    ms, J32, g32 = time_evals(ctx, x, args.steps, args.warmup)
    log(f"fp32 graph replays, mode {mode}: {ms:.3f} ms/eval")
    dist = step_distribution(ctx, x, args.steps)
    log(f"per replay: median {dist['median']:.3f} ms, p10 {dist['p10']:.3f}, p90 {dist['p90']:.3f}")
    ctx.set_graph(False)
    ms_eager, _, _ = time_evals(ctx, x, args.steps, args.warmup)
    log(f"fp32 eager launches, mode {mode}: {ms_eager:.3f} ms/eval")
    fwd_b, adj_b, pts = algorithmic_bytes(ctx, 4, persistent=(mode >= 2))
    fwd_s, adj_s, _ = algorithmic_bytes(ctx, 4)

    def phase_timing(md, reps=10):
        # events around each sweep on the launch stream, after two untimed
        # evaluations (the first launches after idle run at lower clocks)
        ctx.set_exec_mode(md)
        ctx.set_timing(True)
        for _ in range(2):
            ctx.cost_grad(x, J32, g32)
        ctx.get_timing()
        for _ in range(reps):
            ctx.cost_grad(x, J32, g32)
        t = ctx.get_timing()
        ctx.set_timing(False)
        return t

    # phases from separate forward and adjoint launches (in the fused mode,
    # from the same kernels launched one sweep at a time)
    tm = phase_timing(2 if mode == 3 else mode)
    calls = tm["calls"]
    fwd_ms, adj_ms = tm["fwd_ms"] / calls, tm["adj_ms"] / calls
    if mode == 3:
        # the dominant kernel is the fused evaluation itself
        tf = phase_timing(3)
        kernel_ms = tf["fwd_ms"] / tf["fwd_launches"]
        kernel_bytes = fwd_b + adj_b
    else:
        kernel_ms = tm["adj_ms"] / tm["adj_launches"]
        kernel_bytes = adj_b / tm["adj_launches"] * calls
    achieved = kernel_bytes / (kernel_ms * 1e-3) / 1e9
    J32h, g32h = J32.cpu().numpy(), g32.cpu().numpy()
    # the exchange of Alg. 1 (once per outer iteration): every box integrated
    # from x, then rings and overlap targets from the new trajectories
    for _ in range(2):
        ctx.exchange(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        ctx.exchange(x)
    e1.record()
    e1.synchronize()
    exchange_ms = e0.elapsed_time(e1) / 5
    log(f"exchange: {exchange_ms:.3f} ms")
    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        a.fill_(1.0)
        b = a.clone()
        torch.cuda.synchronize()
        log(f"copy probe: {a.numel() * 4} bytes read and written by one clone")
        # partial cache lines: the first 32 B, then the first 64 B, of every
        # 128 B of the same 1 GiB, gathered into a packed copy (how the read
        # counter scales when a kernel uses part of each line it touches)
        for nb in (32, 64):
            c = a.view(-1, 32)[:, :nb // 4].contiguous()
            torch.cuda.synchronize()
            log(f"partial-line probe: {c.numel() * 4} bytes read ({nb} B of every 128 B) "
                f"and written packed")
            del c
        del a, b
    del ctx
    torch.cuda.empty_cache()

    result = {
        "metric": "fwd+adjoint grid-point-steps/s",
        "value": pts / (ms * 1e-3),
        "unit": "local grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"SWE on the sphere {prob.nlat}x{prob.nlon}, {prob.nsteps} steps, "
                        f"{len(J32h)} subdomains "
                        f"({int(len(prob.band_npieces))}x{int(prob.band_npieces[0])} space x "
                        f"{len(prob.time_edges) - 1} time), overlap {prob.overlap_cells} cells/"
                        f"{prob.overlap_steps} steps, {prob.nobs} obs; batched FP32 state, "
                        f"FP64 cost/gradient",
            "local_point_steps_per_eval": int(pts),
            "global_point_steps_per_eval": int(prob.nlat * prob.nlon * prob.nsteps),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": KERNEL_NAMES[mode] + {
                0: " (adjoint step, all subdomains per launch)",
                2: " (persistent adjoint sweep, one workgroup per box)",
                3: " (fused persistent forward + adjoint, one workgroup per box)",
                4: " (persistent adjoint sweep in column strips, one workgroup per box)"}[mode],
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(KERNEL_NAMES[mode] + (f"/{passes}" if mode >= 2 else ""),
                                        args.config),
            "algorithmic_bytes_per_launch": kernel_bytes,
            "bytes_model": ("step kernels: Z^n, lambda^{n+1}, lambda^{n+2} read, lambda^n "
                            "written per level" if mode == 0 else
                            "persistent: each level written once by the forward and read once "
                            "by the adjoint, adjoint vectors on chip"),
            "avg_launch_ms": kernel_ms,
        },
        "phases_ms": {"forward_sweep": fwd_ms, "adjoint_sweep": adj_ms,
                      "reduce": tm["reduce_ms"] / calls, "exchange": exchange_ms},
        "per_replay_ms": dist,
        "exec_mode": EXEC_MODES[mode],
        "autotune": tune,
        "timed": "HIP graph replays of the chosen plan",
        "eager_ms_per_step": ms_eager,
        "forward_sweep_GBs": fwd_b / (fwd_ms * 1e-3) / 1e9,
        "whole_eval_algorithmic_GBs": (fwd_b + adj_b) / (ms * 1e-3) / 1e9,
        # the same evaluation priced with the step-kernel byte model (every
        # level's adjoint vectors through HBM), for comparison across modes
        "whole_eval_step_model_GBs": (fwd_s + adj_s) / (ms * 1e-3) / 1e9,
        "global_point_steps_per_s": prob.nlat * prob.nlon * prob.nsteps / (ms * 1e-3),
    }

    if not args.no_fp64:
        ctx64 = Context(prob, "fp64")
        ms64, J64, g64 = time_evals(ctx64, x, max(2, args.steps // 4), 2)
        J64h, g64h = J64.cpu().numpy(), g64.cpu().numpy()
        ctx64.set_exec_mode(1)
        plain = []
        for _ in range(3):          # one launch per box per step: median of three
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ctx64.cost_grad(x)
            torch.cuda.synchronize()
            plain.append((time.perf_counter() - t1) * 1e3)
        ms_plain = float(np.median(plain))
        del ctx64
        torch.cuda.empty_cache()
        result["fp64_batched_ms"] = ms64
        result["fp64_plain_per_subdomain_ms"] = ms_plain
        result["fp64_plain_per_subdomain_runs_ms"] = plain
        result["speedup_vs_plain_fp64"] = ms_plain / ms
        result["speedup_vs_batched_fp64"] = ms64 / ms
        result["fp32_vs_fp64_rel_err"] = {
            "J_max": float(np.max(np.abs(J32h - J64h) / np.abs(J64h))),
            "grad_norm": float(np.linalg.norm(g32h - g64h) / np.linalg.norm(g64h)),
        }
        log(f"fp64 batched {ms64:.2f} ms, plain {ms_plain:.1f} ms")

    if not args.no_solve:
        result["solve"] = solve_leg(prob, mode)
    if not args.no_gn:
        result["gauss_newton"] = gn_leg(prob, x, mode, passes, args.config,
                                        solves=not args.no_gn_solve)
    if not args.no_tz:
        result["turkel_zwas"] = tz_leg(spec)
    if not args.no_diff:
        result["differentiation"] = differentiation_leg()
    if not args.no_solve:
        # last: its 8 large boxes leave the device memory in another state
        # than the legs above expect for their own allocations
        result["solve"]["few_boxes"] = few_boxes_solve_leg(spec)

    # the targets of this workload, stated beside what was measured
    frac = result["roofline"]["frac"]
    tg = {"hbm_roofline_frac": {"target": 0.6, "achieved": frac, "met": bool(frac >= 0.6)}}
    if "solve" in result:
        sv = result["solve"]
        tg["solve_gradient_reduction_fp64"] = {"target": SOLVE_TARGET,
                                              "achieved": sv["fp64"]["gnorm_ratio_max"],
                                              "met": sv["fp64"]["target_met"]}
        tg["fp32_analysis_rel_err"] = {"target": 1e-4, "achieved": sv["fp32_analysis_rel_err"],
                                       "met": bool(sv["fp32_analysis_rel_err"] <= 1e-4)}
    result["targets"] = tg

    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)
    return 0


def _cpu_model():
    """The host CPU as /proc/cpuinfo and the scheduler describe it."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                continue
            k, v = (t.strip() for t in line.split(":", 1))
            if k in ("model name", "cpu family", "model", "stepping", "cpu MHz", "cache size",
                     "cpu cores", "siblings") and k not in info:
                info[k] = v
    except OSError:
        pass
    info["os_cpu_count"] = os.cpu_count()
    try:
        info["affinity_cores"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    return info


if __name__ == "__main__":
    sys.exit(main())
