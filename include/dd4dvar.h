/*
 * dd4dvar.h -- C ABI of the MI355X space-time domain-decomposed 4D-Var engine.
 *
 * The library evaluates, for every space-time subdomain Delta_j x Omega_i of
 * a shallow-water-on-the-sphere problem, the regularized local 4D-Var
 * functional of the paper's local 4D-Var DA definition (eq. eq:cost:parallel1:
 * background term + observation misfit + overlap penalty) and its gradient,
 * all subdomains at once on one GPU, and runs the DD-4DVar outer loop
 * (Alg. 1) around it.
 *
 * Conventions shared by every call
 *   - Every call returns dd4dvar_status (0 = OK).  Nothing aborts and no C++
 *     exception crosses the ABI.  On failure, dd4dvar_last_error() describes
 *     the cause.
 *   - Fields are ordered (h, u, v).  Grid arrays are [field][lat][lon] with
 *     longitude fastest and latitude running south to north; a cell index is
 *     lat * nlon + lon.  h is the full fluid depth in metres.
 *   - Pointers named *_dev are device pointers owned by the caller (for
 *     example torch tensors); they must stay valid until the work queued on
 *     the given stream has completed.  Pointers without the suffix are host
 *     pointers, read before the call returns.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls marked "asynchronous" only enqueue work on that stream.
 *   - A context is not thread-safe; separate contexts are independent.
 *   - Packed control layout (FP64): the subdomains' controls concatenated in
 *     subdomain order, each [3][ny][nx] over its extended box, starting at
 *     the ctrl_offset reported by dd4dvar_plan_subdomain_info.
 *   - Packed trajectory layout (FP64): per subdomain [nlev][3][ny][nx],
 *     starting at traj_offset.
 */
#ifndef DD4DVAR_H
#define DD4DVAR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dd4dvar_ctx dd4dvar_ctx;    /* owns all device memory */
typedef struct dd4dvar_plan dd4dvar_plan;  /* host-only maps */

typedef enum {
  DD4DVAR_OK = 0,
  DD4DVAR_E_INVALID = 1,       /* bad descriptor or argument; nothing was done */
  DD4DVAR_E_NOMEM = 2,         /* device or host allocation failed */
  DD4DVAR_E_DEVICE = 3,        /* a HIP call failed; last_error holds its text */
  DD4DVAR_E_NONFINITE = 4,     /* NaN/Inf met in a cost or gradient (reported
                                  by dd4dvar_synchronize and dd4dvar_autotune) */
  DD4DVAR_E_NOTCONVERGED = 5,  /* iteration cap hit; outputs are still written */
  DD4DVAR_E_STATE = 6          /* call order violated (e.g. adjoint before forward) */
} dd4dvar_status;

typedef enum { DD4DVAR_FP64 = 0, DD4DVAR_FP32_STATE = 1 } dd4dvar_precision;

/* Grid and model (Sec. 7: SWE on the sphere, unstaggered centred scheme with
 * p = q = 1 and alpha = 0; leapfrog in time with a forward-Euler half
 * increment at the start of every local interval).  nlon must be even (the
 * row beyond a pole is the same row shifted by nlon/2 with u, v negated).
 * dlambda = 2 pi / nlon, dtheta = pi / nlat, cell-centred latitudes.
 * lambda_obs and mu_overlap are lambda of eq. min3sec and mu of
 * eq. eq:cost:parallel1.  precision selects the storage/arithmetic type of the
 * state sweeps (FP32_STATE stores h - h_ref); costs, gradients and all
 * reductions are FP64 in both modes.  weight_mode 0 weights squared terms by
 * 1/(number of boxes covering the point) (restriction weights of Def.
 * defrestrfun); 1 uses unit weights. */
typedef struct {
  int32_t nlat, nlon, nsteps;
  double dt, radius, gravity, omega, h_ref;
  double lambda_obs, mu_overlap;
  int32_t precision;
  int32_t weight_mode;
  /* Turkel-Zwas variant (Sec. 7, discrete U, V, H with offsets p, q and
   * averaging alpha): tz_p = 0 selects the plain scheme above (tz_q and
   * tz_alpha ignored).  tz_p >= 1 takes the pressure-gradient, divergence and
   * Coriolis terms over tz_p columns and tz_q rows, averaged with weight
   * tz_alpha over the points (i +- p, j), (i, j +- q) and the corners
   * (i +- p, j +- q); advection keeps offset one and H is the advective
   * form with h / cos on both divergence terms.  Requires
   * 1 <= tz_p <= nlon / 2, 1 <= tz_q <= nlat / 2, 0 <= tz_alpha <= 1, and
   * for bands of several pieces box width + 2 tz_p <= nlon.  Each box then
   * reads a frozen pad tz_q rows and tz_p columns wide, corners included
   * (see HALO_SRC), in place of the one-cell ring.  Such a context runs the
   * step kernels only (execution modes 0 and 1; the persistent modes return
   * E_INVALID), the tangent-linear and Gauss-Newton entry points included. */
  int32_t tz_p, tz_q;
  double tz_alpha;
} dd4dvar_model_desc;

/* Space-time partition DD(Delta x Omega) (Def. domdecom, eqs. Eq-r, nlocx).
 * band_lat_edges: [n_bands+1], 0 .. nlat strictly increasing.
 * band_npieces:   [n_bands], >= 1.
 * piece_lon_edges: per band npieces+1 edges 0 .. nlon, concatenated.
 * time_edges:     [n_time+1], 0 .. nsteps strictly increasing.
 * Each core grows by overlap_cells on every side (clipped at the poles,
 * wrapped in longitude; a band of one piece spans the circle) and each
 * interval by overlap_steps on each side (clipped to [0, nsteps], closed).
 * Requires overlap_cells <= every core height and multi-piece core width,
 * core width + 2 overlap_cells < nlon, overlap_steps <= every interval. */
typedef struct {
  int32_t n_bands;
  const int32_t* band_lat_edges;
  const int32_t* band_npieces;
  const int32_t* piece_lon_edges;
  int32_t n_time;
  const int32_t* time_edges;
  int32_t overlap_cells, overlap_steps;
} dd4dvar_partition_desc;

/* Background and observations (DA problem setup, Sec. 2).  xb0 is the
 * background initial state [3][nlat][nlon]; sigma_b the per-field background
 * standard deviations (diagonal B); each observation is one field at one
 * cell at one model step with its own standard deviation (diagonal R).
 * Observations must be finite and unique per (step, cell, field). */
typedef struct {
  const double* xb0;
  const double* sigma_b;
  int64_t nobs;
  const int32_t* obs_step;
  const int32_t* obs_cell;
  const int8_t* obs_field;
  const double* obs_value;
  const double* obs_sigma;
} dd4dvar_data_desc;

/* ---- host-only planning (no GPU needed) -------------------------------- */

/* Validates the descriptors and builds every index map (boxes, halo sources,
 * coverage counts, overlap neighbours, observation bins).  Copies all inputs.
 * Returns E_INVALID for bad descriptors, E_NOMEM on allocation failure. */
dd4dvar_status dd4dvar_plan_create(const dd4dvar_model_desc* model,
                                   const dd4dvar_partition_desc* part,
                                   const dd4dvar_data_desc* data,
                                   dd4dvar_plan** out);
void dd4dvar_plan_destroy(dd4dvar_plan* plan);

/* Number of subdomains and total packed control / trajectory lengths. */
dd4dvar_status dd4dvar_plan_sizes(const dd4dvar_plan* plan, int32_t* nsub,
                                  int64_t* ctrl_len, int64_t* traj_len);

/* out[10] = {row0, ny, col0, nx, step0, nlev, ctrl_offset, traj_offset,
 *            spans_all_lon, nring} of subdomain s (s = interval * nspace +
 * piece, pieces band-major).  The box covers global rows row0..row0+ny-1 and
 * columns (col0 + c) mod nlon, c < nx; levels step0..step0+nlev-1. */
dd4dvar_status dd4dvar_plan_subdomain_info(const dd4dvar_plan* plan, int32_t s,
                                           int64_t out[10]);

/* Integer maps for bit-exact checks.  kind:
 *   0 HALO_SRC   per s, [nring]: source subdomain of each ring position, -1
 *                when the position wraps inside the box.  Ring positions:
 *                south row (box row -1, cols 0..nx-1), north row (row ny),
 *                west column (col -1, rows 0..ny-1), east column (col nx).
 *                Under the Turkel-Zwas variant (offsets p, q) the pad: south
 *                block (rows -q..-1) and north block (rows ny..ny+q-1),
 *                row-major over cols -p..nx+p-1 (0..nx-1 for a box spanning
 *                the circle), then for other boxes the west block (rows
 *                0..ny-1, cols -p..-1) and east block (cols nx..nx+p-1),
 *                row-major.  A row beyond a pole maps to the row at the same
 *                depth on the other side, half a circle further.
 *   1 HALO_OFF   per s, [nring]: cell offset in the source box (or in the box
 *                itself for internal positions)
 *   2 HALO_SIGN  per s, [nring]: +1, or -1 across a pole (applies to u, v)
 *   3 COVER      per s, [ny*nx]: number of extended spatial boxes covering
 *                each box cell
 *   4 TIME_COUNT global, [nsteps+1]: number of extended intervals per level
 *   5 NEIGHBORS  per s: sorted subdomains whose extended space-time box
 *                intersects that of s
 *   6 OBS_BIN    per s: sorted indices of the observations inside s
 *   7 HALO_GCELL per s, [nring]: global cell read by each frozen position
 * With buf == NULL the required length is stored in *len; otherwise *len is
 * the capacity of buf (E_INVALID if too small) and receives the length. */
dd4dvar_status dd4dvar_plan_get_map(const dd4dvar_plan* plan, int32_t kind,
                                    int32_t s, int64_t* len, int32_t* buf);

/* Last error of a context, or of the calling thread's last plan/create call
 * when ctx is NULL.  The string stays valid until the next call. */
const char* dd4dvar_last_error(const dd4dvar_ctx* ctx);

/* ---- device context ------------------------------------------------------ */

/* Builds the plan, allocates the device arena on the current HIP device,
 * copies the inputs, runs the background model over the whole window in FP64
 * (Alg. 1, first step) and fills the frozen halo rings, overlap targets and
 * per-subdomain backgrounds from it.  Synchronous.  E_INVALID (with
 * dd4dvar_last_error(NULL) naming the cause) for an invalid descriptor, or when a
 * box overlaps more than 64 other space-time boxes (the overlap-target
 * kernel keeps one bit per neighbour in a 64-bit mask). */
dd4dvar_status dd4dvar_create(const dd4dvar_model_desc* model,
                              const dd4dvar_partition_desc* part,
                              const dd4dvar_data_desc* data, void* stream,
                              dd4dvar_ctx** out);
void dd4dvar_destroy(dd4dvar_ctx* ctx);

/* The plan owned by a context (valid until dd4dvar_destroy). */
const dd4dvar_plan* dd4dvar_ctx_plan(const dd4dvar_ctx* ctx);

/* Packed FP64 background controls x^b_s: the background trajectory at each
 * subdomain's first level on its box (eq. funrestr).  Asynchronous. */
dd4dvar_status dd4dvar_background_controls(dd4dvar_ctx* ctx, double* x_dev,
                                           void* stream);

/* The hot path.  For every subdomain s (or those listed in sub_ids, a host
 * array of nsub ids; NULL = all): J_s(x_s) of eq. eq:cost:parallel1 and its
 * gradient, from the packed FP64 controls x_dev.  Writes J_dev[s] (FP64, one
 * per subdomain, entries of unlisted subdomains untouched) and grad_dev
 * (packed FP64).  Runs the forward sweep, the observation and overlap misfits
 * and the adjoint sweep; the local trajectories are kept for
 * dd4dvar_adjoint_integrate.  Asynchronous: a NaN or Inf in any J_s or
 * gradient entry (for example from a non-finite control, or a time step
 * beyond the scheme's stability limit) sets the context's device flag,
 * which dd4dvar_synchronize reports as E_NONFINITE. */
dd4dvar_status dd4dvar_local_cost_grad(dd4dvar_ctx* ctx, int32_t nsub,
                                       const int32_t* sub_ids,
                                       const double* x_dev, double* J_dev,
                                       double* grad_dev, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * dd4dvar_local_cost_grad over all subdomains, the same kernels and results
 * bit for bit, allocating nothing.  The per-tile FP64 cost partials, which
 * local_cost_grad keeps in the context's arena, live in a static device
 * array of the library instead: 131072 tiles (1 MiB) per GPU, held by each
 * GPU the library runs on until the process ends; a decomposition with more
 * tiles of 256 box cells (more than ~33.5 M box cells) gets E_INVALID.  The
 * array's address is looked up once per device by dd4dvar_create.  Every
 * call on a GPU shares that GPU's array (each call writes every partial it
 * reads), so calls that overlap on one GPU, from any context or stream,
 * race.  Runs eagerly: graph mode and phase timing do not apply.
 * Asynchronous; the non-finite flag as for local_cost_grad. */
dd4dvar_status dd4dvar_local_cost_grad_noalloc(dd4dvar_ctx* ctx, const double* x_dev,
                                               double* J_dev, double* grad_dev,
                                               void* stream);

/* Forward model.  scope 0: the whole grid from x_dev = [3][nlat][nlon] over
 * all nsteps, traj_dev = [nsteps+1][3][nlat][nlon] (required), FP64 always.
 * scope 1: every subdomain's restricted model (eq. restricted) from packed
 * controls x_dev with its frozen halo ring, in the context precision;
 * traj_dev (nullable) receives the packed FP64 trajectories.  Asynchronous. */
dd4dvar_status dd4dvar_forward_integrate(dd4dvar_ctx* ctx, int32_t scope,
                                         const double* x_dev, double* traj_dev,
                                         void* stream);

/* Adjoint model of the last scope-1 forward (adjoint definition of Sec. 2,
 * run step by step in reverse, eq. adjProd).  forcing_dev: packed FP64
 * trajectory-shaped forcing, or NULL for the cost forcing (observation and
 * overlap misfits at the stored trajectory).  adj0_dev receives the packed
 * FP64 adjoint at each subdomain's first level (no background term).
 * scope must be 1.  E_STATE if no scope-1 forward ran.  Asynchronous. */
dd4dvar_status dd4dvar_adjoint_integrate(dd4dvar_ctx* ctx, int32_t scope,
                                         const double* forcing_dev,
                                         double* adj0_dev, void* stream);

/* Tangent linear model of the local sweeps (the TLM step of Alg. 6; the
 * linearized restricted model, eq. restricted) about the trajectories of the
 * last scope-1 forward (forward_integrate, local_cost_grad or exchange):
 * dZ = M' dx for every subdomain from the packed FP64 control perturbation
 * dx_dev; the frozen halo ring is not perturbed.  dtraj_dev (nullable)
 * receives the packed FP64 perturbation trajectories (every level, h as is).
 * Step kernels in every execution mode.  E_INVALID with checkpoints on,
 * E_STATE if no forward ran.  Asynchronous. */
dd4dvar_status dd4dvar_tangent_linear(dd4dvar_ctx* ctx, const double* dx_dev,
                                      double* dtraj_dev, void* stream);

/* Gauss-Newton normal matrix of each local functional (eqs. line5and7,
 * Eq_matrixAV:1) applied to dx_dev, about the trajectories of the last
 * scope-1 forward: out_dev = (B_w^{-1} + M'^T W M') dx_dev, with B_w^{-1}
 * the background weight w^b / sigma_b^2 per control entry and W the weights
 * of the observation and overlap residuals of J_s per trajectory entry.  The
 * tangent-linear sweep then the adjoint sweep forced by W dZ (packed FP64 in
 * and out, distinct buffers).  E_INVALID with checkpoints on or when
 * dx_dev == out_dev, E_STATE if no forward ran.  Asynchronous. */
dd4dvar_status dd4dvar_gn_hessvec(dd4dvar_ctx* ctx, const double* dx_dev,
                                  double* out_dev, void* stream);

/* Exchange (Alg. 1): integrates every subdomain from the packed controls
 * x_dev, then refreshes the frozen halo rings from the owners' trajectories
 * and the overlap targets from the neighbours' trajectories (each target the
 * mean of the other boxes holding the cell and level, summed in neighbour
 * list order; the spread around it goes into the cost constant).  The
 * result is deterministic: with checkpointing on, where the levels are
 * exchanged one at a time, it is the same bits.  Asynchronous. */
dd4dvar_status dd4dvar_exchange(dd4dvar_ctx* ctx, const double* x_dev,
                                void* stream);

/* Partition-of-unity gather (eq. rest) of the subdomains' trajectories from
 * the last scope-1 forward at one global level into out_dev [3][nlat][nlon]
 * (FP64).  Asynchronous. */
dd4dvar_status dd4dvar_gather(dd4dvar_ctx* ctx, int32_t level, double* out_dev,
                              void* stream);

/* Selects how local_cost_grad, forward_integrate (scope 1) and
 * adjoint_integrate launch their kernels:
 *   0 = one launch per time step over all subdomains (default);
 *   1 = one launch per subdomain per step (the plain baseline);
 *   2 = persistent sweeps: one workgroup per subdomain holds the current
 *       level in LDS and the level before it in registers, one launch per
 *       sweep over all subdomains;
 *   3 = as 2, but local_cost_grad over all subdomains is ONE launch in which
 *       each workgroup runs its box's forward and then its adjoint sweep
 *       (forward_integrate and adjoint_integrate as in 2);
 *   4 = as 2, with the adjoint in column strips: each thread walks one
 *       column of up to 11 consecutive rows of its box (needs
 *       ceil(ny / floor(1024 / nx)) <= 11 for every extended box).
 * Modes 2 to 4 need an FP32 context whose extended boxes all fit one
 * workgroup (at most 1024 columns, 11 passes of rows, and the padded level
 * frame with per-row tables and ring staging within 159 KB of LDS).
 * Results of modes 0 and 1 are identical bit for bit; modes 2 and 3 are
 * identical to each other, mode 4 runs their arithmetic (up to the
 * compiler's choice of fused multiply-adds) and sums J's FP64 terms in
 * another order; modes 2 to 4 differ from 0 and 1 by FP32 rounding only (the
 * overlap forcing is formed in FP32 there).  E_INVALID
 * for an unknown mode or for modes 2 to 4 where they do not apply.  The sub_ids form of
 * local_cost_grad always uses the step kernels. */
dd4dvar_status dd4dvar_set_exec_mode(dd4dvar_ctx* ctx, int32_t mode);

/* Execution plan with an explicit pass count: mode as for
 * dd4dvar_set_exec_mode; passes (modes 2 to 4) is the number of 1024-cell
 * passes the persistent forward and box-mapped adjoint are compiled for,
 * 0 = the smallest that holds the largest box, otherwise between that and
 * 11 (E_INVALID outside).  dd4dvar_set_exec_mode(ctx, m) equals
 * dd4dvar_set_exec_plan(ctx, m, 0).  The autotuner chooses among such
 * plans; this call pins one, for tests and measurement. */
dd4dvar_status dd4dvar_set_exec_plan(dd4dvar_ctx* ctx, int32_t mode, int32_t passes);

/* Step kernels of the Turkel-Zwas variant (Sec. 7 discrete U, V, H; its
 * adjoint by the definition of Sec. 2, eq. adjProd), forward and adjoint
 * sweeps: kind 0 = gather form, one thread per cell reading its 13-point
 * neighbourhood (and in the adjoint the state, adjoint and row coefficients
 * of its 12 readers), any p, q; kind 1 = column walk, one wave per block of
 * 64 - 2p columns walking a strip of rows with a five-row window of state
 * (and adjoint) per column in registers, q = 2 and p <= 8 only; kind 2 =
 * the column walk with the forward sweep as one persistent launch (one
 * workgroup per box for the whole interval, the level and its frozen pad
 * in LDS), FP32 state, every level stored (no checkpoints: with them the
 * context turns to kind 1), no box spanning the circle, every box's frame
 * within the LDS.  The default is the highest kind that applies.  The
 * global (whole-grid) forward runs always use kind 0.
 * Both kinds evaluate the same expressions in the same order (the adjoint's
 * per-cell sums in FP64); the column walk adds the observation forcing to
 * the adjoint state after it is rounded to the state precision (one more
 * rounding at observed cells) and keeps J's terms in other partial sums.
 * E_INVALID for another kind, or kind 1 where it does not apply. */
dd4dvar_status dd4dvar_set_tz_kernels(dd4dvar_ctx* ctx, int32_t kind);

/* out[2] = {Turkel-Zwas kernel kind in use, the highest kind that applies
 * (0 if the column walk does not)}. */
dd4dvar_status dd4dvar_get_tz_kernels(const dd4dvar_ctx* ctx, int32_t out[2]);

/* Vector work of the local solvers (the L-BFGS iteration of the remark
 * after Alg. 5, the Gauss-Newton updates of Alg. 5 with CG or the Lanczos
 * method of Alg. 7, and the background block of dd4dvar_gn_hessvec): every
 * box's packed control is cut into parts of `entries` entries (the last
 * part of a box shorter), one workgroup per part, and each per-box dot
 * product is the sum of its parts' partial sums in part order
 * (deterministic for a given part length; another length changes the
 * rounding of the sums only).  Default 16384; E_INVALID outside
 * [64, 2^24].  Waits for the device to be idle before it replaces the part
 * map; not to be called while another call on this context is running. */
dd4dvar_status dd4dvar_set_solver_parts(dd4dvar_ctx* ctx, int32_t entries);

/* out[2] = {entries per part, number of parts over all boxes}. */
dd4dvar_status dd4dvar_get_solver_parts(const dd4dvar_ctx* ctx, int32_t out[2]);

/* The plan in use: out[4] = {execution mode, pass count of the persistent
 * kernels (0 when they do not apply), rows per column strip of the mode-4
 * adjoint (0 when it does not apply), 1 if the persistent modes apply}. */
dd4dvar_status dd4dvar_get_exec_plan(const dd4dvar_ctx* ctx, int32_t out[4]);

/* Waits for the work queued on stream, then reads and clears the context's
 * non-finite flag: E_NONFINITE if any cost J_s, gradient entry, or
 * first-level adjoint entry (adjoint_integrate, gn_hessvec) computed since
 * the last check was NaN or Inf, else OK.  The flag is also read and cleared
 * by dd4dvar_autotune (which returns E_NONFINITE for it) and cleared by
 * dd4dvar_solve / dd4dvar_solve_mixed, whose line search meets overflowing
 * trial steps by design and checks its own iterates. */
dd4dvar_status dd4dvar_synchronize(dd4dvar_ctx* ctx, void* stream);

/* Storage of the local trajectories for the adjoint (Sec. 2 adjoint model;
 * square-root checkpointing of the forward states).  stride = 0 (default):
 * every level of every box is kept.  stride >= 3: only the level pairs
 * n = k stride, k stride + 1 are kept, plus one segment of stride - 2 levels
 * per box; the adjoint recomputes each segment from its pair, last segment
 * first, so a local cost/gradient costs one more forward sweep and the state
 * arena shrinks from L + 1 to about 2 (L / stride + 1) + stride - 2 levels per
 * box (smallest near stride = sqrt(2 L)).  Results are identical bit for bit
 * to stride 0.  The exchange then integrates the boxes in step by global
 * level and stages the new rings until the end.  gather is limited to levels
 * that every box covering them keeps (level 0 always), and forward_integrate
 * writes trajectory output level by level as it computes.  Not with the
 * persistent execution modes 2 and 3 (E_INVALID).  Reallocates the state
 * arena (synchronizes the device, drops recorded graphs) and clears the
 * stored forward (an adjoint needs a new forward: E_STATE).  *state_bytes
 * (nullable) receives the arena size. */
dd4dvar_status dd4dvar_set_checkpointing(dd4dvar_ctx* ctx, int32_t stride, int64_t* state_bytes);

/* Graph mode (on != 0): local_cost_grad over all subdomains (sub_ids NULL)
 * records its launches into a HIP graph the first time it meets a given
 * (x_dev, J_dev, grad_dev, execution plan) and replays that graph afterwards
 * (up to 8 graphs are kept; the oldest is dropped).  The graph reads the
 * buffers' contents at replay time, so new controls in the same buffer, an
 * exchange or a solve in between are all seen.  Calls with sub_ids, with
 * phase timing on, or inside dd4dvar_solve run eagerly.  Off by default. */
dd4dvar_status dd4dvar_set_graph(dd4dvar_ctx* ctx, int32_t on);

/* Autotuner of the execution plan of local_cost_grad: candidates are the
 * step kernels (mode 0) and, where the persistent sweeps apply, mode 2 with
 * the smallest pass count (1024 cells per pass) that holds the largest box,
 * mode 2 with the maximum pass count, mode 3, and mode 4 where it applies.
 * Each candidate evaluates
 * every subdomain at x_dev once untimed and then reps times (1..1000) between
 * HIP events on the stream, writing J_dev / grad_dev (caller's scratch, the
 * local_cost_grad layouts; in graph mode the replays are timed).  The fastest
 * becomes the context's plan; the report lists every candidate.  Blocks until
 * the timing is read.  Nothing is allocated on the device. */
typedef struct {
  int32_t ncand;        /* candidates timed (<= 8) */
  int32_t mode[8];      /* execution mode of each */
  int32_t passes[8];    /* pass count of the persistent kernels (0 for mode 0) */
  double ms[8];         /* milliseconds per evaluation */
  int32_t chosen;       /* index of the plan now in use */
} dd4dvar_tune_report;
dd4dvar_status dd4dvar_autotune(dd4dvar_ctx* ctx, const double* x_dev, double* J_dev,
                                double* grad_dev, int32_t reps, void* stream,
                                dd4dvar_tune_report* report);

/* Phase timing of local_cost_grad, for measurement: when on, every call
 * records HIP events on its stream around the forward sweep, the adjoint
 * sweep and the final reduction.  dd4dvar_get_timing waits for them and
 * returns, summed over the calls since the last query, out[6] = {forward ms,
 * adjoint ms, reduction ms, forward launches, adjoint launches, calls}, then
 * clears the record. */
dd4dvar_status dd4dvar_set_timing(dd4dvar_ctx* ctx, int32_t on);
dd4dvar_status dd4dvar_get_timing(dd4dvar_ctx* ctx, double out[6]);

/* ---- DD-4DVar solve (Alg. 1) --------------------------------------------- */
typedef struct {
  int32_t lbfgs_m;      /* stored pairs (8) */
  int32_t max_iter;     /* L-BFGS iterations per local solve */
  int32_t max_outer;    /* outer DD sweeps */
  int32_t max_ls;       /* Armijo trials per iteration (30) */
  double grad_rtol;     /* stop a local solve at |g| <= grad_rtol |g0| */
  double outer_tol;     /* stop when max_s |xi_s - xi_s_prev|_inf < outer_tol */
  double armijo_c1;     /* 1e-4 */
  double j_noise_rtol;  /* evaluation noise floor of J, relative (0 = off): a
                           local solve stops when the decrease a step can
                           still show, alpha |g^T d|, is at most
                           j_noise_rtol |J| (FP32 state: J carries ~1e-7
                           relative rounding noise, and backtracking below it
                           only burns evaluations) */
  int32_t local_solver; /* 0 = L-BFGS (default); 1 = Gauss-Newton (Alg. 5 /
                           Alg. 6): max_iter full updates per local solve,
                           each solving the normal equations of eq. line5and7
                           in xi by conjugate gradients from zero; stops at
                           |g| <= grad_rtol |g0| like L-BFGS; needs every
                           level stored (no checkpoints), else E_INVALID */
  int32_t cg_max_iter;  /* CG iterations per Gauss-Newton update (>= 0) */
  double cg_rtol;       /* CG stop at |r| <= cg_rtol |r0| (also stops when the
                           curvature p^T A p is not positive) */
  int32_t krylov;       /* solver of the Gauss-Newton normal equations: 0 = CG,
                           1 = Lanczos (Alg. 7): the same caps and stop tests,
                           the CG iterates in exact arithmetic; keeps its basis
                           (cg_max_iter vectors of the control length, FP64)
                           and reports Ritz values; needs local_solver = 1 */
} dd4dvar_solve_opts;

typedef struct {
  int32_t outer_iters, total_evals;
  int32_t lbfgs_iters;       /* local iterations (L-BFGS or Gauss-Newton), the
                                maximum over subdomains summed over sweeps */
  int32_t gn_products;       /* batched normal-matrix products (CG iterations) */
  double J_final;            /* sum over subdomains of the final local J */
  double gnorm_ratio_max;    /* max_s |g_s| / |g_s,0| at the end */
  double seconds;
  double ritz_min, ritz_max; /* Lanczos: smallest and largest Ritz value of the
                                preconditioned normal matrices over the
                                subdomains' last runs (0 otherwise) */
} dd4dvar_solve_report;

/* Runs Alg. 1 from x_init_dev (packed controls, NULL = background): batched
 * local solves (L-BFGS, or Gauss-Newton with CG or Lanczos, see local_solver
 * and krylov) over all subdomains in xi = (x - x^b_s) / sigma_b, then
 * forward, exchange and the outer stop test; finally the partition-of-unity
 * gather of level 0 into xa_host [3][nlat][nlon].  From NULL the halo rings
 * and overlap targets are first reset to those of the background run; from
 * given controls the solve continues with the rings and targets of the last
 * exchange (or the background, before any).  x_out_dev (nullable) receives
 * the final packed controls.  Synchronous.  E_NOTCONVERGED when max_outer was
 * reached without meeting outer_tol (outputs are written). */
dd4dvar_status dd4dvar_solve(dd4dvar_ctx* ctx, const dd4dvar_solve_opts* opts,
                             const double* x_init_dev, double* x_out_dev,
                             double* xa_host, dd4dvar_solve_report* report);

/* Mixed-precision Gauss-Newton solve (Alg. 1 with the local solver of
 * Alg. 5 / Alg. 6): ctx (FP64) evaluates every J_s and gradient, the stop
 * tests, the exchange and the gather; ctx_lo, an FP32-state context created
 * from the same descriptors on the same device, integrates each iterate
 * again in FP32 and supplies the normal-matrix products of the conjugate
 * gradients from its own sweeps (persistent ones in its execution modes 2 to
 * 4).  An inexact Newton method: the iterates converge to the stationary
 * point of the FP64 functionals while most of the sweeps run in FP32.  opts
 * as for dd4dvar_solve with local_solver = 1; both contexts are exchanged at
 * every outer iteration.  E_INVALID for another local solver, wrong
 * precisions, differing plans or devices, or checkpoints on either context.
 * Synchronous; outputs as for dd4dvar_solve. */
dd4dvar_status dd4dvar_solve_mixed(dd4dvar_ctx* ctx, dd4dvar_ctx* ctx_lo,
                                   const dd4dvar_solve_opts* opts,
                                   const double* x_init_dev, double* x_out_dev,
                                   double* xa_host, dd4dvar_solve_report* report);

#ifdef __cplusplus
}
#endif
#endif /* DD4DVAR_H */
