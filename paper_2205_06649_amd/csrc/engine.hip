// Device context of the DD 4D-Var engine: arena layout, uploads, the
// background run, and the C ABI entry points that enqueue the sweeps.
//
// All subdomains live in device memory for the whole run (the paper keeps
// every work array resident on the device before processing; here all of
// them share one GPU).  Per subdomain s:
//   state     [nlev][3][ny][nx]  T     (h stored as h - h_ref)
//   targets   [nlev][3][ny][nx]  T     (mean neighbour trajectory)
//   ring      [nlev][3][nring]   T     (frozen halo, signs applied)
//   adjoint   [3 slots][3][ny][nx] T   (rolling levels of the adjoint sweep)
// plus FP64 background controls, per-cell coverage counts (uint8), the
// observation lists binned per (256-cell tile, level), and FP64 per-tile
// cost accumulators.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.h"
#include "launch.h"
#include "gn.h"
#include "plan.h"
#include "solve.h"

using namespace dd4dvar;

namespace dd4dvar {
dd4dvar_status solve_impl(dd4dvar_ctx* ctx, const dd4dvar_solve_opts* opts, const double* x_init,
                          double* x_out, double* xa_host, dd4dvar_solve_report* rep,
                          dd4dvar_ctx* lo);
}

struct DeviceArrays {
  std::vector<void*> owned;
  ~DeviceArrays() {
    for (void* p : owned) (void)hipFree(p);
  }
};

struct dd4dvar_ctx {
  dd4dvar_plan plan;
  std::string err;
  int device = 0;
  int prec = 0;
  int exec_mode = 0;
  bool have_forward = false;
  int ntiles = 0, maxlev = 0, ring_blocks = 1, nsub = 0;
  std::vector<SubDev> subs;
  std::vector<int2> tiles;
  SubDev* d_subs = nullptr;
  int2* d_tiles = nullptr;
  void *traj = nullptr, *ring = nullptr, *targ = nullptr, *adj = nullptr;
  void *rows = nullptr, *cosx = nullptr;
  RowCoef<double>* rows64 = nullptr;
  double* cosx64 = nullptr;
  uint8_t* cover = nullptr;
  int32_t* tcount = nullptr;
  int32_t *obs_ptr = nullptr, *obs_code = nullptr;
  double *obs_val = nullptr, *obs_q = nullptr;
  double *jpart = nullptr, *jc = nullptr, *jconst = nullptr;
  // per-tile cost partials in use: jpart, or the device's static scratch
  // during dd4dvar_local_cost_grad_noalloc
  double* jpart_use = nullptr;
  double* scratch = nullptr;            // this device's static scratch array
  int32_t *nbr_idx = nullptr, *hsrc = nullptr, *hoff = nullptr, *hsign = nullptr, *hgcell = nullptr;
  double* xb = nullptr;
  int32_t *cptr = nullptr, *cpiece = nullptr;
  int32_t* d_ids = nullptr;
  uint32_t* nonfinite = nullptr;
  const uint8_t* eval_mask = nullptr;   // subdomains evaluated by the sweeps (null = all)
  bool box_ok = false;                  // persistent per-box sweeps possible
  size_t box_lds = 0;
  int box_k = 0;                        // passes of 1024 cells of the launches
  int box_kmin = 0;                     // passes that hold the largest box
  bool box_span = false;                // some box spans the circle
  int strip_k = 0;                      // rows per column strip of the strip adjoint (0: n/a)
  // Turkel-Zwas variant (tz_p > 0): step kernels only
  int tz_p = 0, tz_q = 1;
  double tz_alpha = 0;
  // column-walk adjoint of the variant (q = 2): work list of every box's
  // waves (box by box), each box's range in it, available / in use
  TzWork* tz_work = nullptr;
  int tz_nwork = 0;
  std::vector<int> tz_work_box;
  // the forward's waves (shorter strips: no J slots; more waves in flight)
  TzWork* tz_fwork = nullptr;
  std::vector<int> tz_fwork_box;
  // per local level, the tiles with observation entries there (CSR)
  int32_t* tz_obs_tiles = nullptr;
  std::vector<int> tz_obs_ptr;
  bool tz_col_ok = false, tz_col = false;
  // persistent forward of the variant (FP32, no box spanning the circle):
  // available / in use, LDS bytes of the largest frame, cells of the
  // largest box
  bool tz_box_ok = false, tz_box = false;
  size_t tz_box_lds = 0;
  int tz_box_cells = 0;
  // the solvers' vector work: every box's control cut into parts of
  // part_len entries
  PartMap parts{};
  int part_len = 0;
  // state storage: every level (ckpt = 0), or checkpoint pairs every ckpt
  // levels plus one segment that the adjoint recomputes
  int ckpt = 0;
  int nslot = 0;                        // slots per box with checkpoints
  int32_t* d_zslot = nullptr;           // slot of each local level
  int32_t* d_zslot_id = nullptr;        // identity (every level stored; global runs)
  void* ring_next = nullptr;            // exchange staging for the rings (with checkpoints)
  void* dz = nullptr;                   // tangent-linear trajectory, every level (first use)
  size_t traj_bytes = 0, ring_bytes = 0;
  std::vector<int32_t> h_order;         // boxes, longest first
  int32_t* d_order = nullptr;
  // the whole grid as one box (FP64), for background and global runs
  SubDev gsub{};
  int gtiles = 0;
  SubDev* d_gsub = nullptr;
  int2* d_gtiles = nullptr;
  double st = 0, stg = 0;
  // optional phase timing: events recorded around the sweeps of each
  // local_cost_grad on the caller's stream
  bool timing = false;
  struct Mark {
    hipEvent_t ev[4];
    int nfwd, nadj;
  };
  std::vector<Mark> marks;
  // graph mode: local_cost_grad over all subdomains recorded once per
  // (x, J, grad, execution plan) into a HIP graph and replayed
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;     // recording stream (the caller's may be the null stream)
  struct GraphEntry {
    hipGraph_t graph;
    hipGraphExec_t exec;
    const double* x;
    double *J, *grad;
    int mode, passes;
  };
  std::vector<GraphEntry> graphs;
  DeviceArrays mem;
  ~dd4dvar_ctx() {
    for (Mark& m : marks)
      for (hipEvent_t e : m.ev) (void)hipEventDestroy(e);
    for (GraphEntry& g : graphs) {
      (void)hipGraphExecDestroy(g.exec);
      (void)hipGraphDestroy(g.graph);
    }
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

namespace {

// Static scratch of dd4dvar_local_cost_grad_noalloc: the per-tile FP64 cost
// partials of one evaluation (1 MiB: 131072 tiles of 256 cells, 33.5 M box
// cells).  Each GPU the library runs on holds its own copy until the process
// ends.  In host code the array's name is only a stand-in: its device
// address is looked up once per device (with that device current) and kept.
constexpr int64_t kScratchTiles = 131072;
__device__ __align__(256) double scratch[kScratchTiles];

std::mutex scratch_mu;
std::map<int, double*> scratch_addr;   // device -> address of its scratch

struct DevError {
  dd4dvar_status st;
  std::string msg;
};

void chk(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
      throw DevError{DD4DVAR_E_NOMEM, std::string(what) + ": " + hipGetErrorString(e)};
    throw DevError{DD4DVAR_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e)};
  }
}

template <typename P>
P* dalloc(dd4dvar_ctx* c, size_t count) {
  if (count == 0) count = 1;
  void* p = nullptr;
  chk(hipMalloc(&p, count * sizeof(P)), "hipMalloc");
  c->mem.owned.push_back(p);
  return static_cast<P*>(p);
}

template <typename P>
P* upload(dd4dvar_ctx* c, const std::vector<P>& v, hipStream_t st) {
  P* d = dalloc<P>(c, v.size());
  if (!v.empty()) chk(hipMemcpyAsync(d, v.data(), v.size() * sizeof(P), hipMemcpyHostToDevice, st), "upload");
  return d;
}

// the solvers' part map: every box's control cut into parts of len entries
// (the last part of a box ragged); replaces an earlier map, whose buffers are
// released once the device is idle
void build_parts(dd4dvar_ctx* c, int len, hipStream_t st) {
  std::vector<Part> parts;
  std::vector<int2> boxp(c->subs.size());
  for (size_t s = 0; s < c->subs.size(); ++s) {
    const SubDev& S = c->subs[s];
    const int n = 3 * S.ncell;
    boxp[s] = make_int2(int(parts.size()), (n + len - 1) / len);
    for (int lo = 0; lo < n; lo += len)
      parts.push_back(Part{S.ctrl_off, S.cell_off, int32_t(s), S.ncell, lo, std::min(lo + len, n)});
  }
  if (c->parts.part) {
    chk(hipDeviceSynchronize(), "sync");
    auto& owned = c->mem.owned;
    for (void* q : {(void*)c->parts.part, (void*)c->parts.box, (void*)c->parts.acc}) {
      owned.erase(std::remove(owned.begin(), owned.end(), q), owned.end());
      chk(hipFree(q), "hipFree");
    }
  }
  c->parts.part = upload(c, parts, st);
  c->parts.box = upload(c, boxp, st);
  c->parts.nparts = int(parts.size());
  c->parts.acc = dalloc<double>(c, size_t(kPartSlots) * parts.size());
  c->part_len = len;
  // the host vectors are pageable: the copies complete before they go
  chk(hipStreamSynchronize(st), "sync");
}

template <typename T>
Dom<T> local_dom(const dd4dvar_ctx* c) {
  Dom<T> D{};
  D.subs = c->d_subs;
  D.tiles = c->d_tiles;
  D.traj = static_cast<T*>(c->traj);
  D.ring = static_cast<T*>(c->ring);
  D.targ = static_cast<T*>(c->targ);
  D.adj = static_cast<T*>(c->adj);
  D.dz = static_cast<T*>(c->dz);
  D.rows = static_cast<const RowCoef<T>*>(c->rows);
  D.cosx = static_cast<const T*>(c->cosx);
  D.cover = c->cover;
  D.tcount = c->tcount;
  D.obs_ptr = c->obs_ptr;
  D.obs_code = c->obs_code;
  D.obs_val = c->obs_val;
  D.obs_q = c->obs_q;
  D.jpart = c->jpart_use ? c->jpart_use : c->jpart;
  D.nbr_idx = c->nbr_idx;
  D.hsrc = c->hsrc;
  D.hoff = c->hoff;
  D.hsign = c->hsign;
  D.hgcell = c->hgcell;
  D.active = c->eval_mask;
  D.nonfinite = c->nonfinite;
  D.zslot = c->d_zslot;
  D.st = T(c->st);
  D.stg = T(c->stg);
  D.h0 = T(c->plan.model.h_ref);
  D.mu = c->plan.model.mu_overlap;
  for (int f = 0; f < 3; ++f) D.isb2[f] = 1.0 / (c->plan.sigma_b[f] * c->plan.sigma_b[f]);
  D.nlon = c->plan.model.nlon;
  D.half = c->plan.model.nlon / 2;
  D.maxlev = c->maxlev;
  D.weight_mode = c->plan.model.weight_mode;
  return D;
}

Dom<double> global_dom(const dd4dvar_ctx* c, double* traj) {
  Dom<double> D{};
  D.subs = c->d_gsub;
  D.tiles = c->d_gtiles;
  D.traj = traj;
  D.zslot = c->d_zslot_id;
  D.rows = c->rows64;
  D.cosx = c->cosx64;
  D.st = c->st;
  D.stg = c->stg;
  D.h0 = c->plan.model.h_ref;
  D.nlon = c->plan.model.nlon;
  D.half = c->plan.model.nlon / 2;
  D.weight_mode = c->plan.model.weight_mode;
  return D;
}

template <typename T>
void fill_rows(const dd4dvar_model_desc& m, std::vector<RowCoef<T>>& rows, std::vector<T>& cosx) {
  const double dth = M_PI / m.nlat, dla = 2.0 * M_PI / m.nlon;
  const double sl = m.dt / (m.radius * dla), st = m.dt / (m.radius * dth);
  rows.resize(m.nlat);
  cosx.resize(m.nlat + 2);
  std::vector<double> c(m.nlat);
  for (int j = 0; j < m.nlat; ++j) {
    const double th = -M_PI / 2 + (j + 0.5) * dth;
    c[j] = std::cos(th);
    RowCoef<T>& r = rows[j];
    r.a1 = T(sl / c[j]);
    r.a2 = T(sl * m.gravity / c[j]);
    r.a3 = T(st / c[j]);
    r.cf = T(2.0 * m.dt * 2.0 * m.omega * std::sin(th));
    r.ct = T(2.0 * m.dt * std::tan(th) / m.radius);
    r.c = T(c[j]);
  }
  cosx[0] = T(c[0]);
  for (int j = 0; j < m.nlat; ++j) cosx[j + 1] = T(c[j]);
  cosx[m.nlat + 1] = T(c[m.nlat - 1]);
}

// The column-walk waves of the boxes whose tiles are [tile_base, tile_base +
// ntiles) (a run of whole boxes: every box, one interval's, or one box);
// none when the column walk is off
void tz_work_range(const dd4dvar_ctx* c, int tile_base, int ntiles, const TzWork** work, int* nwork,
                   bool forward = false) {
  *work = nullptr;
  *nwork = 0;
  if (!c->tz_col) return;
  const std::vector<int>& wb = forward ? c->tz_fwork_box : c->tz_work_box;
  TzWork* base = forward ? c->tz_fwork : c->tz_work;
  size_t s0 = c->subs.size(), s1 = c->subs.size();
  for (size_t s = 0; s < c->subs.size(); ++s) {
    if (c->subs[s].tile0 == tile_base) s0 = s;
    if (c->subs[s].tile0 + c->subs[s].ntile == tile_base + ntiles) s1 = s;
  }
  if (s0 == c->subs.size() || s1 == c->subs.size() || s1 < s0)
    throw DevError{DD4DVAR_E_INVALID, "sweep launch over a tile range that is not a run of boxes"};
  *work = base + wb[s0];
  *nwork = wb[s1 + 1] - wb[s0];
}

// One forward and one adjoint step of the step kernels in the scheme that the
// model selects (plain centred, or Turkel-Zwas); global: the whole-grid run
// (gather kernels only)
template <typename T>
void fwd_step(const dd4dvar_ctx* c, const Dom<T>& D, int n, int tile_base, int ntiles, hipStream_t st,
              bool global = false) {
  if (c->tz_p > 0) {
    const TzWork* work = nullptr;
    int nwork = 0;
    if (!global) tz_work_range(c, tile_base, ntiles, &work, &nwork, true);
    launch_fwd_tz<T>(D, n, tile_base, ntiles, c->tz_p, c->tz_q, c->tz_alpha, c->plan.model.nlat,
                     work, nwork, st);
  } else {
    launch_fwd<T>(D, n, tile_base, ntiles, st);
  }
}

template <typename T>
void adj_step(const dd4dvar_ctx* c, const Dom<T>& D, int n, int tile_base, int ntiles, int mode,
              const double* x, const double* forcing, double* out, hipStream_t st) {
  if (c->tz_p > 0) {
    // the column-walk kernel takes the waves of the launched boxes
    const TzWork* work = nullptr;
    int nwork = 0;
    tz_work_range(c, tile_base, ntiles, &work, &nwork);
    const int32_t* otiles = nullptr;
    int nobs = 0;
    if (work) {
      otiles = c->tz_obs_tiles + c->tz_obs_ptr[n];
      nobs = c->tz_obs_ptr[n + 1] - c->tz_obs_ptr[n];
    }
    launch_adj_tz<T>(D, n, tile_base, ntiles, mode, c->tz_p, c->tz_q, c->tz_alpha,
                     c->plan.model.nlat, x, c->xb, forcing, out, work, nwork, otiles, nobs, st);
  } else {
    launch_adj<T>(D, n, tile_base, ntiles, mode, x, c->xb, forcing, out, st);
  }
}

// Global forward run (FP64) of x (device [3][ncell], full h) into traj
// ([nsteps+1][3][ncell], h stored as an anomaly).
void global_forward(dd4dvar_ctx* c, const double* x, double* traj, hipStream_t st) {
  Dom<double> G = global_dom(c, traj);
  launch_init<double>(G, x, 0, c->gtiles, st);
  for (int n = 0; n < c->plan.model.nsteps; ++n) fwd_step<double>(c, G, n, 0, c->gtiles, st, true);
  chk(hipGetLastError(), "global forward launch");
}

// local forward sweeps of every box; traj_out (nullable) receives the packed
// FP64 trajectory, level by level as it is computed when levels share slots
template <typename T>
void local_forward(dd4dvar_ctx* c, const double* x, hipStream_t st, double* traj_out = nullptr) {
  Dom<T> D = local_dom<T>(c);
  if constexpr (std::is_same<T, float>::value) {
    if (c->tz_p > 0 && c->tz_box && c->ckpt == 0) {
      chk(launch_fwd_tz_box(D, x, c->d_order, c->nsub, c->tz_box_lds, c->tz_box_cells, c->tz_p,
                            c->tz_q, c->tz_alpha, c->plan.model.nlat, st),
          "persistent Turkel-Zwas forward launch");
      if (traj_out) launch_traj_out<T>(D, traj_out, 0, c->ntiles, -1, st);
      c->have_forward = true;
      return;
    }
    if (c->exec_mode >= 2) {
      chk(launch_fwd_box(D, x, c->d_order, c->nsub, c->box_lds, c->box_k, c->box_span, st),
          "persistent forward launch");
      if (traj_out) launch_traj_out<T>(D, traj_out, 0, c->ntiles, -1, st);
      c->have_forward = true;
      return;
    }
  }
  const bool per_level = traj_out && c->ckpt;
  auto sweep = [&](int tile_base, int ntiles, int nlev) {
    launch_init<T>(D, x, tile_base, ntiles, st);
    if (per_level) launch_traj_out<T>(D, traj_out, tile_base, ntiles, 0, st);
    for (int n = 0; n + 1 < nlev; ++n) {
      fwd_step<T>(c, D, n, tile_base, ntiles, st);
      if (per_level) launch_traj_out<T>(D, traj_out, tile_base, ntiles, n + 1, st);
    }
  };
  if (c->exec_mode != 1) {
    sweep(0, c->ntiles, c->maxlev);
  } else {
    for (const SubDev& S : c->subs) sweep(S.tile0, S.ntile, S.nlev);
  }
  if (traj_out && !per_level) launch_traj_out<T>(D, traj_out, 0, c->ntiles, -1, st);
  chk(hipGetLastError(), "forward launch");
  c->have_forward = true;
}

template <typename T>
void local_adjoint(dd4dvar_ctx* c, int mode, const double* x, const double* forcing, double* out,
                   const std::vector<int32_t>* ids, hipStream_t st) {
  Dom<T> D = local_dom<T>(c);
  if constexpr (std::is_same<T, float>::value) {
    if (!ids && c->exec_mode >= 2) {
      const bool strip = c->exec_mode == 4;
      chk(launch_adj_box(D, mode, x, c->xb, forcing, out, c->d_order, c->nsub, c->box_lds,
                         strip ? c->strip_k : c->box_k, c->box_span, strip, st),
          "persistent adjoint launch");
      return;
    }
  }
  // adjoint levels lmax .. 0 of a tile range; with checkpoints, segment by
  // segment from the last, each first recomputed from its checkpoint pair
  // (levels lo, lo+1) into the shared segment slots
  auto levels = [&](int tile_base, int ntiles, int lmax) {
    const int cs = c->ckpt;
    if (cs == 0) {
      for (int n = lmax; n >= 0; --n)
        adj_step<T>(c, D, n, tile_base, ntiles, mode, x, forcing, out, st);
      return;
    }
    for (int lo = (lmax / cs) * cs; lo >= 0; lo -= cs) {
      const int hi = std::min(lo + cs - 1, lmax);
      for (int n = lo + 1; n < hi; ++n) fwd_step<T>(c, D, n, tile_base, ntiles, st);
      for (int n = hi; n >= lo; --n)
        adj_step<T>(c, D, n, tile_base, ntiles, mode, x, forcing, out, st);
    }
  };
  if (!ids && c->exec_mode != 1) {
    levels(0, c->ntiles, c->maxlev - 1);
  } else {
    auto run = [&](const SubDev& S) { levels(S.tile0, S.ntile, S.nlev - 1); };
    if (ids)
      for (int32_t s : *ids) run(c->subs[s]);
    else
      for (const SubDev& S : c->subs) run(S);
  }
  chk(hipGetLastError(), "adjoint launch");
}

// tangent-linear trajectory arena (every level, the layout of the state
// arena without checkpoints), allocated on first use
void ensure_dz(dd4dvar_ctx* c) {
  if (c->dz) return;
  const size_t tsz = c->prec == DD4DVAR_FP64 ? sizeof(double) : sizeof(float);
  c->dz = dalloc<char>(c, size_t(c->plan.traj_total) * tsz + kBoxArenaTail);
}

// tangent-linear sweeps of every box (or of the boxes in c->eval_mask) about
// the stored trajectory: dZ = M' dx, every level into the dz arena (the
// persistent per-box kernel in modes 2 and 3, else the step kernels)
template <typename T>
void local_tlm(dd4dvar_ctx* c, const double* dx, hipStream_t st) {
  ensure_dz(c);
  Dom<T> D = local_dom<T>(c);
  if constexpr (std::is_same<T, float>::value) {
    if (c->exec_mode >= 2) {
      chk(launch_tlm_box(D, dx, c->d_order, c->nsub, c->box_lds, c->box_k, c->box_span, st),
          "persistent tangent-linear launch");
      return;
    }
  }
  auto sweep = [&](int tile_base, int ntiles, int nlev) {
    launch_tlm_init<T>(D, dx, tile_base, ntiles, st);
    const TzWork* work = nullptr;
    int nwork = 0;
    if (c->tz_p > 0) tz_work_range(c, tile_base, ntiles, &work, &nwork, true);
    for (int n = 0; n + 1 < nlev; ++n) {
      if (c->tz_p > 0)
        launch_tlm_tz<T>(D, n, tile_base, ntiles, c->tz_p, c->tz_q, c->tz_alpha, c->plan.model.nlat,
                         work, nwork, st);
      else
        launch_tlm<T>(D, n, tile_base, ntiles, st);
    }
  };
  if (c->exec_mode != 1) {
    sweep(0, c->ntiles, c->maxlev);
  } else {
    for (const SubDev& S : c->subs) sweep(S.tile0, S.ntile, S.nlev);
  }
  chk(hipGetLastError(), "tangent-linear launch");
}

// M'^T W M' dx (no background block): the tangent-linear sweep, then the
// adjoint sweep forced by the observation and overlap weights applied to dZ
template <typename T>
void gn_product(dd4dvar_ctx* c, const double* dx, double* out, hipStream_t st) {
  local_tlm<T>(c, dx, st);
  local_adjoint<T>(c, 3, nullptr, nullptr, out, nullptr, st);
}

void mark(dd4dvar_ctx* c, int which, hipStream_t st) {
  if (!c->timing) return;
  if (which == 0) {
    dd4dvar_ctx::Mark m{};
    for (hipEvent_t& e : m.ev) chk(hipEventCreate(&e), "hipEventCreate");
    c->marks.push_back(m);
  }
  chk(hipEventRecord(c->marks.back().ev[which], st), "hipEventRecord");
}

template <typename T>
void cost_grad_impl(dd4dvar_ctx* c, const std::vector<int32_t>* ids, const double* x, double* J,
                    double* grad, hipStream_t st) {
  Dom<T> D = local_dom<T>(c);
  mark(c, 0, st);
  if constexpr (std::is_same<T, float>::value) {
    if (!ids && c->exec_mode == 3) {
      // one fused persistent launch: each workgroup runs its box's forward
      // sweep and then its adjoint sweep
      chk(launch_eval_box(D, x, c->xb, grad, c->d_order, c->nsub, c->box_lds, c->box_k, c->box_span,
                          st),
          "persistent evaluation launch");
      c->have_forward = true;
      mark(c, 1, st);
      mark(c, 2, st);
      launch_reduce_j(c->d_subs, c->nsub, nullptr, D.jpart, c->jconst, J, c->nonfinite, st);
      chk(hipGetLastError(), "reduce launch");
      mark(c, 3, st);
      if (c->timing) {
        c->marks.back().nfwd = 1;       // the fused launch is timed as the forward phase
        c->marks.back().nadj = 0;
      }
      return;
    }
  }
  if (ids) {
    for (int32_t s : *ids) {
      const SubDev& S = c->subs[s];
      launch_init<T>(D, x, S.tile0, S.ntile, st);
      for (int n = 0; n + 1 < S.nlev; ++n) fwd_step<T>(c, D, n, S.tile0, S.ntile, st);
    }
    chk(hipGetLastError(), "forward launch");
    c->have_forward = true;
  } else {
    local_forward<T>(c, x, st);
  }
  mark(c, 1, st);
  local_adjoint<T>(c, 0, x, nullptr, grad, ids, st);
  mark(c, 2, st);
  if (ids) {
    // the id list lives in pageable host memory owned by the caller's frame:
    // wait for the copy before returning
    chk(hipMemcpyAsync(c->d_ids, ids->data(), ids->size() * sizeof(int32_t), hipMemcpyHostToDevice, st),
        "ids upload");
    chk(hipStreamSynchronize(st), "ids upload sync");
    launch_reduce_j(c->d_subs, int(ids->size()), c->d_ids, D.jpart, c->jconst, J, c->nonfinite, st);
  } else {
    launch_reduce_j(c->d_subs, c->nsub, nullptr, D.jpart, c->jconst, J, c->nonfinite, st);
  }
  chk(hipGetLastError(), "reduce launch");
  mark(c, 3, st);
  if (c->timing) {
    int nf = 0, na = 0;
    if (!ids && (c->exec_mode == 2 || c->exec_mode == 4) && std::is_same<T, float>::value) {
      nf = na = 1;                      // one persistent launch per sweep
    } else if (!ids && c->exec_mode == 0) {
      nf = c->maxlev;
      na = c->maxlev;
    } else {
      for (const SubDev& S : c->subs)
        if (!ids || std::find(ids->begin(), ids->end(), int32_t(&S - c->subs.data())) != ids->end()) {
          nf += S.nlev;
          na += S.nlev;
        }
    }
    c->marks.back().nfwd = nf;
    c->marks.back().nadj = na;
  }
}

// Exchange when levels share slots: the boxes advance in step by global
// level, interval by interval, and every level's rings and targets are taken
// as soon as all intervals hold it.  The forward keeps using the rings of the
// previous exchange (as the local solves did): the new ones are written to a
// staging arena that replaces the rings at the end.
template <typename T>
void exchange_lockstep(dd4dvar_ctx* c, const double* x, hipStream_t st) {
  const dd4dvar_plan& P = c->plan;
  Dom<T> D = local_dom<T>(c);
  Dom<T> Dn = D;
  Dn.ring = static_cast<T*>(c->ring_next);
  const int nsp = P.nspace, ntm = P.ntime;
  std::vector<int> tb(ntm), nt(ntm), lev0(ntm), nlev(ntm);
  for (int j = 0; j < ntm; ++j) {
    const SubDev& A = c->subs[j * nsp];
    const SubDev& B = c->subs[(j + 1) * nsp - 1];
    tb[j] = A.tile0;
    nt[j] = B.tile0 + B.ntile - A.tile0;
    lev0[j] = A.lev0;
    nlev[j] = A.nlev;
  }
  launch_init<T>(D, x, 0, c->ntiles, st);
  for (int g = 0; g <= P.model.nsteps; ++g) {
    for (int j = 0; j < ntm; ++j) {
      const int n = g - lev0[j];
      if (n >= 1 && n < nlev[j]) fwd_step<T>(c, D, n - 1, tb[j], nt[j], st);
    }
    for (int j = 0; j < ntm; ++j) {
      const int n = g - lev0[j];
      if (n < 0 || n >= nlev[j]) continue;
      launch_ring_from_local<T>(Dn, j * nsp, nsp, c->ring_blocks, n, st);
      launch_targets_from_local<T>(D, n, tb[j], nt[j], c->jc, st);
    }
  }
  launch_reduce_jconst(c->d_subs, c->nsub, c->jc, 0.5 * P.model.mu_overlap, c->jconst, st);
  chk(hipGetLastError(), "exchange launch");
  // every frozen ring entry of every level has been staged; copied (not
  // swapped) so that recorded graphs keep pointing at the live rings
  chk(hipMemcpyAsync(c->ring, c->ring_next, c->ring_bytes, hipMemcpyDeviceToDevice, st), "ring copy");
  c->have_forward = true;
}

template <typename T>
void exchange_impl(dd4dvar_ctx* c, const double* x, hipStream_t st) {
  if (c->ckpt) {
    exchange_lockstep<T>(c, x, st);
    return;
  }
  local_forward<T>(c, x, st);
  Dom<T> D = local_dom<T>(c);
  launch_ring_from_local<T>(D, 0, c->nsub, c->ring_blocks, -1, st);
  launch_targets_from_local<T>(D, -1, 0, c->ntiles, c->jc, st);   // every level
  launch_reduce_jconst(c->d_subs, c->nsub, c->jc, 0.5 * c->plan.model.mu_overlap, c->jconst, st);
  chk(hipGetLastError(), "exchange launch");
}

template <typename T>
void background_impl(dd4dvar_ctx* c, hipStream_t st) {
  const dd4dvar_model_desc& m = c->plan.model;
  const int64_t ncell = int64_t(m.nlat) * m.nlon;
  double* x0 = nullptr;
  double* bg = nullptr;
  chk(hipMalloc(&x0, size_t(3 * ncell) * sizeof(double)), "hipMalloc background");
  hipError_t e = hipMalloc(&bg, size_t(m.nsteps + 1) * 3 * ncell * sizeof(double));
  if (e != hipSuccess) {
    (void)hipFree(x0);
    chk(e, "hipMalloc background trajectory");
  }
  try {
    chk(hipMemcpyAsync(x0, c->plan.xb0.data(), size_t(3 * ncell) * sizeof(double),
                       hipMemcpyHostToDevice, st), "upload xb0");
    global_forward(c, x0, bg, st);
    Dom<T> D = local_dom<T>(c);
    for (int n = 0; n < c->maxlev; ++n) launch_from_global<T>(D, bg, ncell, c->xb, n, c->ntiles, st);
    launch_ring_from_global<T>(D, c->nsub, c->ring_blocks, bg, ncell, st);
    launch_fill(c->jconst, c->nsub, 0.0, st);
    chk(hipGetLastError(), "background launch");
    chk(hipStreamSynchronize(st), "background sync");
  } catch (...) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(x0);
    (void)hipFree(bg);
    throw;
  }
  chk(hipFree(x0), "hipFree");
  chk(hipFree(bg), "hipFree");
}

void build_device(dd4dvar_ctx* c, hipStream_t st) {
  const dd4dvar_plan& P = c->plan;
  const dd4dvar_model_desc& m = P.model;
  c->prec = m.precision;
  c->nsub = P.nsub;
  const size_t tsz = c->prec == DD4DVAR_FP64 ? sizeof(double) : sizeof(float);
  chk(hipGetDevice(&c->device), "hipGetDevice");
  {
    // this device's static scratch (set-up of the no-allocation entry point)
    std::lock_guard<std::mutex> lock(scratch_mu);
    auto it = scratch_addr.find(c->device);
    if (it == scratch_addr.end()) {
      void* ptr = nullptr;
      chk(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
      it = scratch_addr.emplace(c->device, static_cast<double*>(ptr)).first;
    }
    c->scratch = it->second;
  }

  // subdomain table and tiles
  int64_t ring_off = 0, adj_off = 0;
  int tile = 0, maxring = 0;
  c->maxlev = 0;
  c->subs.resize(P.nsub);
  for (int s = 0; s < P.nsub; ++s) {
    const BoxInfo& b = P.boxes[s];
    SubDev& S = c->subs[s];
    S.row0 = b.row0; S.ny = b.ny; S.col0 = b.col0; S.nx = b.nx;
    S.lev0 = b.lev0; S.nlev = b.nlev;
    S.span = b.span; S.pole_s = b.pole_s; S.pole_n = b.pole_n;
    S.ncell = int32_t(b.ncell());
    S.nring = b.nring;
    S.tile0 = tile;
    S.ntile = int32_t((b.ncell() + kTile - 1) / kTile);
    S.nbr0 = int32_t(P.nbr_ptr[s]);
    S.nbr1 = int32_t(P.nbr_ptr[s + 1]);
    if (S.nbr1 - S.nbr0 > 64)
      throw DevError{DD4DVAR_E_INVALID, "a box overlaps more than 64 others (exchange limit)"};
    S.pad_ = 0;
    S.traj_off = b.traj_off;
    S.zoff = b.traj_off;
    S.ring_off = ring_off;
    S.adj_off = adj_off;
    S.ctrl_off = b.ctrl_off;
    S.cell_off = P.cell_ptr[s];
    S.hmap_off = P.ring_ptr[s];
    ring_off += int64_t(b.nlev) * 3 * b.nring;
    adj_off += int64_t(9) * b.ncell();
    tile += S.ntile;
    c->maxlev = std::max(c->maxlev, b.nlev);
    maxring = std::max(maxring, b.nring);
  }
  c->ntiles = tile;
  c->ring_blocks = (maxring + 255) / 256;
  // persistent per-box sweeps: FP32, every box within one workgroup's cells
  // and LDS; boxes run longest first
  {
    size_t lds = 0;
    int kmax = 0;
    bool ok = c->prec == DD4DVAR_FP32_STATE && c->plan.model.tz_p == 0;
    int strip = 0;
    for (const SubDev& S : c->subs) {
      const int rs = box_strip_rows(S.ny, S.nx, S.nring, S.nlev);
      strip = (rs == 0 || strip < 0) ? -1 : std::max(strip, rs);
      lds = std::max(lds, box_lds_bytes(S.ny, S.nx, S.nring, S.nlev));
      const int k = box_passes(S.ny, S.nx, S.nring, S.nlev);
      if (k == 0) ok = false;
      kmax = std::max(kmax, k);
      if (S.span) c->box_span = true;
    }
    c->box_ok = ok;
    c->strip_k = (ok && strip > 0) ? strip : 0;
    c->box_lds = lds;
    c->box_k = kmax;
    c->box_kmin = kmax;
    // LDS limits of the persistent kernels are set here, outside any stream
    // capture, for the pass counts the context can run
    if (ok) {
      chk(box_prepare(kmax), "persistent kernel set-up");
      chk(box_prepare(box_passes_max()), "persistent kernel set-up");
    }
    std::vector<int32_t> order(P.nsub);
    for (int s = 0; s < P.nsub; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return int64_t(c->subs[a].ncell) * c->subs[a].nlev > int64_t(c->subs[b].ncell) * c->subs[b].nlev;
    });
    c->h_order = order;
  }
  c->tiles.resize(tile);
  for (int s = 0; s < P.nsub; ++s)
    for (int t = 0; t < c->subs[s].ntile; ++t) c->tiles[c->subs[s].tile0 + t] = make_int2(s, t);

  // whole-grid box
  SubDev& G = c->gsub;
  G = SubDev{};
  G.row0 = 0; G.ny = m.nlat; G.col0 = 0; G.nx = m.nlon;
  G.lev0 = 0; G.nlev = m.nsteps + 1; G.span = 1; G.pole_s = 1; G.pole_n = 1;
  G.ncell = m.nlat * m.nlon;
  G.nring = 0;
  G.ntile = (G.ncell + kTile - 1) / kTile;
  c->gtiles = G.ntile;
  std::vector<int2> gt(G.ntile);
  for (int t = 0; t < G.ntile; ++t) gt[t] = make_int2(0, t);

  // coefficient tables
  const double dth = M_PI / m.nlat;
  c->st = m.dt / (m.radius * dth);
  c->stg = c->st * m.gravity;
  std::vector<RowCoef<double>> r64;
  std::vector<double> c64;
  fill_rows<double>(m, r64, c64);

  // coverage (uint8) and observation bins per (tile, level)
  std::vector<uint8_t> cover(P.cover_box.size());
  for (size_t i = 0; i < cover.size(); ++i) {
    if (P.cover_box[i] > 255) throw DevError{DD4DVAR_E_INVALID, "coverage count above 255"};
    cover[i] = uint8_t(P.cover_box[i]);
  }
  const int64_t nkeys = int64_t(tile) * c->maxlev;
  std::vector<int32_t> optr(nkeys + 1, 0);
  const int nlon = m.nlon;
  auto key_of = [&](int s, int64_t k, int* loc_out) {
    const BoxInfo& b = P.boxes[s];
    const int64_t cell = P.obs_cell[k];
    const int row = int(cell / nlon), col = int(cell % nlon);
    int cc = col - b.col0;
    if (cc < 0) cc += nlon;
    const int loc = (row - b.row0) * b.nx + cc;
    *loc_out = loc;
    const SubDev& S = c->subs[s];
    return obs_key(S.tile0, S.ntile, c->maxlev, loc / kTile, P.obs_step[k] - b.lev0);
  };
  for (int s = 0; s < P.nsub; ++s)
    for (int64_t q = P.obs_ptr[s]; q < P.obs_ptr[s + 1]; ++q) {
      int loc;
      optr[key_of(s, P.obs_idx[q], &loc) + 1] += 1;
    }
  for (int64_t k = 0; k < nkeys; ++k) optr[k + 1] += optr[k];
  const int64_t nent = optr[nkeys];
  std::vector<int32_t> ocode(nent);
  std::vector<double> oval(nent), oq(nent);
  {
    std::vector<int32_t> fillp(optr.begin(), optr.end() - 1);
    for (int s = 0; s < P.nsub; ++s) {
      const BoxInfo& b = P.boxes[s];
      for (int64_t q = P.obs_ptr[s]; q < P.obs_ptr[s + 1]; ++q) {
        const int64_t k = P.obs_idx[q];
        int loc;
        const int64_t key = key_of(s, k, &loc);
        const int32_t pos = fillp[key]++;
        const int f = P.obs_field[k];
        ocode[pos] = loc * 4 + f;
        oval[pos] = f == 0 ? P.obs_value[k] - m.h_ref : P.obs_value[k];
        double w = 1.0;
        if (m.weight_mode == 0)
          w = 1.0 / (double(P.cover_box[P.cell_ptr[s] + loc]) * double(P.time_count[P.obs_step[k]]));
        oq[pos] = m.lambda_obs * w / (P.obs_sigma[k] * P.obs_sigma[k]);
        (void)b;
      }
    }
  }

  // coverage CSR per global cell for the gather
  const int64_t ncell = int64_t(m.nlat) * m.nlon;
  std::vector<int32_t> cptr(ncell + 1, 0);
  for (int64_t g = 0; g < ncell; ++g) cptr[g + 1] = cptr[g] + P.cover_sp[g];
  std::vector<int32_t> cpiece(cptr[ncell]);
  {
    std::vector<int32_t> f(cptr.begin(), cptr.end() - 1);
    for (int i = 0; i < P.nspace; ++i) {
      const BoxInfo& b = P.boxes[i];
      for (int r = 0; r < b.ny; ++r)
        for (int cc = 0; cc < b.nx; ++cc) {
          int col = b.col0 + cc;
          if (col >= nlon) col -= nlon;
          const int64_t g = int64_t(b.row0 + r) * nlon + col;
          cpiece[f[g]++] = i;
        }
    }
  }

  // uploads
  c->d_subs = upload(c, c->subs, st);
  build_parts(c, kPartLen, st);
  c->d_tiles = upload(c, c->tiles, st);
  c->d_order = upload(c, c->h_order, st);
  c->d_gsub = upload(c, std::vector<SubDev>{G}, st);
  {
    std::vector<int32_t> id(std::max<int>(c->maxlev, m.nsteps + 1));
    for (size_t i = 0; i < id.size(); ++i) id[i] = int32_t(i);
    c->d_zslot_id = upload(c, id, st);
    c->d_zslot = c->d_zslot_id;
  }
  c->d_gtiles = upload(c, gt, st);
  c->rows64 = upload(c, r64, st);
  c->cosx64 = upload(c, c64, st);
  if (c->prec == DD4DVAR_FP64) {
    c->rows = c->rows64;
    c->cosx = c->cosx64;
  } else {
    std::vector<RowCoef<float>> r32;
    std::vector<float> c32;
    fill_rows<float>(m, r32, c32);
    c->rows = upload(c, r32, st);
    c->cosx = upload(c, c32, st);
  }
  c->cover = upload(c, cover, st);
  c->tcount = upload(c, P.time_count, st);
  c->obs_ptr = upload(c, optr, st);
  c->obs_code = upload(c, ocode, st);
  c->obs_val = upload(c, oval, st);
  c->obs_q = upload(c, oq, st);
  c->nbr_idx = upload(c, P.nbr_idx, st);
  c->hsrc = upload(c, P.halo_src, st);
  c->hoff = upload(c, P.halo_off, st);
  c->hsign = upload(c, P.halo_sign, st);
  c->hgcell = upload(c, P.halo_gcell, st);
  c->cptr = upload(c, cptr, st);
  c->cpiece = upload(c, cpiece, st);
  c->jpart = dalloc<double>(c, tile);
  c->jc = dalloc<double>(c, tile);
  c->jconst = dalloc<double>(c, P.nsub);
  c->xb = dalloc<double>(c, P.ctrl_total);
  c->d_ids = dalloc<int32_t>(c, P.nsub);
  c->nonfinite = dalloc<uint32_t>(c, 1);
  chk(hipMemsetAsync(c->nonfinite, 0, sizeof(uint32_t), st), "memset");
  // large arenas
  c->traj_bytes = size_t(P.traj_total) * tsz;
  c->traj = dalloc<char>(c, c->traj_bytes + kBoxArenaTail);
  c->targ = dalloc<char>(c, size_t(P.traj_total) * tsz + kBoxArenaTail);
  c->ring_bytes = size_t(std::max<int64_t>(ring_off, 1)) * tsz;
  c->ring = dalloc<char>(c, c->ring_bytes);
  c->adj = dalloc<char>(c, size_t(std::max<int64_t>(adj_off, 1)) * tsz);
  if (P.model.tz_p > 0) {
    c->tz_p = P.model.tz_p;
    c->tz_q = P.model.tz_q;
    c->tz_alpha = P.model.tz_alpha;
    // column-walk kernels (q = 2, p <= 8): each box in column blocks of
    // 64 - 2p outputs and row strips (a strip reloads the four rows around
    // it): at least 32 rows for the adjoint, with at most one wave per
    // 256-cell tile of the box (each wave owns one J slot of the box), and
    // at least 16 for the forward (more waves in flight)
    if (c->tz_q == 2 && c->tz_p <= 8) {
      const int cw = 64 - 2 * c->tz_p;
      // waves of every box with strips of at least rmin rows; false when some
      // box has more column blocks than tiles
      auto build_list = [&](int rmin, std::vector<TzWork>& wl, std::vector<int>& wb) {
        wb.assign(c->subs.size() + 1, 0);
        for (size_t s = 0; s < c->subs.size(); ++s) {
          const SubDev& S = c->subs[s];
          wb[s] = int(wl.size());
          const int ncb = (S.nx + cw - 1) / cw;
          if (ncb > S.ntile) return false;
          const int maxstrips = S.ntile / ncb;
          const int R = std::max(rmin, (S.ny + maxstrips - 1) / maxstrips);
          const int nstr = (S.ny + R - 1) / R;
          int j = 0;
          for (int cb = 0; cb < ncb; ++cb)
            for (int k = 0; k < nstr; ++k, ++j) {
              TzWork w{};
              w.box = int32_t(s);
              w.c0 = cb * cw;
              w.r0 = k * R;
              w.r1 = std::min(S.ny, (k + 1) * R);
              w.slot = S.tile0 + j;
              w.zero0 = w.zero1 = 0;
              if (j == 0) {
                w.zero0 = S.tile0 + ncb * nstr;
                w.zero1 = S.tile0 + S.ntile;
              }
              wl.push_back(w);
            }
        }
        wb.back() = int(wl.size());
        return !wl.empty();
      };
      std::vector<TzWork> wl, fl;
      std::vector<int> wb, fb;
      if (build_list(32, wl, wb) && build_list(16, fl, fb)) {
        std::vector<int> otp(c->maxlev + 1, 0);
        std::vector<int32_t> otl;
        for (int n = 0; n < c->maxlev; ++n) {
          otp[n] = int(otl.size());
          for (const SubDev& S : c->subs)
            for (int t = 0; t < S.ntile; ++t) {
              const int64_t key = obs_key(S.tile0, S.ntile, c->maxlev, t, n);
              if (optr[key + 1] > optr[key]) otl.push_back(S.tile0 + t);
            }
        }
        otp[c->maxlev] = int(otl.size());
        c->tz_obs_tiles = upload(c, otl, st);
        c->tz_obs_ptr = otp;
        c->tz_work = upload(c, wl, st);
        c->tz_nwork = int(wl.size());
        c->tz_work_box = wb;
        c->tz_fwork = upload(c, fl, st);
        c->tz_fwork_box = fb;
        c->tz_col_ok = c->tz_col = true;
      }
    }
    if (c->prec == DD4DVAR_FP32_STATE) {
      bool ok = !c->subs.empty();
      size_t lds = 0;
      int cells = 0;
      for (const SubDev& S : c->subs) {
        const size_t b = tz_box_lds_bytes(S.nx, S.ny, c->tz_p, c->tz_q);
        // the pad layout the frame fill assumes: q rows of nx + 2p above and
        // below the box, p columns either side of each box row
        const int pads = 2 * c->tz_q * (S.nx + 2 * c->tz_p) + 2 * S.ny * c->tz_p;
        ok = ok && !S.span && S.nring == pads && tz_box_fits(S.ncell, S.nring, b);
        lds = std::max(lds, b);
        cells = std::max(cells, S.ncell);
      }
      if (ok) {
        chk(prepare_fwd_tz_box(), "persistent Turkel-Zwas forward set-up");
        // the default with the column walk
        c->tz_box_ok = true;
        c->tz_box = c->tz_col;
        c->tz_box_lds = lds;
        c->tz_box_cells = cells;
      }
    }
  }
  chk(hipMemsetAsync(c->ring, 0, size_t(std::max<int64_t>(ring_off, 1)) * tsz, st), "memset ring");
  chk(hipMemsetAsync(c->targ, 0, size_t(P.traj_total) * tsz, st), "memset targets");
  chk(hipStreamSynchronize(st), "upload sync");

  if (c->prec == DD4DVAR_FP64) background_impl<double>(c, st);
  else background_impl<float>(c, st);
}

// reads and clears the context's non-finite flag after the stream's work
bool take_nonfinite(dd4dvar_ctx* c, hipStream_t st) {
  uint32_t h = 0;
  chk(hipMemcpyAsync(&h, c->nonfinite, sizeof(uint32_t), hipMemcpyDeviceToHost, st), "read flag");
  chk(hipStreamSynchronize(st), "sync");
  if (h) {
    chk(hipMemsetAsync(c->nonfinite, 0, sizeof(uint32_t), st), "clear flag");
    chk(hipStreamSynchronize(st), "sync");
  }
  return h != 0;
}

dd4dvar_status fail(dd4dvar_ctx* c, dd4dvar_status s, const std::string& msg) {
  if (c) c->err = msg;
  else set_thread_error(msg);
  return s;
}

// local_cost_grad of every subdomain, eagerly or (graph mode) by replaying
// the graph recorded for these pointers and this execution plan; recorded on
// a stream of the context's own (the caller's may be the null stream, which
// cannot be captured) and launched on the caller's
void eval_all(dd4dvar_ctx* c, const double* x, double* J, double* grad, hipStream_t st) {
  auto eager = [&](hipStream_t s) {
    if (c->prec == DD4DVAR_FP64)
      cost_grad_impl<double>(c, nullptr, x, J, grad, s);
    else
      cost_grad_impl<float>(c, nullptr, x, J, grad, s);
  };
  if (!c->use_graph || c->timing || c->eval_mask) {
    eager(st);
    return;
  }
  dd4dvar_ctx::GraphEntry* hit = nullptr;
  for (dd4dvar_ctx::GraphEntry& g : c->graphs)
    if (g.x == x && g.J == J && g.grad == grad && g.mode == c->exec_mode && g.passes == c->box_k)
      hit = &g;
  if (!hit) {
    if (!c->cap_stream) chk(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "stream");
    hipGraph_t g = nullptr;
    chk(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    try {
      eager(c->cap_stream);
    } catch (...) {
      (void)hipStreamEndCapture(c->cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    chk(hipStreamEndCapture(c->cap_stream, &g), "end capture");
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      chk(e, "graph instantiate");
    }
    if (c->graphs.size() >= 8) {              // a small cache: drop the oldest
      (void)hipGraphExecDestroy(c->graphs.front().exec);
      (void)hipGraphDestroy(c->graphs.front().graph);
      c->graphs.erase(c->graphs.begin());
    }
    c->graphs.push_back({g, ex, x, J, grad, c->exec_mode, c->box_k});
    hit = &c->graphs.back();
  }
  chk(hipGraphLaunch(hit->exec, st), "graph launch");
  c->have_forward = true;
}

#define API_GUARD(ctx, ...)                                    \
  try {                                                        \
    __VA_ARGS__                                                \
  } catch (const DevError& e) {                                \
    return fail(ctx, e.st, e.msg);                             \
  } catch (const std::bad_alloc&) {                            \
    return fail(ctx, DD4DVAR_E_NOMEM, "host allocation failed"); \
  }

}  // namespace

extern "C" {

dd4dvar_status dd4dvar_create(const dd4dvar_model_desc* model, const dd4dvar_partition_desc* part,
                              const dd4dvar_data_desc* data, void* stream, dd4dvar_ctx** out) {
  if (!out) return fail(nullptr, DD4DVAR_E_INVALID, "null output pointer");
  *out = nullptr;
  dd4dvar_ctx* c = new (std::nothrow) dd4dvar_ctx();
  if (!c) return fail(nullptr, DD4DVAR_E_NOMEM, "host allocation failed");
  std::string err;
  dd4dvar_status s = build_plan(model, part, data, &c->plan, &err);
  if (s != DD4DVAR_OK) {
    delete c;
    return fail(nullptr, s, err);
  }
  try {
    build_device(c, static_cast<hipStream_t>(stream));
  } catch (const DevError& e) {
    delete c;
    return fail(nullptr, e.st, e.msg);
  } catch (const std::bad_alloc&) {
    delete c;
    return fail(nullptr, DD4DVAR_E_NOMEM, "host allocation failed");
  }
  set_thread_error("");
  *out = c;
  return DD4DVAR_OK;
}

void dd4dvar_destroy(dd4dvar_ctx* ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  delete ctx;
}

const dd4dvar_plan* dd4dvar_ctx_plan(const dd4dvar_ctx* ctx) { return ctx ? &ctx->plan : nullptr; }

const char* dd4dvar_last_error(const dd4dvar_ctx* ctx) {
  return ctx ? ctx->err.c_str() : thread_error();
}

dd4dvar_status dd4dvar_set_exec_mode(dd4dvar_ctx* ctx, int32_t mode) {
  if (!ctx || mode < 0 || mode > 4) return fail(ctx, DD4DVAR_E_INVALID, "bad exec mode");
  if (mode == 4 && ctx->box_ok && ctx->strip_k == 0)
    return fail(ctx, DD4DVAR_E_INVALID, "the column-strip adjoint needs at most 11 rows per strip");
  if (mode >= 2 && !ctx->box_ok)
    return fail(ctx, DD4DVAR_E_INVALID,
                "persistent per-box sweeps need FP32 state and boxes that fit one workgroup's LDS");
  if (mode >= 2 && ctx->ckpt)
    return fail(ctx, DD4DVAR_E_INVALID, "persistent per-box sweeps store every level (checkpoints on)");
  ctx->exec_mode = mode;
  if (mode >= 2) ctx->box_k = ctx->box_kmin;
  return DD4DVAR_OK;
}

dd4dvar_status dd4dvar_set_exec_plan(dd4dvar_ctx* ctx, int32_t mode, int32_t passes) {
  if (!ctx) return fail(ctx, DD4DVAR_E_INVALID, "null context");
  if (passes != 0 && (mode < 2 || mode > 4 || !ctx->box_ok || passes < ctx->box_kmin ||
                      passes > box_passes_max()))
    return fail(ctx, DD4DVAR_E_INVALID, "passes must be 0 or hold the largest box (modes 2 to 4)");
  const dd4dvar_status s = dd4dvar_set_exec_mode(ctx, mode);
  if (s != DD4DVAR_OK) return s;
  if (mode >= 2) ctx->box_k = passes ? passes : ctx->box_kmin;
  return DD4DVAR_OK;
}

dd4dvar_status dd4dvar_set_tz_kernels(dd4dvar_ctx* ctx, int32_t kind) {
  if (!ctx || kind < 0 || kind > 2) return fail(ctx, DD4DVAR_E_INVALID, "bad Turkel-Zwas kernel kind");
  if (kind >= 1 && !ctx->tz_col_ok)
    return fail(ctx, DD4DVAR_E_INVALID,
                "the column-walk kernels need the Turkel-Zwas variant with q = 2 and p <= 8");
  if (kind == 2 && (!ctx->tz_box_ok || ctx->ckpt))
    return fail(ctx, DD4DVAR_E_INVALID,
                "the persistent Turkel-Zwas forward needs FP32 state, every level stored, no box "
                "spanning the circle and every box's frame within the LDS");
  ctx->tz_col = kind >= 1;
  ctx->tz_box = kind == 2;
  return DD4DVAR_OK;
}

dd4dvar_status dd4dvar_get_tz_kernels(const dd4dvar_ctx* ctx, int32_t out[2]) {
  if (!ctx || !out) return fail(const_cast<dd4dvar_ctx*>(ctx), DD4DVAR_E_INVALID, "null argument");
  out[0] = ctx->tz_box ? 2 : (ctx->tz_col ? 1 : 0);
  out[1] = ctx->tz_col_ok ? (ctx->tz_box_ok && !ctx->ckpt ? 2 : 1) : 0;
  return DD4DVAR_OK;
}

dd4dvar_status dd4dvar_set_solver_parts(dd4dvar_ctx* ctx, int32_t entries) {
  if (!ctx || entries < 64 || entries > (1 << 24))
    return fail(ctx, DD4DVAR_E_INVALID, "entries per part must lie in [64, 2^24]");
  API_GUARD(ctx, {
    build_parts(ctx, entries, nullptr);
    return DD4DVAR_OK;
  })
}

dd4dvar_status dd4dvar_get_solver_parts(const dd4dvar_ctx* ctx, int32_t out[2]) {
  if (!ctx || !out) return fail(const_cast<dd4dvar_ctx*>(ctx), DD4DVAR_E_INVALID, "null argument");
  out[0] = ctx->part_len;
  out[1] = ctx->parts.nparts;
  return DD4DVAR_OK;
}

dd4dvar_status dd4dvar_get_exec_plan(const dd4dvar_ctx* ctx, int32_t out[4]) {
  if (!ctx || !out) return fail(const_cast<dd4dvar_ctx*>(ctx), DD4DVAR_E_INVALID, "null argument");
  out[0] = ctx->exec_mode;
  out[1] = ctx->box_ok ? ctx->box_k : 0;
  out[2] = ctx->strip_k;
  out[3] = ctx->box_ok ? 1 : 0;
  return DD4DVAR_OK;
}

dd4dvar_status dd4dvar_synchronize(dd4dvar_ctx* ctx, void* stream) {
  if (!ctx) return fail(ctx, DD4DVAR_E_INVALID, "null context");
  API_GUARD(ctx, {
    if (take_nonfinite(ctx, static_cast<hipStream_t>(stream)))
      return fail(ctx, DD4DVAR_E_NONFINITE,
                  "a cost, gradient or first-level adjoint entry was NaN or Inf since the last check");
    return DD4DVAR_OK;
  })
}

dd4dvar_status dd4dvar_set_timing(dd4dvar_ctx* ctx, int32_t on) {
  if (!ctx) return fail(ctx, DD4DVAR_E_INVALID, "null context");
  ctx->timing = on != 0;
  return DD4DVAR_OK;
}

dd4dvar_status dd4dvar_get_timing(dd4dvar_ctx* ctx, double out[6]) {
  if (!ctx || !out) return fail(ctx, DD4DVAR_E_INVALID, "null argument");
  API_GUARD(ctx, {
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (dd4dvar_ctx::Mark& m : ctx->marks) {
      chk(hipEventSynchronize(m.ev[3]), "hipEventSynchronize");
      float a = 0, b = 0, d = 0;
      chk(hipEventElapsedTime(&a, m.ev[0], m.ev[1]), "elapsed");
      chk(hipEventElapsedTime(&b, m.ev[1], m.ev[2]), "elapsed");
      chk(hipEventElapsedTime(&d, m.ev[2], m.ev[3]), "elapsed");
      acc[0] += a;
      acc[1] += b;
      acc[2] += d;
      acc[3] += m.nfwd;
      acc[4] += m.nadj;
      acc[5] += 1;
      for (hipEvent_t e : m.ev) (void)hipEventDestroy(e);
    }
    ctx->marks.clear();
    std::memcpy(out, acc, sizeof(acc));
    return DD4DVAR_OK;
  })
}

dd4dvar_status dd4dvar_background_controls(dd4dvar_ctx* ctx, double* x_dev, void* stream) {
  if (!ctx || !x_dev) return fail(ctx, DD4DVAR_E_INVALID, "null argument");
  API_GUARD(ctx, {
    chk(hipMemcpyAsync(x_dev, ctx->xb, size_t(ctx->plan.ctrl_total) * sizeof(double),
                       hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)),
        "copy background controls");
    return DD4DVAR_OK;
  })
}

dd4dvar_status dd4dvar_local_cost_grad(dd4dvar_ctx* ctx, int32_t nsub, const int32_t* sub_ids,
                                       const double* x_dev, double* J_dev, double* grad_dev,
                                       void* stream) {
  if (!ctx || !x_dev || !J_dev || !grad_dev) return fail(ctx, DD4DVAR_E_INVALID, "null argument");
  std::vector<int32_t> ids;
  if (sub_ids) {
    if (nsub < 0 || nsub > ctx->nsub) return fail(ctx, DD4DVAR_E_INVALID, "bad nsub");
    ids.assign(sub_ids, sub_ids + nsub);
    std::vector<char> seen(ctx->nsub, 0);
    for (int32_t s : ids) {
      if (s < 0 || s >= ctx->nsub || seen[s]) return fail(ctx, DD4DVAR_E_INVALID, "bad subdomain id");
      seen[s] = 1;
    }
    if (ids.empty()) return DD4DVAR_OK;
  }
  API_GUARD(ctx, {
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!sub_ids) {
      eval_all(ctx, x_dev, J_dev, grad_dev, st);
    } else if (ctx->prec == DD4DVAR_FP64) {
      cost_grad_impl<double>(ctx, &ids, x_dev, J_dev, grad_dev, st);
    } else {
      cost_grad_impl<float>(ctx, &ids, x_dev, J_dev, grad_dev, st);
    }
    return DD4DVAR_OK;
  })
}

dd4dvar_status dd4dvar_local_cost_grad_noalloc(dd4dvar_ctx* ctx, const double* x_dev,
                                               double* J_dev, double* grad_dev, void* stream) {
  if (!ctx || !x_dev || !J_dev || !grad_dev) return fail(ctx, DD4DVAR_E_INVALID, "null argument");
  if (int64_t(ctx->ntiles) > kScratchTiles)
    return fail(ctx, DD4DVAR_E_INVALID,
                "the no-allocation evaluation holds at most " + std::to_string(kScratchTiles) +
                    " tile partials; this decomposition has " + std::to_string(ctx->ntiles));
  if (!ctx->scratch) return fail(ctx, DD4DVAR_E_STATE, "no static scratch address for this device");
  API_GUARD(ctx, {
    // the same launches as local_cost_grad over all subdomains, eagerly (no
    // graph, no timing events), with the tile partials in the static scratch;
    // every partial is written before it is read, so nothing is cleared
    struct Restore {
      dd4dvar_ctx* c;
      bool timing;
      ~Restore() {
        c->jpart_use = nullptr;
        c->timing = timing;
      }
    } restore{ctx, ctx->timing};
    ctx->jpart_use = ctx->scratch;
    ctx->timing = false;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (ctx->prec == DD4DVAR_FP64)
      cost_grad_impl<double>(ctx, nullptr, x_dev, J_dev, grad_dev, st);
    else
      cost_grad_impl<float>(ctx, nullptr, x_dev, J_dev, grad_dev, st);
    return DD4DVAR_OK;
  })
}

dd4dvar_status dd4dvar_set_checkpointing(dd4dvar_ctx* ctx, int32_t stride, int64_t* state_bytes) {
  if (!ctx) return fail(ctx, DD4DVAR_E_INVALID, "null context");
  if (stride != 0 && stride < 3) return fail(ctx, DD4DVAR_E_INVALID, "stride must be 0 or >= 3");
  if (stride != 0 && ctx->exec_mode >= 2)
    return fail(ctx, DD4DVAR_E_INVALID, "persistent per-box sweeps store every level");
  API_GUARD(ctx, {
    const size_t tsz = ctx->prec == DD4DVAR_FP64 ? sizeof(double) : sizeof(float);
    const int maxl = ctx->maxlev - 1;
    std::vector<int32_t> slot(ctx->maxlev);
    int nslot = 0;
    if (stride) {
      const int K = maxl / stride + 1;                 // checkpoint pairs
      for (int n = 0; n <= maxl; ++n) {
        const int r = n % stride;
        slot[n] = r < 2 ? 2 * (n / stride) + r : 2 * K + r - 2;
      }
      nslot = 2 * K + stride - 2;
    }
    // each box gets as many slots as its own levels reach
    std::vector<SubDev> subs = ctx->subs;
    int64_t off = 0;
    for (SubDev& S : subs) {
      int need = S.nlev;
      if (stride) {
        need = 0;
        for (int n = 0; n < S.nlev; ++n) need = std::max(need, slot[n] + 1);
      }
      S.zoff = off;
      off += int64_t(need) * 3 * S.ncell;
    }
    const size_t bytes = size_t(std::max<int64_t>(off, 1)) * tsz;
    chk(hipDeviceSynchronize(), "sync");
    // graphs recorded with the old arena would read freed memory
    for (dd4dvar_ctx::GraphEntry& g : ctx->graphs) {
      (void)hipGraphExecDestroy(g.exec);
      (void)hipGraphDestroy(g.graph);
    }
    ctx->graphs.clear();
    void* fresh = nullptr;
    chk(hipMalloc(&fresh, bytes + kBoxArenaTail), "hipMalloc state arena");
    auto& owned = ctx->mem.owned;
    owned.erase(std::remove(owned.begin(), owned.end(), ctx->traj), owned.end());
    (void)hipFree(ctx->traj);
    ctx->traj = fresh;
    owned.push_back(fresh);
    ctx->traj_bytes = bytes;
    if (stride && !ctx->ring_next) ctx->ring_next = dalloc<char>(ctx, ctx->ring_bytes);
    if (stride) {
      if (ctx->d_zslot == ctx->d_zslot_id) ctx->d_zslot = dalloc<int32_t>(ctx, ctx->maxlev);
      chk(hipMemcpy(ctx->d_zslot, slot.data(), slot.size() * sizeof(int32_t), hipMemcpyHostToDevice),
          "upload slots");
    } else {
      ctx->d_zslot = ctx->d_zslot_id;
    }
    chk(hipMemcpy(ctx->d_subs, subs.data(), subs.size() * sizeof(SubDev), hipMemcpyHostToDevice),
        "upload subdomains");
    ctx->subs = subs;
    ctx->ckpt = stride;
    // the persistent Turkel-Zwas forward stores every level: with
    // checkpoints the column walk's forward steps run (kind 1)
    if (stride != 0) ctx->tz_box = false;
    ctx->nslot = nslot;
    ctx->have_forward = false;
    if (state_bytes) *state_bytes = int64_t(bytes);
    return DD4DVAR_OK;
  })
}

dd4dvar_status dd4dvar_set_graph(dd4dvar_ctx* ctx, int32_t on) {
  if (!ctx) return fail(ctx, DD4DVAR_E_INVALID, "null context");
  ctx->use_graph = on != 0;
  return DD4DVAR_OK;
}

dd4dvar_status dd4dvar_autotune(dd4dvar_ctx* ctx, const double* x_dev, double* J_dev,
                                double* grad_dev, int32_t reps, void* stream,
                                dd4dvar_tune_report* report) {
  if (!ctx || !x_dev || !J_dev || !grad_dev || !report) return fail(ctx, DD4DVAR_E_INVALID, "null argument");
  if (reps < 1 || reps > 1000) return fail(ctx, DD4DVAR_E_INVALID, "reps must be in 1..1000");
  API_GUARD(ctx, {
    hipStream_t st = static_cast<hipStream_t>(stream);
    // candidate execution plans (mode, passes of the forward): step kernels,
    // then the persistent sweeps (one launch per sweep, or fused) with the
    // smallest pass count that holds the largest box and with the maximum
    // one, and the column-strip adjoint where it applies
    const int kmin = ctx->box_kmin, kmax = box_passes_max();
    std::vector<std::pair<int, int>> cand = {{0, kmin}};
    if (ctx->box_ok && !ctx->ckpt) {
      cand.push_back({2, kmin});
      if (kmax != kmin) cand.push_back({2, kmax});
      cand.push_back({3, kmin});
      if (ctx->strip_k > 0) cand.push_back({4, kmin});
    }
    const int mode0 = ctx->exec_mode, k0 = ctx->box_k;
    const bool timing0 = ctx->timing;
    ctx->timing = false;
    hipEvent_t a = nullptr, b = nullptr;
    try {
      chk(hipEventCreate(&a), "event");
      chk(hipEventCreate(&b), "event");
      std::memset(report, 0, sizeof(*report));
      report->ncand = int32_t(cand.size());
      double best = 0;
      for (size_t i = 0; i < cand.size(); ++i) {
        ctx->exec_mode = cand[i].first;
        ctx->box_k = cand[i].second;
        eval_all(ctx, x_dev, J_dev, grad_dev, st);           // warm-up (records a graph in graph mode)
        chk(hipEventRecord(a, st), "event");
        for (int r = 0; r < reps; ++r) eval_all(ctx, x_dev, J_dev, grad_dev, st);
        chk(hipEventRecord(b, st), "event");
        chk(hipEventSynchronize(b), "event sync");
        float ms = 0;
        chk(hipEventElapsedTime(&ms, a, b), "elapsed");
        report->mode[i] = cand[i].first;
        report->passes[i] = cand[i].first == 4 ? ctx->strip_k : (cand[i].first >= 2 ? cand[i].second : 0);
        report->ms[i] = double(ms) / reps;
        if (i == 0 || report->ms[i] < best) {
          best = report->ms[i];
          report->chosen = int32_t(i);
        }
      }
    } catch (...) {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
      ctx->exec_mode = mode0;
      ctx->box_k = k0;
      ctx->timing = timing0;
      throw;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    ctx->exec_mode = report->mode[report->chosen];
    ctx->box_k = cand[report->chosen].second;
    ctx->timing = timing0;
    if (take_nonfinite(ctx, st))
      return fail(ctx, DD4DVAR_E_NONFINITE, "a cost or gradient entry at x was NaN or Inf");
    return DD4DVAR_OK;
  })
}

dd4dvar_status dd4dvar_forward_integrate(dd4dvar_ctx* ctx, int32_t scope, const double* x_dev,
                                         double* traj_dev, void* stream) {
  if (!ctx || !x_dev) return fail(ctx, DD4DVAR_E_INVALID, "null argument");
  if (scope != 0 && scope != 1) return fail(ctx, DD4DVAR_E_INVALID, "scope must be 0 or 1");
  if (scope == 0 && !traj_dev) return fail(ctx, DD4DVAR_E_INVALID, "global scope needs traj_dev");
  API_GUARD(ctx, {
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (scope == 0) {
      const dd4dvar_model_desc& m = ctx->plan.model;
      const int64_t plane = int64_t(m.nlat) * m.nlon;
      global_forward(ctx, x_dev, traj_dev, st);
      launch_add_href(traj_dev, m.nsteps + 1, plane, m.h_ref, st);
      chk(hipGetLastError(), "global forward");
      return DD4DVAR_OK;
    }
    if (ctx->prec == DD4DVAR_FP64)
      local_forward<double>(ctx, x_dev, st, traj_dev);
    else
      local_forward<float>(ctx, x_dev, st, traj_dev);
    chk(hipGetLastError(), "trajectory output");
    return DD4DVAR_OK;
  })
}

dd4dvar_status dd4dvar_adjoint_integrate(dd4dvar_ctx* ctx, int32_t scope, const double* forcing_dev,
                                         double* adj0_dev, void* stream) {
  if (!ctx || !adj0_dev) return fail(ctx, DD4DVAR_E_INVALID, "null argument");
  if (scope != 1) return fail(ctx, DD4DVAR_E_INVALID, "only scope 1 is supported");
  if (!ctx->have_forward) return fail(ctx, DD4DVAR_E_STATE, "adjoint before any forward");
  API_GUARD(ctx, {
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int mode = forcing_dev ? 1 : 2;
    if (ctx->prec == DD4DVAR_FP64)
      local_adjoint<double>(ctx, mode, nullptr, forcing_dev, adj0_dev, nullptr, st);
    else
      local_adjoint<float>(ctx, mode, nullptr, forcing_dev, adj0_dev, nullptr, st);
    return DD4DVAR_OK;
  })
}

dd4dvar_status dd4dvar_tangent_linear(dd4dvar_ctx* ctx, const double* dx_dev, double* dtraj_dev,
                                      void* stream) {
  if (!ctx || !dx_dev) return fail(ctx, DD4DVAR_E_INVALID, "null argument");
  if (ctx->ckpt) return fail(ctx, DD4DVAR_E_INVALID, "the tangent-linear model needs every level stored");
  if (!ctx->have_forward) return fail(ctx, DD4DVAR_E_STATE, "tangent-linear model before any forward");
  API_GUARD(ctx, {
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (ctx->prec == DD4DVAR_FP64) {
      local_tlm<double>(ctx, dx_dev, st);
      if (dtraj_dev) launch_dz_out<double>(local_dom<double>(ctx), dtraj_dev, 0, ctx->ntiles, st);
    } else {
      local_tlm<float>(ctx, dx_dev, st);
      if (dtraj_dev) launch_dz_out<float>(local_dom<float>(ctx), dtraj_dev, 0, ctx->ntiles, st);
    }
    chk(hipGetLastError(), "tangent-linear output launch");
    return DD4DVAR_OK;
  })
}

dd4dvar_status dd4dvar_gn_hessvec(dd4dvar_ctx* ctx, const double* dx_dev, double* out_dev,
                                  void* stream) {
  if (!ctx || !dx_dev || !out_dev) return fail(ctx, DD4DVAR_E_INVALID, "null argument");
  if (dx_dev == out_dev) return fail(ctx, DD4DVAR_E_INVALID, "dx_dev and out_dev must differ");
  if (ctx->ckpt) return fail(ctx, DD4DVAR_E_INVALID, "Gauss-Newton products need every level stored");
  if (!ctx->have_forward) return fail(ctx, DD4DVAR_E_STATE, "Gauss-Newton product before any forward");
  API_GUARD(ctx, {
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (ctx->prec == DD4DVAR_FP64) gn_product<double>(ctx, dx_dev, out_dev, st);
    else gn_product<float>(ctx, dx_dev, out_dev, st);
    launch_add_bdiag(ctx->parts, ctx->cover, ctx->plan.model.weight_mode, ctx->plan.sigma_b.data(),
                     dx_dev, out_dev, st);
    chk(hipGetLastError(), "background block launch");
    return DD4DVAR_OK;
  })
}

dd4dvar_status dd4dvar_exchange(dd4dvar_ctx* ctx, const double* x_dev, void* stream) {
  if (!ctx || !x_dev) return fail(ctx, DD4DVAR_E_INVALID, "null argument");
  API_GUARD(ctx, {
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (ctx->prec == DD4DVAR_FP64) exchange_impl<double>(ctx, x_dev, st);
    else exchange_impl<float>(ctx, x_dev, st);
    return DD4DVAR_OK;
  })
}

dd4dvar_status dd4dvar_gather(dd4dvar_ctx* ctx, int32_t level, double* out_dev, void* stream) {
  if (!ctx || !out_dev) return fail(ctx, DD4DVAR_E_INVALID, "null argument");
  if (level < 0 || level > ctx->plan.model.nsteps) return fail(ctx, DD4DVAR_E_INVALID, "bad level");
  if (!ctx->have_forward) return fail(ctx, DD4DVAR_E_STATE, "gather before any forward");
  if (ctx->ckpt) {
    // only checkpoint levels stay stored
    for (const SubDev& S : ctx->subs) {
      const int n = level - S.lev0;
      if (n >= 0 && n < S.nlev && n % ctx->ckpt >= 2)
        return fail(ctx, DD4DVAR_E_STATE, "level not stored: checkpoints keep levels kc, kc+1 only");
    }
  }
  API_GUARD(ctx, {
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t ncell = int64_t(ctx->plan.model.nlat) * ctx->plan.model.nlon;
    if (ctx->prec == DD4DVAR_FP64)
      launch_gather<double>(local_dom<double>(ctx), ctx->plan.nspace, ctx->plan.ntime, level, ncell,
                            ctx->cptr, ctx->cpiece, out_dev, st);
    else
      launch_gather<float>(local_dom<float>(ctx), ctx->plan.nspace, ctx->plan.ntime, level, ncell,
                           ctx->cptr, ctx->cpiece, out_dev, st);
    chk(hipGetLastError(), "gather launch");
    return DD4DVAR_OK;
  })
}

dd4dvar_status dd4dvar_solve(dd4dvar_ctx* ctx, const dd4dvar_solve_opts* opts,
                             const double* x_init_dev, double* x_out_dev, double* xa_host,
                             dd4dvar_solve_report* report) {
  if (!ctx || !opts || !xa_host) return fail(ctx, DD4DVAR_E_INVALID, "null argument");
  API_GUARD(ctx, {
    const dd4dvar_status r = solve_impl(ctx, opts, x_init_dev, x_out_dev, xa_host, report, nullptr);
    // trial steps of the line search may overflow; the solve handles them
    (void)take_nonfinite(ctx, nullptr);
    return r;
  })
}

dd4dvar_status dd4dvar_solve_mixed(dd4dvar_ctx* ctx, dd4dvar_ctx* ctx_lo,
                                   const dd4dvar_solve_opts* opts, const double* x_init_dev,
                                   double* x_out_dev, double* xa_host,
                                   dd4dvar_solve_report* report) {
  if (!ctx || !ctx_lo || !opts || !xa_host) return fail(ctx, DD4DVAR_E_INVALID, "null argument");
  if (ctx == ctx_lo) return fail(ctx, DD4DVAR_E_INVALID, "the two contexts must differ");
  API_GUARD(ctx, {
    const dd4dvar_status r = solve_impl(ctx, opts, x_init_dev, x_out_dev, xa_host, report, ctx_lo);
    (void)take_nonfinite(ctx, nullptr);
    (void)take_nonfinite(ctx_lo, nullptr);
    return r;
  })
}

}  // extern "C"

namespace dd4dvar {

namespace {
// device buffers of one solve, released on every exit path
struct SolveBuffers {
  std::vector<void*> p;
  ~SolveBuffers() {
    for (void* q : p) (void)hipFree(q);
  }
  template <typename P>
  P* get(size_t n) {
    void* q = nullptr;
    chk(hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(P)), "hipMalloc solve");
    p.push_back(q);
    return static_cast<P*>(q);
  }
};

template <typename P>
P read1(const P* d, hipStream_t st) {
  P h{};
  chk(hipMemcpyAsync(&h, d, sizeof(P), hipMemcpyDeviceToHost, st), "read");
  chk(hipStreamSynchronize(st), "sync");
  return h;
}

// lo (nullable, Gauss-Newton only): an FP32-state context of the same plan
// whose sweeps supply the normal-matrix products, linearized about its own
// trajectory of the current iterate; c evaluates J and the gradient
template <typename T>
dd4dvar_status solve_typed(dd4dvar_ctx* c, const dd4dvar_solve_opts* o, const double* x_init,
                           double* x_out, double* xa_host, dd4dvar_solve_report* rep,
                           dd4dvar_ctx* lo) {
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = nullptr;
  chk(hipDeviceSynchronize(), "sync");
  const int nsub = c->nsub;
  const int64_t N = c->plan.ctrl_total;
  SolveBuffers B;
  LbState L{};
  L.subs = c->d_subs;
  L.nsub = nsub;
  L.m = o->lbfgs_m;
  L.max_iter = o->max_iter;
  L.max_ls = o->max_ls;
  L.N = N;
  for (int f = 0; f < 3; ++f) L.sb[f] = c->plan.sigma_b[f];
  L.c1 = o->armijo_c1;
  L.jnoise = o->j_noise_rtol;
  L.grad_rtol = o->grad_rtol;
  L.xb = c->xb;
  L.xi = B.get<double>(N);
  L.xi0 = B.get<double>(N);
  L.g = B.get<double>(N);
  L.d = B.get<double>(N);
  L.xt = B.get<double>(N);
  L.xphys = B.get<double>(N);
  L.gradx = B.get<double>(N);
  const bool use_gn = o->local_solver == 1;
  // the pair memory only for L-BFGS
  L.S = B.get<double>(use_gn ? 1 : size_t(L.m) * N);
  L.Y = B.get<double>(use_gn ? 1 : size_t(L.m) * N);
  L.J = B.get<double>(nsub);
  L.Jt = B.get<double>(nsub);
  L.gd = B.get<double>(nsub);
  L.alpha = B.get<double>(nsub);
  L.rho = B.get<double>(size_t(L.m) * nsub);
  L.gamma = B.get<double>(nsub);
  L.g0norm = B.get<double>(nsub);
  L.gnorm = B.get<double>(nsub);
  L.step = B.get<double>(nsub);
  L.npairs = B.get<int32_t>(nsub);
  L.head = B.get<int32_t>(nsub);
  L.status = B.get<int32_t>(nsub);
  L.iters = B.get<int32_t>(nsub);
  L.trials = B.get<int32_t>(nsub);
  L.ls = B.get<uint8_t>(nsub);
  L.pending = B.get<int32_t>(1);
  L.P = c->parts;
  L.alph = B.get<double>(size_t(L.m) * nsub);
  L.acc = B.get<uint8_t>(nsub);
  L.wslot = B.get<int32_t>(nsub);
  // Gauss-Newton state: iterate, evaluation, norms and stop flags shared
  // with the L-BFGS state above, CG vectors of its own
  GnState G{};
  if (use_gn) {
    G.subs = c->d_subs;
    G.nsub = nsub;
    G.max_iter = o->max_iter;
    G.cg_max_iter = o->cg_max_iter;
    G.weight_mode = c->plan.model.weight_mode;
    G.N = N;
    for (int f = 0; f < 3; ++f) G.sb[f] = c->plan.sigma_b[f];
    G.grad_rtol = o->grad_rtol;
    G.cg_rtol = o->cg_rtol;
    G.xb = c->xb;
    G.cover = c->cover;
    G.xi = L.xi;
    G.xi0 = L.xi0;
    G.xphys = L.xphys;
    G.gradx = L.gradx;
    G.dxi = B.get<double>(N);
    G.r = B.get<double>(N);
    G.p = B.get<double>(N);
    G.dx = B.get<double>(N);
    G.hv = B.get<double>(N);
    G.J = L.J;
    G.Jt = L.Jt;
    G.g0norm = L.g0norm;
    G.gnorm = L.gnorm;
    G.step = L.step;
    G.rr = B.get<double>(nsub);
    G.rr0 = B.get<double>(nsub);
    G.status = L.status;
    G.iters = L.iters;
    G.cg_k = B.get<int32_t>(nsub);
    G.cg_total = B.get<int32_t>(nsub);
    G.gn_on = B.get<uint8_t>(nsub);
    G.cg_on = B.get<uint8_t>(nsub);
    G.pending = L.pending;
    G.P = c->parts;
    G.ca = B.get<double>(nsub);
    G.cb = B.get<double>(nsub);
    G.krylov = o->krylov;
    if (o->krylov == 1) {
      // Lanczos basis (cg_max_iter vectors) and per-subdomain coefficients
      const size_t K = size_t(std::max(o->cg_max_iter, 1));
      G.lv = B.get<double>(K * size_t(N));
      G.la = B.get<double>(size_t(nsub) * (K + 1));
      G.lb = B.get<double>(size_t(nsub) * (K + 1));
      G.ly = B.get<double>(size_t(nsub) * (K + 1));
      G.ld = B.get<double>(size_t(nsub) * (K + 1));
      G.lz = B.get<double>(size_t(nsub) * (K + 1));
      G.ritz_lo = B.get<double>(nsub);
      G.ritz_hi = B.get<double>(nsub);
      launch_fill(G.ritz_lo, nsub, 0.0, st);
      launch_fill(G.ritz_hi, nsub, 0.0, st);
    }
  }
  double* xa_dev = B.get<double>(size_t(3) * c->plan.model.nlat * c->plan.model.nlon);

  struct MaskReset {
    dd4dvar_ctx *c, *lo;
    ~MaskReset() {
      c->eval_mask = nullptr;
      if (lo) lo->eval_mask = nullptr;
    }
  } reset{c, lo};

  if (x_init) {
    lb_from_x(L, x_init, st);
  } else {
    // Alg. 1 from the background: halo rings and overlap targets of the
    // background run, whatever an earlier solve left in them
    background_impl<T>(c, st);
    if (lo) background_impl<float>(lo, st);
    launch_fill(L.xi, N, 0.0, st);
  }
  int evals = 0, outer = 0, lbfgs_iters = 0, products = 0;
  bool met = false;
  std::vector<int32_t> iters_h(nsub);
  for (outer = 1; outer <= o->max_outer; ++outer) {
    // local solves, all subdomains at once
    c->eval_mask = nullptr;
    lb_to_x(L, 0, 0, st);
    cost_grad_impl<T>(c, nullptr, L.xphys, L.Jt, L.gradx, st);
    ++evals;
    if (use_gn) {
      // Gauss-Newton: CG on the normal equations about the stored
      // trajectory, the full update, a new evaluation (masked to the
      // subdomains still iterating)
      gn_start(G, st);
      for (;;) {
        chk(hipMemsetAsync(L.pending, 0, sizeof(int32_t), st), "memset");
        gn_count(G, st);
        if (read1(L.pending, st) == 0) break;
        if (lo) {
          // the products' linearization: lo's trajectory of the current x
          lo->eval_mask = G.gn_on;
          local_forward<float>(lo, L.xphys, st);
          lo->eval_mask = nullptr;
        }
        if (G.krylov == 1) gn_lz_start(G, st);
        else gn_cg_start(G, st);
        for (;;) {
          chk(hipMemsetAsync(L.pending, 0, sizeof(int32_t), st), "memset");
          gn_cg_count(G, st);
          if (read1(L.pending, st) == 0) break;
          gn_cg_dir(G, st);
          if (lo) {
            lo->eval_mask = G.cg_on;
            gn_product<float>(lo, G.dx, G.hv, st);
            lo->eval_mask = nullptr;
          } else {
            c->eval_mask = G.cg_on;
            gn_product<T>(c, G.dx, G.hv, st);
            c->eval_mask = nullptr;
          }
          ++products;
          if (G.krylov == 1) gn_lz_update(G, st);
          else gn_cg_update(G, st);
        }
        if (G.krylov == 1) gn_lz_finish(G, st);
        gn_update(G, st);
        lb_to_x(L, 0, 0, st);
        c->eval_mask = G.gn_on;
        cost_grad_impl<T>(c, nullptr, L.xphys, L.Jt, L.gradx, st);
        c->eval_mask = nullptr;
        ++evals;
        gn_after(G, st);
      }
    } else {
      lb_start(L, st);
      for (;;) {
        chk(hipMemsetAsync(L.pending, 0, sizeof(int32_t), st), "memset");
        lb_count(L, st);
        if (read1(L.pending, st) == 0) break;
        lb_direction(L, st);
        for (;;) {
          lb_trial(L, st);
          c->eval_mask = L.ls;
          cost_grad_impl<T>(c, nullptr, L.xphys, L.Jt, L.gradx, st);
          c->eval_mask = nullptr;
          ++evals;
          chk(hipMemsetAsync(L.pending, 0, sizeof(int32_t), st), "memset");
          lb_armijo(L, st);
          if (read1(L.pending, st) == 0) break;
        }
      }
    }
    chk(hipMemcpyAsync(iters_h.data(), L.iters, nsub * sizeof(int32_t), hipMemcpyDeviceToHost, st),
        "read iters");
    lb_step(L, st);
    std::vector<double> step(nsub);
    chk(hipMemcpyAsync(step.data(), L.step, nsub * sizeof(double), hipMemcpyDeviceToHost, st),
        "read step");
    chk(hipStreamSynchronize(st), "sync");
    lbfgs_iters += *std::max_element(iters_h.begin(), iters_h.end());
    // exchange (Alg. 1): integrate the new controls, refresh rings and targets
    lb_to_x(L, 0, 0, st);
    exchange_impl<T>(c, L.xphys, st);
    if (lo) exchange_impl<float>(lo, L.xphys, st);
    const double mx = *std::max_element(step.begin(), step.end());
    if (!std::isfinite(mx)) {
      c->err = "non-finite iterate in the local solves";
      return DD4DVAR_E_NONFINITE;
    }
    if (mx < o->outer_tol) {
      met = true;
      break;
    }
  }
  if (outer > o->max_outer) outer = o->max_outer;
  // gather the analysis at level 0 (partition of unity, eq. rest)
  const int64_t ncell = int64_t(c->plan.model.nlat) * c->plan.model.nlon;
  launch_gather<T>(local_dom<T>(c), c->plan.nspace, c->plan.ntime, 0, ncell, c->cptr, c->cpiece,
                   xa_dev, st);
  chk(hipGetLastError(), "gather launch");
  chk(hipMemcpyAsync(xa_host, xa_dev, size_t(3 * ncell) * sizeof(double), hipMemcpyDeviceToHost, st),
      "copy analysis");
  if (x_out)
    chk(hipMemcpyAsync(x_out, L.xphys, size_t(N) * sizeof(double), hipMemcpyDeviceToDevice, st),
        "copy controls");
  std::vector<double> J(nsub), gn(nsub), g0(nsub);
  chk(hipMemcpyAsync(J.data(), L.J, nsub * sizeof(double), hipMemcpyDeviceToHost, st), "read J");
  chk(hipMemcpyAsync(gn.data(), L.gnorm, nsub * sizeof(double), hipMemcpyDeviceToHost, st), "read g");
  chk(hipMemcpyAsync(g0.data(), L.g0norm, nsub * sizeof(double), hipMemcpyDeviceToHost, st), "read g0");
  std::vector<double> rlo(nsub, 0.0), rhi(nsub, 0.0);
  if (use_gn && G.krylov == 1) {
    chk(hipMemcpyAsync(rlo.data(), G.ritz_lo, nsub * sizeof(double), hipMemcpyDeviceToHost, st), "read ritz");
    chk(hipMemcpyAsync(rhi.data(), G.ritz_hi, nsub * sizeof(double), hipMemcpyDeviceToHost, st), "read ritz");
  }
  chk(hipStreamSynchronize(st), "sync");
  if (rep) {
    rep->outer_iters = outer;
    rep->total_evals = evals;
    rep->lbfgs_iters = lbfgs_iters;
    rep->gn_products = products;
    double js = 0, ratio = 0;
    for (int s = 0; s < nsub; ++s) {
      js += J[s];
      if (g0[s] > 0) ratio = std::max(ratio, gn[s] / g0[s]);
    }
    rep->J_final = js;
    rep->gnorm_ratio_max = ratio;
    // extreme Ritz values over the subdomains' last Lanczos runs
    double rmin = 0, rmax = 0;
    bool any = false;
    for (int s = 0; s < nsub; ++s) {
      if (!(rhi[s] > 0)) continue;
      rmin = any ? std::min(rmin, rlo[s]) : rlo[s];
      rmax = any ? std::max(rmax, rhi[s]) : rhi[s];
      any = true;
    }
    rep->ritz_min = rmin;
    rep->ritz_max = rmax;
    rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (!met) {
    c->err = "outer iterations exhausted before the exchange step fell below outer_tol";
    return DD4DVAR_E_NOTCONVERGED;
  }
  return DD4DVAR_OK;
}
}  // namespace

dd4dvar_status solve_impl(dd4dvar_ctx* ctx, const dd4dvar_solve_opts* o, const double* x_init,
                          double* x_out, double* xa_host, dd4dvar_solve_report* rep,
                          dd4dvar_ctx* lo) {
  if (o->lbfgs_m < 1 || o->lbfgs_m > kMaxPairs || o->max_iter < 0 || o->max_outer < 1 ||
      o->max_ls < 1 || !(o->grad_rtol >= 0) || !(o->outer_tol >= 0) || !(o->armijo_c1 > 0) ||
      !(o->armijo_c1 < 1) || !(o->j_noise_rtol >= 0) || !std::isfinite(o->j_noise_rtol) ||
      o->local_solver < 0 || o->local_solver > 1 || o->cg_max_iter < 0 || !(o->cg_rtol >= 0) ||
      o->krylov < 0 || o->krylov > 1 || (o->krylov == 1 && o->local_solver != 1) ||
      !std::isfinite(o->cg_rtol)) {
    ctx->err = "bad solve options";
    return DD4DVAR_E_INVALID;
  }
  if (o->local_solver == 1 && ctx->ckpt) {
    ctx->err = "the Gauss-Newton local solver needs every level stored (checkpoints on)";
    return DD4DVAR_E_INVALID;
  }
  if (lo) {
    if (o->local_solver != 1 || ctx->prec != DD4DVAR_FP64 || lo->prec != DD4DVAR_FP32_STATE) {
      ctx->err = "the mixed-precision solve is Gauss-Newton with an FP64 and an FP32-state context";
      return DD4DVAR_E_INVALID;
    }
    if (lo->ckpt || lo->device != ctx->device || lo->nsub != ctx->nsub ||
        lo->plan.ctrl_total != ctx->plan.ctrl_total || lo->plan.traj_total != ctx->plan.traj_total) {
      ctx->err = "the two contexts of a mixed-precision solve need the same plan, device and no checkpoints";
      return DD4DVAR_E_INVALID;
    }
    for (int s = 0; s < ctx->nsub; ++s) {
      const SubDev &a = ctx->subs[s], &b = lo->subs[s];
      if (a.ncell != b.ncell || a.nlev != b.nlev || a.ctrl_off != b.ctrl_off ||
          a.traj_off != b.traj_off || a.row0 != b.row0 || a.col0 != b.col0 || a.lev0 != b.lev0) {
        ctx->err = "the two contexts of a mixed-precision solve need the same plan";
        return DD4DVAR_E_INVALID;
      }
    }
    return solve_typed<double>(ctx, o, x_init, x_out, xa_host, rep, lo);
  }
  if (ctx->prec == DD4DVAR_FP64) return solve_typed<double>(ctx, o, x_init, x_out, xa_host, rep, nullptr);
  return solve_typed<float>(ctx, o, x_init, x_out, xa_host, rep, nullptr);
}
}  // namespace dd4dvar
