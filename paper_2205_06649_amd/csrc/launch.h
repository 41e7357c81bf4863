// Kernel launchers (defined in sweep.hip and exchange.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace dd4dvar {

template <typename T>
void launch_init(const Dom<T>& D, const double* x, int tile_base, int ntiles, hipStream_t st);
template <typename T>
void launch_fwd(const Dom<T>& D, int n, int tile_base, int ntiles, hipStream_t st);
template <typename T>
void launch_adj(const Dom<T>& D, int n, int tile_base, int ntiles, int mode, const double* x,
                const double* xb, const double* forcing, double* out, hipStream_t st);
void launch_reduce_j(const SubDev* subs, int count, const int32_t* ids, const double* jpart,
                     const double* jconst, double* J, uint32_t* nonfinite, hipStream_t st);
template <typename T>
void launch_traj_out(const Dom<T>& D, double* out, int tile_base, int ntiles, int level,
                     hipStream_t st);

// exchange.hip
template <typename T>
void launch_from_global(const Dom<T>& D, const double* bg, int64_t gplane, double* xb,
                        int level, int ntiles, hipStream_t st);
template <typename T>
void launch_ring_from_global(const Dom<T>& D, int nsub, int ring_blocks, const double* bg,
                             int64_t gplane, hipStream_t st);
template <typename T>
void launch_ring_from_local(const Dom<T>& D, int box_base, int nbox, int ring_blocks, int level,
                            hipStream_t st);
template <typename T>
void launch_targets_from_local(const Dom<T>& D, int level, int tile_base, int ntiles, double* jc,
                               hipStream_t st);
void launch_reduce_jconst(const SubDev* subs, int nsub, const double* jc, double half_mu,
                          double* jconst, hipStream_t st);
template <typename T>
void launch_gather(const Dom<T>& D, int nspace, int ntime, int level, int64_t ncell,
                   const int32_t* cptr, const int32_t* cpiece, double* out, hipStream_t st);
void launch_add_href(double* traj, int64_t nlev, int64_t plane, double h0, hipStream_t st);
void launch_fill(double* p, int64_t n, double v, hipStream_t st);

// tlm.hip: tangent linear model of the local sweeps
template <typename T>
void launch_tlm_init(const Dom<T>& D, const double* dx, int tile_base, int ntiles, hipStream_t st);
template <typename T>
void launch_tlm(const Dom<T>& D, int n, int tile_base, int ntiles, hipStream_t st);
template <typename T>
void launch_dz_out(const Dom<T>& D, double* out, int tile_base, int ntiles, hipStream_t st);

// tz.hip: Turkel-Zwas step kernels (boxes with frozen pads q rows and p
// columns wide)

// one wave's share of the column-walk Turkel-Zwas adjoint (offset q = 2):
// box, first column of its outputs' block (c0, lanes p .. 63 - p), rows
// r0 .. r1 - 1, its J slot, and the box's J slots no wave writes
// [zero0, zero1) (set on the box's first wave only)
struct TzWork {
  int32_t box, c0, r0, r1, slot, zero0, zero1, pad_;
};
// persistent Turkel-Zwas forward sweep (FP32): one workgroup per box for the
// whole interval, the level and its pad in an LDS frame; boxes that span the
// circle are not taken.  LDS bytes of a box's frame and row table, whether
// a box fits (cells, pad positions, LDS), and the launch over the nboxes
// boxes of order (max_cells: the largest box)
size_t tz_box_lds_bytes(int nx, int ny, int p, int q);
bool tz_box_fits(int ncell, int nring, size_t lds_bytes);
hipError_t prepare_fwd_tz_box();          // once, before any launch: the LDS allowance
hipError_t launch_fwd_tz_box(const Dom<float>& D, const double* x, const int32_t* order, int nboxes,
                             size_t lds_bytes, int max_cells, int p, int q, double alpha, int nlat,
                             hipStream_t st);
// forward step: work == nullptr, the gather kernel (one thread per cell,
// any p, q); otherwise the column walk over the nwork waves
template <typename T>
void launch_fwd_tz(const Dom<T>& D, int n, int tile_base, int ntiles, int p, int q, double alpha,
                   int nlat, const TzWork* work, int nwork, hipStream_t st);
// adjoint step: work == nullptr, the gather kernel (one thread per cell, any p, q);
// otherwise the column walk over the nwork waves, and the observation
// forcing over obs_tiles (the tiles with observation entries at level n)
template <typename T>
void launch_adj_tz(const Dom<T>& D, int n, int tile_base, int ntiles, int mode, int p, int q,
                   double alpha, int nlat, const double* x, const double* xb,
                   const double* forcing, double* out, const TzWork* work, int nwork,
                   const int32_t* obs_tiles, int nobs_tiles, hipStream_t st);
// tangent-linear step: work == nullptr, the gather kernel; otherwise the
// column walk over the nwork waves
template <typename T>
void launch_tlm_tz(const Dom<T>& D, int n, int tile_base, int ntiles, int p, int q, double alpha,
                   int nlat, const TzWork* work, int nwork, hipStream_t st);

// box.hip: persistent per-box sweeps (FP32 state)
//
// Their loads of the state, target and tangent-linear arenas may reach past
// a box's last level: lanes whose rows or cells lie past the box read at
// addresses that follow the pattern of the lanes inside it, and discard the
// values.  The offset past the last level's end is below (1024 div nx + K +
// 2) rows of nx cells plus one cell (column strips) or 1024 + nx + 1 cells
// (cells t + 1024 k), under 64 KiB for nx <= 1022 and K <= 11; every arena
// those kernels read is allocated with this many bytes after its end, so
// that all their loads stay inside the allocation.
constexpr size_t kBoxArenaTail = size_t(64) * 1024;
size_t box_lds_bytes(int ny, int nx, int nring, int nlev);
int box_passes(int ny, int nx, int nring, int nlev);
int box_passes_max();
int box_strip_rows(int ny, int nx, int nring, int nlev);
hipError_t box_prepare(int passes);
hipError_t launch_fwd_box(const Dom<float>& D, const double* x, const int32_t* order, int nboxes,
                          size_t lds_bytes, int passes, bool span, hipStream_t st);
hipError_t launch_tlm_box(const Dom<float>& D, const double* dx, const int32_t* order, int nboxes,
                          size_t lds_bytes, int passes, bool span, hipStream_t st);
hipError_t launch_adj_box(const Dom<float>& D, int mode, const double* x, const double* xb,
                          const double* forcing, double* out, const int32_t* order, int nboxes,
                          size_t lds_bytes, int passes, bool span, bool strip, hipStream_t st);
hipError_t launch_eval_box(const Dom<float>& D, const double* x, const double* xb, double* grad,
                           const int32_t* order, int nboxes, size_t lds_bytes, int passes,
                           bool span, hipStream_t st);

}  // namespace dd4dvar
