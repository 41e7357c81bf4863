// Device data structures shared by the HIP kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace dd4dvar {

constexpr int kTile = 256;  // cells per work tile = threads per workgroup
constexpr int kXcd = 8;     // MI355X: 8 accelerator dies, each with its own L2

// Workgroups are dealt to the XCDs round-robin (block i runs on XCD i % 8).
// Remap block i to tile index so that each XCD receives one contiguous range
// of tiles: consecutive tiles of a box (whose rows are each other's north and
// south halos) then share an L2.  Bijective on [0, nblocks).
__device__ __forceinline__ int xcd_tile(int i, int nblocks) {
  const int per = nblocks / kXcd, rem = nblocks % kXcd;
  const int x = i % kXcd, k = i / kXcd;
  return x * per + (x < rem ? x : rem) + k;
}

// Key of the observation bin of (tile t_local of a box, level n) in the CSR
// over bins.  A box's bins are ordered by level, then by tile: the entries of
// one tile at one level form one range (the step kernels), and so do the
// entries of the whole box at one level (the per-box kernels:
// obs_key(.., 0, n) .. obs_key(.., 0, n + 1)).  Bijective from [0, maxlev) x
// [0, ntile) onto the box's keys [tile0 maxlev, (tile0 + ntile) maxlev).
__host__ __device__ inline int64_t obs_key(int tile0, int ntile, int maxlev, int t_local, int n) {
  return int64_t(tile0) * maxlev + int64_t(n) * ntile + t_local;
}

// One subdomain (or the whole grid) as the kernels see it.
struct SubDev {
  int32_t row0, ny, col0, nx;
  int32_t lev0, nlev;        // first global level, number of levels
  int32_t span, pole_s, pole_n;
  int32_t ncell, nring, tile0, ntile;
  int32_t nbr0, nbr1;        // neighbour list range
  int32_t pad_;
  int64_t traj_off;          // packed FP64 trajectory and overlap-target offset
  int64_t ring_off;          // ring arena offset, level stride 3*nring
  int64_t adj_off;           // adjoint arena offset: 3 slots x 3 x ncell
  int64_t ctrl_off;          // packed control offset
  int64_t cell_off;          // per-cell coverage offset
  int64_t hmap_off;          // halo map offset
  int64_t zoff;              // state arena offset (level slots, see Dom::zslot)
};

// Per-row coefficients of the discrete increment.
template <typename T>
struct RowCoef {
  T a1;   // sigma_lon / cos
  T a2;   // sigma_lon * g / cos
  T a3;   // sigma_lat / cos
  T cf;   // 2 dt f
  T ct;   // 2 dt tan / a
  T c;    // cos
};

template <typename T>
struct Dom {
  const SubDev* subs;
  const int2* tiles;         // (subdomain, tile within subdomain)
  T* traj;                   // [slots][3][ncell] per subdomain, h stored as h - h_ref
  T* ring;                   // [nlev][3][nring] per subdomain, signs applied
  T* targ;                   // mean overlap target, traj layout
  T* adj;                    // rolling adjoint levels
  T* dz;                     // tangent-linear trajectory, every level (zoff layout)
  const RowCoef<T>* rows;    // [nlat]
  const T* cosx;             // [nlat+2]: cos of rows -1..nlat (pole-mapped)
  const uint8_t* cover;      // spatial coverage count per box cell
  const int32_t* tcount;     // temporal coverage count per global level
  const int32_t* obs_ptr;    // CSR over the (tile, level) bins, keyed by obs_key
  const int32_t* obs_code;   // local cell * 4 + field
  const double* obs_val;     // value (h as anomaly)
  const double* obs_q;       // lambda * w_o / sigma_o^2
  double* jpart;             // per-tile cost accumulator
  const int32_t* nbr_idx;
  const int32_t* hsrc;
  const int32_t* hoff;
  const int32_t* hsign;
  const int32_t* hgcell;
  const uint8_t* active;     // per subdomain, 0 = skip (nullptr = all active)
  uint32_t* nonfinite;       // set to 1 when a cost or first-level adjoint / gradient
                             // entry is NaN or Inf (read and cleared by the host)
  // slot of the state arena holding each local level: the level itself when
  // every level is stored; with checkpoints, level pairs n = kc, kc+1 keep
  // their own slots and the others share a segment that the adjoint refills
  const int32_t* zslot;
  T st, stg, h0;
  double mu;
  double isb2[3];            // 1 / sigma_b^2
  int32_t nlon, half, maxlev, weight_mode;
};

// flags a non-finite output value (no store while every value is finite)
__device__ __forceinline__ void flag_nonfinite(uint32_t* flag, bool bad) {
  if (bad && flag) atomicOr(flag, 1u);
}

// state of local level n of subdomain S
template <typename T>
__device__ __forceinline__ T* zlevel(const Dom<T>& D, const SubDev& S, int n) {
  return D.traj + S.zoff + int64_t(D.zslot[n]) * 3 * S.ncell;
}

}  // namespace dd4dvar
