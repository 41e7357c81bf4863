// The solvers' vector work over parts: each box's packed control (3 ncell
// FP64 entries) is cut into parts of at most kPartLen entries, one workgroup
// per part, so that a launch holds many workgroups whether the decomposition
// has thousands of small boxes or a few that cover the sphere.  A per-box
// scalar (a dot product, a norm, a maximum) is the sum over the box's parts,
// in part order, of the partial sums that each workgroup leaves in a slot:
// the same bits for every reader, whatever the launch order.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace dd4dvar {

constexpr int kPartB = 256;          // threads per part workgroup
constexpr int kPartLen = 16384;      // entries per part (64 per thread)
constexpr int kPartSlots = 4;        // partial-sum slots per part

struct Part {
  int64_t off;        // packed control offset of the box
  int64_t cell_off;   // the box's per-cell coverage offset
  int32_t box;
  int32_t ncell;      // cells of the box: entry i is field i / ncell
  int32_t lo, hi;     // entries [lo, hi) of the box
};

struct PartMap {
  const Part* part;   // every box's parts, box by box, in entry order
  const int2* box;    // per box: (first part, number of parts)
  int nparts;
  double* acc;        // [kPartSlots][nparts] partial sums
};

// sum over a kPartB-thread workgroup, returned to every thread
__device__ inline double part_bsum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();                   // sh may still be read from a previous call
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < kPartB / 64; ++i) r += sh[i];
  return r;
}

__device__ inline double part_bmax(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = sh[0];
  for (int i = 1; i < kPartB / 64; ++i) r = fmax(r, sh[i]);
  return r;
}

// the workgroup's partial sum of v into slot k of part p
__device__ inline void part_put(const PartMap& M, int k, int p, double v, double* sh) {
  v = part_bsum(v, sh);
  if (threadIdx.x == 0) M.acc[int64_t(k) * M.nparts + p] = v;
}

// total of slot k over box s's parts, for a whole wave (every lane active):
// lane-strided sums in part order, then a butterfly whose pairs add the same
// two values in either order, so that every lane, and every wave that asks,
// holds the same bits
__device__ inline double box_total(const PartMap& M, int k, int s) {
  const int2 b = M.box[s];
  const double* a = M.acc + int64_t(k) * M.nparts + b.x;
  double v = 0.0;
  for (int j = int(threadIdx.x & 63); j < b.y; j += 64) v += a[j];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double box_max(const PartMap& M, int k, int s) {
  const int2 b = M.box[s];
  const double* a = M.acc + int64_t(k) * M.nparts + b.x;
  double v = 0.0;
  for (int j = int(threadIdx.x & 63); j < b.y; j += 64) v = fmax(v, a[j]);
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// one wave per box for the per-box scalar kernels
constexpr int kBoxWaves = 4;
__device__ inline int wave_box() {
  return int(blockIdx.x) * kBoxWaves + int(threadIdx.x >> 6);
}
inline unsigned box_wave_blocks(int nsub) {
  return unsigned((nsub + kBoxWaves - 1) / kBoxWaves);
}

}  // namespace dd4dvar
