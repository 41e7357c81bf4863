// Stencil helpers shared by the step kernels (sweep.hip) and the per-box
// kernels (box.hip): neighbour indexing of a box cell (inside, wrapped, or a
// frozen ring position) and branch-free loads.
#pragma once

#include "kernels.h"

namespace dd4dvar {
namespace stencil {


template <typename T>
struct V3 {
  T h, u, v;
};

template <typename T>
__device__ __forceinline__ V3<T> ld_box(const T* Z, int64_t plane, int64_t idx, T sgn) {
  return {Z[idx], sgn * Z[plane + idx], sgn * Z[2 * plane + idx]};
}

template <typename T>
__device__ __forceinline__ V3<T> ld_ring(const T* R, int nring, int k) {
  return {R[k], R[nring + k], R[2 * nring + k]};
}

// Neighbour positions of box cell (r, c): index into the box (>= 0) or ring
// position (encoded as -1 - k), plus the sign applied to u, v.  Computed
// with selects only, so that every neighbour load is issued unconditionally
// (branches around loads make the compiler wait for each one in turn).
struct NbrIdx {
  int e, w, n, s;
  int sn, ss;       // -1 across a pole
};

__device__ __forceinline__ NbrIdx nbr_index(const SubDev& S, int r, int c, int half) {
  NbrIdx q;
  const int m = r * S.nx + c;
  int ch = c + half;                       // column across the pole (span boxes)
  ch = ch >= S.nx ? ch - S.nx : ch;
  const bool e_in = c + 1 < S.nx, w_in = c > 0, n_in = r + 1 < S.ny, s_in = r > 0;
  q.e = e_in ? m + 1 : (S.span ? m + 1 - S.nx : -1 - (2 * S.nx + S.ny + r));
  q.w = w_in ? m - 1 : (S.span ? m - 1 + S.nx : -1 - (2 * S.nx + r));
  q.n = n_in ? m + S.nx : (S.pole_n ? r * S.nx + ch : -1 - (S.nx + c));
  q.s = s_in ? m - S.nx : (S.pole_s ? ch : -1 - c);
  q.sn = (!n_in && S.pole_n) ? -1 : 1;
  q.ss = (!s_in && S.pole_s) ? -1 : 1;
  return q;
}

template <typename T>
__device__ __forceinline__ V3<T> ld_nbr(const T* Z, const T* R, int64_t plane, int nring,
                                        int idx, int sgn) {
  const bool in = idx >= 0;
  const T* p = in ? Z + idx : R + (-1 - idx);
  const int64_t st = in ? plane : int64_t(nring);
  const T sg = T(in ? sgn : 1);
  return {p[0], sg * p[st], sg * p[2 * st]};
}

// Adjoint of level n+1 at a neighbour, zero when the neighbour is a frozen
// ring position (its increment is not part of the local model).  The load
// is unconditional (from the cell itself when the neighbour is frozen).
template <typename T>
__device__ __forceinline__ V3<T> ld_lam(const T* L1, int64_t plane, int idx, int m) {
  const bool in = idx >= 0;
  const int i = in ? idx : m;
  const T h = L1[i], u = L1[plane + i], v = L1[2 * plane + i];
  return {in ? h : T(0), in ? u : T(0), in ? v : T(0)};
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < int(blockDim.x >> 6); ++i) r += sh[i];
  return r;
}


}  // namespace stencil
}  // namespace dd4dvar
