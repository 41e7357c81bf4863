// Exchange between subdomains in device memory ("Exchange u_ji between
// adjacent subdomains", Alg. 1) and the partition-of-unity gather (eq. rest).
//
// * Halo rings: every frozen ring position of subdomain s reads, at each of
//   its levels, the core owner of the (pole-mapped) cell in the same time
//   interval, with u and v negated across a pole.
// * Overlap targets: for every (level, cell) of s covered by K other extended
//   space-time boxes, the mean of their trajectories there and, once per
//   subdomain, the constant sum_{s'} (T_{s'} - mean)^2 / sigma_b^2, so that
//   sum_{s'} (Z - T_{s'})^2 = K (Z - mean)^2 + constant.
// * Before any local solve both come from the global background run.
#include "kernels.h"
#include "launch.h"

namespace dd4dvar {

namespace {
// neighbour entries of a level whose loads are issued together (FP64 values
// take twice the registers)
template <typename T>
constexpr int kGather = sizeof(T) == 4 ? 8 : 4;

__device__ __forceinline__ double block_sum2(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < int(blockDim.x >> 6); ++i) r += sh[i];
  return r;
}

}  // namespace

// targets (and backgrounds at level 0) from the global FP64 trajectory, whose
// h is stored as h - h_ref
template <typename T>
__global__ __launch_bounds__(kTile) void k_from_global(Dom<T> D, const double* __restrict__ bg,
                                                       int64_t gplane, double* __restrict__ xb,
                                                       int n) {
  const int2 wt = D.tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const SubDev S = D.subs[wt.x];
  if (n >= S.nlev) return;
  const int m = wt.y * kTile + threadIdx.x;
  if (m >= S.ncell) return;
  const int r = m / S.nx, c = m - r * S.nx;
  int gcol = S.col0 + c;
  if (gcol >= D.nlon) gcol -= D.nlon;
  const int64_t g = int64_t(S.row0 + r) * D.nlon + gcol;
  const double* B = bg + int64_t(S.lev0 + n) * 3 * gplane;
  const int64_t plane = S.ncell;
  T* Tg = D.targ + S.traj_off + int64_t(n) * 3 * plane;
  Tg[m] = T(B[g]);
  Tg[plane + m] = T(B[gplane + g]);
  Tg[2 * plane + m] = T(B[2 * gplane + g]);
  if (n == 0) {
    double* xo = xb + S.ctrl_off;
    xo[m] = B[g] + double(D.h0);
    xo[plane + m] = B[gplane + g];
    xo[2 * plane + m] = B[2 * gplane + g];
  }
}

template <typename T>
__global__ void k_ring_from_global(Dom<T> D, const double* __restrict__ bg, int64_t gplane) {
  const SubDev S = D.subs[blockIdx.x];
  const int k = blockIdx.y * blockDim.x + threadIdx.x;
  if (k >= S.nring) return;
  const int src = D.hsrc[S.hmap_off + k];
  if (src < 0) return;
  const int64_t g = D.hgcell[S.hmap_off + k];
  const T sg = T(D.hsign[S.hmap_off + k]);
  for (int n = 0; n < S.nlev; ++n) {
    const double* B = bg + int64_t(S.lev0 + n) * 3 * gplane;
    T* R = D.ring + S.ring_off + int64_t(n) * 3 * S.nring;
    R[k] = T(B[g]);
    R[S.nring + k] = sg * T(B[gplane + g]);
    R[2 * S.nring + k] = sg * T(B[2 * gplane + g]);
  }
}

// every level (level < 0) or one local level of the boxes box_base, ...
template <typename T>
__global__ void k_ring_from_local(Dom<T> D, int box_base, int level) {
  const SubDev S = D.subs[box_base + blockIdx.x];
  const int k = blockIdx.y * blockDim.x + threadIdx.x;
  if (k >= S.nring) return;
  const int src = D.hsrc[S.hmap_off + k];
  if (src < 0) return;
  const SubDev P = D.subs[src];
  const int64_t off = D.hoff[S.hmap_off + k];
  const T sg = T(D.hsign[S.hmap_off + k]);
  const int n0 = level < 0 ? 0 : level, n1 = level < 0 ? S.nlev : (level < S.nlev ? level + 1 : level);
  for (int n = n0; n < n1; ++n) {   // same interval: same levels
    const T* Z = zlevel(D, P, n);
    T* R = D.ring + S.ring_off + int64_t(n) * 3 * S.nring;
    R[k] = Z[off];
    R[S.nring + k] = sg * Z[P.ncell + off];
    R[2 * S.nring + k] = sg * Z[2 * P.ncell + off];
  }
}

// Overlap targets of one local level (level >= 0) or of every level (level
// < 0) of the boxes of a tile range.  Each cell first marks, once, the
// entries of its box's neighbour list whose extended boxes contain it in
// space (one bit per entry, at most 64; the list itself is staged in LDS),
// then at each level visits the entries marked by some lane of its wave and
// takes the mean and the spread of the marked neighbours that hold the
// level, in one pass with sums shifted by the first value (the values of one
// cell differ little between boxes, so the shifted sums lose nothing to
// cancellation).
template <typename T>
__global__ __launch_bounds__(kTile) void k_targets_from_local(Dom<T> D, int level, int tile_base,
                                                              double* __restrict__ jc) {
  __shared__ double red[kTile / 64];
  // the box's neighbour list, staged once: first level, levels, first row
  // and column, width, cells, state offset
  __shared__ int nb_lev0[64], nb_nlev[64], nb_row0[64], nb_col0[64], nb_nx[64], nb_ny[64],
      nb_ncell[64];
  __shared__ int64_t nb_zoff[64];
  const int w = tile_base + xcd_tile(blockIdx.x, gridDim.x);
  const int2 wt = D.tiles[w];
  const SubDev S = D.subs[wt.x];
  const int n0 = level < 0 ? 0 : level, n1 = level < 0 ? S.nlev : level + 1;
  if (n0 >= S.nlev) return;                 // uniform over the block
  const int nq = S.nbr1 - S.nbr0;           // <= 64 (checked at set-up)
  for (int i = threadIdx.x; i < nq; i += kTile) {
    const SubDev P = D.subs[D.nbr_idx[S.nbr0 + i]];
    nb_lev0[i] = P.lev0;
    nb_nlev[i] = P.nlev;
    nb_row0[i] = P.row0;
    nb_col0[i] = P.col0;
    nb_nx[i] = P.nx;
    nb_ny[i] = P.ny;
    nb_ncell[i] = P.ncell;
    nb_zoff[i] = P.zoff;
  }
  __syncthreads();
  const int m = wt.y * kTile + threadIdx.x;
  const bool valid = m < S.ncell;
  const int mm = valid ? m : 0;
  const int r = mm / S.nx, c = mm - r * S.nx;
  const int grow = S.row0 + r;
  int gcol = S.col0 + c;
  if (gcol >= D.nlon) gcol -= D.nlon;
  // per lane: the entries whose boxes contain the cell; per wave: their union
  uint64_t hits = 0;
  for (int i = 0; i < nq; ++i) {
    const int rr = grow - nb_row0[i];
    int cc = gcol - nb_col0[i];
    if (cc < 0) cc += D.nlon;
    if (valid && rr >= 0 && rr < nb_ny[i] && cc < nb_nx[i])
      hits |= uint64_t(1) << i;
  }
  uint32_t wlo = uint32_t(hits), whi = uint32_t(hits >> 32);
  for (int off = 32; off > 0; off >>= 1) {
    wlo |= __shfl_xor(wlo, off, 64);
    whi |= __shfl_xor(whi, off, 64);
  }
  // the union is the same in every lane: keep it in scalar registers
  const uint64_t wave_hits = (uint64_t(__builtin_amdgcn_readfirstlane(whi)) << 32) |
                             uint32_t(__builtin_amdgcn_readfirstlane(wlo));
  // lane i < nq holds entry i's level range, for one ballot per level
  const int lane = threadIdx.x & 63;
  const int my_lev0 = lane < nq ? nb_lev0[lane] : 0, my_nlev = lane < nq ? nb_nlev[lane] : 0;
  const int cov = valid ? int(D.cover[S.cell_off + mm]) : 0;
  const int64_t plane = S.ncell;
  double acc = 0.0;                         // thread 0: the tile's sum over levels
  for (int n = n0; n < n1; ++n) {
    double jloc = 0.0;
    const int K = cov * D.tcount[S.lev0 + n] - 1;
    const int gl = S.lev0 + n;
    // entries that some lane of the wave hits and that hold the level, in
    // list order; the first kGather<T> of them are loaded together, before any
    // is used, then summed in list order
    const int my_pl = gl - my_lev0;
    uint64_t rem = wave_hits & uint64_t(__ballot(my_pl >= 0 && my_pl < my_nlev));
    T zh[kGather<T>], zu[kGather<T>], zv[kGather<T>];
    bool hk[kGather<T>];
#pragma unroll
    for (int k = 0; k < kGather<T>; ++k) {
      hk[k] = false;
      zh[k] = zu[k] = zv[k] = T(0);
      if (rem) {                                               // uniform
        const int i = __builtin_ctzll(rem);
        rem &= rem - 1;
        hk[k] = (hits >> i) & 1;
        if (hk[k]) {
          const int pl = gl - nb_lev0[i];
          const int rr = grow - nb_row0[i];
          int cc = gcol - nb_col0[i];
          if (cc < 0) cc += D.nlon;
          const int64_t pc = nb_ncell[i];
          const T* Z = D.traj + nb_zoff[i] + int64_t(D.zslot[pl]) * 3 * pc + int64_t(rr) * nb_nx[i] + cc;
          zh[k] = Z[0];
          zu[k] = Z[pc];
          zv[k] = Z[2 * pc];
        }
      }
    }
    double ch = 0, cu = 0, cv = 0;                 // shift: the first value
    double ah = 0, au = 0, av = 0, bh = 0, bu = 0, bv = 0;
    int cnt = 0;
    auto add = [&](double z0, double z1, double z2) {
      if (cnt == 0) {
        ch = z0;
        cu = z1;
        cv = z2;
      }
      const double dh = z0 - ch, du = z1 - cu, dv = z2 - cv;
      ah += dh;
      au += du;
      av += dv;
      bh += dh * dh;
      bu += du * du;
      bv += dv * dv;
      ++cnt;
    };
#pragma unroll
    for (int k = 0; k < kGather<T>; ++k)
      if (hk[k]) add(double(zh[k]), double(zu[k]), double(zv[k]));
    for (; rem; rem &= rem - 1) {                              // beyond kGather<T> entries
      const int i = __builtin_ctzll(rem);
      if (!((hits >> i) & 1)) continue;
      const int pl = gl - nb_lev0[i];
      const int rr = grow - nb_row0[i];
      int cc = gcol - nb_col0[i];
      if (cc < 0) cc += D.nlon;
      const int64_t pc = nb_ncell[i];
      const T* Z = D.traj + nb_zoff[i] + int64_t(D.zslot[pl]) * 3 * pc + int64_t(rr) * nb_nx[i] + cc;
      add(double(Z[0]), double(Z[pc]), double(Z[2 * pc]));
    }
    if (K > 0 && cnt > 0) {
      const double inv = 1.0 / double(cnt);
      T* Tg = D.targ + S.traj_off + int64_t(n) * 3 * plane;
      Tg[m] = T(ch + ah * inv);
      Tg[plane + m] = T(cu + au * inv);
      Tg[2 * plane + m] = T(cv + av * inv);
      // sum over the neighbours of (value - mean)^2
      const double sh = bh - ah * ah * inv, su = bu - au * au * inv, sv = bv - av * av * inv;
      jloc = sh * D.isb2[0] + su * D.isb2[1] + sv * D.isb2[2];
    }
    // the level's tile sum, added in level order (as one launch per level
    // adds them), so both ways give the same bits
    __syncthreads();                        // red may still be read from the previous level
    const double tot = block_sum2(jloc, red);
    if (threadIdx.x == 0) acc = (n == n0) ? tot : acc + tot;
  }
  if (threadIdx.x == 0) jc[w] = (n0 == 0) ? acc : jc[w] + acc;
}

// one wave per box: lane l sums tiles l, l + 64, ... in order, then a
// butterfly whose pairs add the same two values in either order
__global__ __launch_bounds__(256) void k_reduce_jconst(const SubDev* __restrict__ subs, int nsub,
                                                       const double* __restrict__ jc, double half_mu,
                                                       double* __restrict__ jconst) {
  const int s = int(blockIdx.x) * 4 + int(threadIdx.x >> 6);
  if (s >= nsub) return;                    // uniform over the wave
  const SubDev S = subs[s];
  double acc = 0.0;
  for (int t = int(threadIdx.x & 63); t < S.ntile; t += 64) acc += jc[S.tile0 + t];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) jconst[s] = half_mu * acc;
}

template <typename T>
__global__ void k_gather(Dom<T> D, int nspace, int ntime, int level, int64_t ncell,
                         const int32_t* __restrict__ cptr, const int32_t* __restrict__ cpiece,
                         double* __restrict__ out) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= ncell) return;
  const int row = int(g / D.nlon), col = int(g - int64_t(row) * D.nlon);
  double ah = 0, au = 0, av = 0;
  int cnt = 0;
  for (int q = cptr[g]; q < cptr[g + 1]; ++q) {
    const int p = cpiece[q];
    for (int j = 0; j < ntime; ++j) {
      const SubDev S = D.subs[j * nspace + p];
      if (level < S.lev0 || level >= S.lev0 + S.nlev) continue;
      int cc = col - S.col0;
      if (cc < 0) cc += D.nlon;
      const T* Z = zlevel(D, S, level - S.lev0) + int64_t(row - S.row0) * S.nx + cc;
      ah += double(Z[0]);
      au += double(Z[S.ncell]);
      av += double(Z[2 * S.ncell]);
      ++cnt;
    }
  }
  const double inv = 1.0 / double(cnt);
  out[g] = ah * inv + double(D.h0);
  out[ncell + g] = au * inv;
  out[2 * ncell + g] = av * inv;
}

__global__ void k_add_href(double* traj, int64_t nlev, int64_t plane, double h0) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nlev * plane) return;
  const int64_t n = i / plane, g = i - n * plane;
  traj[n * 3 * plane + g] += h0;
}

__global__ void k_fill(double* p, int64_t n, double v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---- launchers --------------------------------------------------------------
template <typename T>
void launch_from_global(const Dom<T>& D, const double* bg, int64_t gplane, double* xb, int level,
                        int ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_from_global<T>, dim3(ntiles), dim3(kTile), 0, st, D, bg, gplane, xb, level);
}
// grid.y covers the largest ring; positions beyond a box's own ring exit
template <typename T>
void launch_ring_from_global(const Dom<T>& D, int nsub, int ring_blocks, const double* bg,
                             int64_t gplane, hipStream_t st) {
  hipLaunchKernelGGL(k_ring_from_global<T>, dim3(nsub, ring_blocks), dim3(256), 0, st, D, bg,
                     gplane);
}
template <typename T>
void launch_ring_from_local(const Dom<T>& D, int box_base, int nbox, int ring_blocks, int level,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_ring_from_local<T>, dim3(nbox, ring_blocks), dim3(256), 0, st, D, box_base,
                     level);
}
template <typename T>
void launch_targets_from_local(const Dom<T>& D, int level, int tile_base, int ntiles, double* jc,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_targets_from_local<T>, dim3(ntiles), dim3(kTile), 0, st, D, level, tile_base,
                     jc);
}
void launch_reduce_jconst(const SubDev* subs, int nsub, const double* jc, double half_mu,
                          double* jconst, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_jconst, dim3((nsub + 3) / 4), dim3(256), 0, st, subs, nsub, jc, half_mu,
                     jconst);
}
template <typename T>
void launch_gather(const Dom<T>& D, int nspace, int ntime, int level, int64_t ncell,
                   const int32_t* cptr, const int32_t* cpiece, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gather<T>, dim3(unsigned((ncell + 255) / 256)), dim3(256), 0, st, D, nspace,
                     ntime, level, ncell, cptr, cpiece, out);
}
void launch_add_href(double* traj, int64_t nlev, int64_t plane, double h0, hipStream_t st) {
  const int64_t n = nlev * plane;
  hipLaunchKernelGGL(k_add_href, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, traj, nlev,
                     plane, h0);
}
void launch_fill(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, p, n, v);
}

#define DD4DVAR_INST(T)                                                                          \
  template void launch_from_global<T>(const Dom<T>&, const double*, int64_t, double*, int, int,  \
                                      hipStream_t);                                              \
  template void launch_ring_from_global<T>(const Dom<T>&, int, int, const double*, int64_t,      \
                                           hipStream_t);                                         \
  template void launch_ring_from_local<T>(const Dom<T>&, int, int, int, int, hipStream_t);       \
  template void launch_targets_from_local<T>(const Dom<T>&, int, int, int, double*, hipStream_t); \
  template void launch_gather<T>(const Dom<T>&, int, int, int, int64_t, const int32_t*,          \
                                 const int32_t*, double*, hipStream_t);
DD4DVAR_INST(float)
DD4DVAR_INST(double)
#undef DD4DVAR_INST

}  // namespace dd4dvar
