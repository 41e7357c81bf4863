// Batched forward and adjoint sweeps of the restricted shallow-water model
// over every subdomain at once (one workgroup per 256-cell tile of a box).
//
// Forward (restricted model, eq. restricted; discrete U, V, H of Sec. 7 with
// p = q = 1, alpha = 0): Z^1 = Z^0 + F(Z^0)/2, Z^{n+1} = Z^{n-1} + F(Z^n),
// where F is the centred 2 dt increment; neighbours outside the box come from
// the frozen halo ring of that level or, for boxes spanning the circle, from
// the box itself across the seam or the pole (u, v negated across a pole).
// h is stored as h - h_ref; the height flux difference is formed as
// h_ref * (difference of u) + difference of (h - h_ref) u, so FP32 storage
// keeps the anomaly resolution.
//
// Adjoint (adjoint definition of Sec. 2, applied step by step in reverse,
// eq. adjProd): with lambda^n the adjoint of level n,
//   lambda^n = forcing^n + lambda^{n+2} + J_F(Z^n)^T lambda^{n+1}   (n >= 1)
//   lambda^0 = forcing^0 + lambda^2 + lambda^1 + J_F(Z^0)^T lambda^1 / 2
// computed in gather form: each cell collects the transposed stencil
// coefficients of itself and of the neighbours whose increment reads it.
// The forcing is the derivative of the observation and overlap terms of the
// local functional (eq. eq:cost:parallel1), fused into the same pass, which
// also accumulates the cost in FP64 per tile.
#include "kernels.h"
#include "launch.h"
#include "stencil.h"

#ifndef DD4DVAR_SWEEP_T
#error "compile with -DDD4DVAR_SWEEP_T=float or double"
#endif

namespace dd4dvar {

using namespace stencil;

// Z^0 = x - (h_ref, 0, 0)
template <typename T>
__global__ __launch_bounds__(kTile) void k_init(Dom<T> D, const double* __restrict__ x,
                                                int tile_base) {
  const int2 wt = D.tiles[tile_base + xcd_tile(blockIdx.x, gridDim.x)];
  if (D.active && !D.active[wt.x]) return;
  const SubDev S = D.subs[wt.x];
  const int m = wt.y * kTile + threadIdx.x;
  if (m >= S.ncell) return;
  const double* xs = x + S.ctrl_off;
  T* Z = zlevel(D, S, 0);
  Z[m] = T(xs[m] - double(D.h0));
  Z[S.ncell + m] = T(xs[S.ncell + m]);
  Z[2 * S.ncell + m] = T(xs[2 * S.ncell + m]);
}

template <typename T>
__global__ __launch_bounds__(kTile) void k_fwd(Dom<T> D, int n, int tile_base) {
  const int2 wt = D.tiles[tile_base + xcd_tile(blockIdx.x, gridDim.x)];
  if (D.active && !D.active[wt.x]) return;
  const SubDev S = D.subs[wt.x];
  if (n >= S.nlev - 1) return;
  const int m = wt.y * kTile + threadIdx.x;
  if (m >= S.ncell) return;
  const int r = m / S.nx, c = m - r * S.nx;
  const int64_t plane = S.ncell;
  const T* Z = zlevel(D, S, n);
  const T* R = D.ring + S.ring_off + int64_t(n) * 3 * S.nring;
  const NbrIdx q = nbr_index(S, r, c, D.half);
  // level n-1 (level 0 itself for the Euler start, whose base is Z^0)
  const T* P = n >= 1 ? zlevel(D, S, n - 1) : Z;
  const int j = S.row0 + r;
  // every load first, unconditionally
  const V3<T> C = ld_box(Z, plane, m, T(1));
  const V3<T> E = ld_nbr(Z, R, plane, S.nring, q.e, 1);
  const V3<T> W = ld_nbr(Z, R, plane, S.nring, q.w, 1);
  const V3<T> N = ld_nbr(Z, R, plane, S.nring, q.n, q.sn);
  const V3<T> Sv = ld_nbr(Z, R, plane, S.nring, q.s, q.ss);
  const V3<T> B = ld_box(P, plane, m, T(1));
  const RowCoef<T> rc = D.rows[j];
  const T cN = D.cosx[j + 2], cS = D.cosx[j];
  const T st = D.st, stg = D.stg, h0 = D.h0;
  const T cor = rc.cf + rc.ct * C.u;
  const T U = -rc.a1 * C.u * (E.u - W.u) - st * C.v * (N.u - Sv.u) - rc.a2 * (E.h - W.h) + cor * C.v;
  const T V = -rc.a1 * C.u * (E.v - W.v) - st * C.v * (N.v - Sv.v) - stg * (N.h - Sv.h) - cor * C.u;
  const T H = -rc.a1 * (h0 * (E.u - W.u) + (E.h * E.u - W.h * W.u))
              - rc.a3 * (h0 * (N.v * cN - Sv.v * cS) + (N.h * N.v * cN - Sv.h * Sv.v * cS));
  const T wgt = n == 0 ? T(0.5) : T(1);
  T* out = zlevel(D, S, n + 1);
  out[m] = B.h + wgt * H;
  out[plane + m] = B.u + wgt * U;
  out[2 * plane + m] = B.v + wgt * V;
}

// mode 0: cost forcing (observations + overlap), writes grad and J at level 0
// mode 1: caller forcing (packed FP64, trajectory layout), writes adj0
// mode 2: cost forcing, writes adj0 (no background term)
// mode 3: Gauss-Newton forcing W dZ^n from the tangent-linear trajectory
//         (the observation and overlap weights of the cost applied to the
//         perturbation; eq. line5and7), writes adj0, no cost
template <typename T, int MODE>
__global__ __launch_bounds__(kTile) void k_adj(Dom<T> D, int n, int tile_base,
                                               const double* __restrict__ x,
                                               const double* __restrict__ xb,
                                               const double* __restrict__ forcing,
                                               double* __restrict__ out) {
  __shared__ double fo[3][kTile];
  __shared__ double red[kTile / 64];
  const int w = tile_base + xcd_tile(blockIdx.x, gridDim.x);
  const int2 wt = D.tiles[w];
  if (D.active && !D.active[wt.x]) return;  // uniform over the block
  const SubDev S = D.subs[wt.x];
  const int L = S.nlev - 1;
  if (n > L) return;                      // uniform over the block
  const int m = wt.y * kTile + threadIdx.x;
  const bool valid = m < S.ncell;
  const int mm = valid ? m : 0;           // a valid address for inactive lanes
  const int64_t plane = S.ncell;
  const T* Z = zlevel(D, S, n);
  const T* R = D.ring + S.ring_off + int64_t(n) * 3 * S.nring;
  T* A = D.adj + S.adj_off;
  const bool has1 = n + 1 <= L, has2 = n + 2 <= L;       // uniform
  const T* L1 = A + int64_t((n + 1) % 3) * 3 * plane;
  const T* L2 = A + int64_t((n + 2) % 3) * 3 * plane;
  double jloc = 0.0;

  // ---- issue every load of this cell first (selects, no branches) ---------
  int K = 0;                               // other extended boxes covering (n, m)
  if (MODE != 1) K = int(D.cover[S.cell_off + mm]) * D.tcount[S.lev0 + n] - 1;
  const int r = mm / S.nx, c = mm - r * S.nx;
  const NbrIdx q = nbr_index(S, r, c, D.half);
  const int j = S.row0 + r;
  // rows of the north / south neighbours whose increments read this cell
  const int jn = (q.n >= 0 && q.sn > 0) ? j + 1 : j;
  const int js = (q.s >= 0 && q.ss > 0) ? j - 1 : j;
  const RowCoef<T> rc = D.rows[j];
  const T a3n = D.rows[jn].a3, a3s = D.rows[js].a3;
  const V3<T> C = ld_box(Z, plane, mm, T(1));
  const V3<T> E = ld_nbr(Z, R, plane, S.nring, q.e, 1);
  const V3<T> W = ld_nbr(Z, R, plane, S.nring, q.w, 1);
  const V3<T> N = ld_nbr(Z, R, plane, S.nring, q.n, q.sn);
  const V3<T> Sv = ld_nbr(Z, R, plane, S.nring, q.s, q.ss);
  V3<T> l0 = ld_box(L1, plane, mm, T(1));
  V3<T> kE = ld_lam(L1, plane, q.e, mm);
  V3<T> kW = ld_lam(L1, plane, q.w, mm);
  V3<T> kN = ld_lam(L1, plane, q.n, mm);
  V3<T> kS = ld_lam(L1, plane, q.s, mm);
  V3<T> l2 = ld_box(L2, plane, mm, T(1));
  double fh = 0, fu = 0, fv = 0;
  V3<T> tg = {T(0), T(0), T(0)};
  if (MODE == 3) {
    // the perturbation at the cell takes the place of the overlap residual
    tg = ld_box(D.dz + S.zoff + int64_t(n) * 3 * plane, plane, mm, T(1));
  } else if (MODE != 1) {
    // cells outside every overlap all read element 0 (one shared cache line)
    // instead of branching around the load; their weight K is zero
    tg = ld_box(D.targ + S.traj_off + int64_t(n) * 3 * plane, plane, K > 0 ? mm : 0, T(1));
  } else {
    const double* Fz = forcing + S.traj_off + int64_t(n) * 3 * plane;
    fh = Fz[mm];
    fu = Fz[plane + mm];
    fv = Fz[2 * plane + mm];
  }

  // ---- observation misfits of this tile at level n (uniform test) --------
  if (MODE != 1) {
    const int64_t key = obs_key(S.tile0, S.ntile, D.maxlev, wt.y, n);
    const int o0 = D.obs_ptr[key], o1 = D.obs_ptr[key + 1];
    if (o1 > o0) {
      fo[0][threadIdx.x] = 0.0;
      fo[1][threadIdx.x] = 0.0;
      fo[2][threadIdx.x] = 0.0;
      __syncthreads();
      for (int o = o0 + int(threadIdx.x); o < o1; o += kTile) {
        const int code = D.obs_code[o];
        const int loc = code >> 2, f = code & 3;
        const double rr = MODE == 3 ? double(D.dz[S.zoff + int64_t(n) * 3 * plane + f * plane + loc])
                                    : double(Z[f * plane + loc]) - D.obs_val[o];
        const double qo = D.obs_q[o];
        if (MODE != 3) jloc += 0.5 * qo * rr * rr;
        fo[f][loc - wt.y * kTile] = qo * rr;
      }
      __syncthreads();
      fh = fo[0][threadIdx.x];
      fu = fo[1][threadIdx.x];
      fv = fo[2][threadIdx.x];
    }
  }

  if (valid) {
    if (!has1) l0 = kE = kW = kN = kS = V3<T>{T(0), T(0), T(0)};
    if (!has2) l2 = V3<T>{T(0), T(0), T(0)};
    const T st = D.st, stg = D.stg;
    const T hm = D.h0 + C.h;

    // J_F(Z^n)^T lambda^{n+1}: self terms, then the neighbours k whose
    // increment reads this cell (east k sees it as west, north k as south,
    // across a pole the north k sees it as north with u, v negated)
    T au = l0.u * (-rc.a1 * (E.u - W.u) + rc.ct * C.v) +
           l0.v * (-rc.a1 * (E.v - W.v) - rc.cf - T(2) * rc.ct * C.u);
    T av = l0.u * (-st * (N.u - Sv.u) + rc.cf + rc.ct * C.u) + l0.v * (-st * (N.v - Sv.v));
    T ah = T(0);
    au += rc.a1 * (kE.u * E.u + kE.h * hm) - rc.a1 * (kW.u * W.u + kW.h * hm);
    av += rc.a1 * kE.v * E.u - rc.a1 * kW.v * W.u;
    ah += (rc.a2 * kE.u + rc.a1 * kE.h * C.u) - (rc.a2 * kW.u + rc.a1 * kW.h * C.u);
    const T vkn = T(q.sn) * N.v, vks = T(q.ss) * Sv.v;    // raw v at the neighbours
    au += kN.u * st * vkn - kS.u * st * vks;
    av += (kN.v * st * vkn + kN.h * a3n * hm * rc.c) - (kS.v * st * vks + kS.h * a3s * hm * rc.c);
    ah += (T(q.sn) * kN.v * stg + kN.h * a3n * C.v * rc.c) -
          (T(q.ss) * kS.v * stg + kS.h * a3s * C.v * rc.c);
    if (n == 0) {
      au = l0.u + T(0.5) * au;
      av = l0.v + T(0.5) * av;
      ah = l0.h + T(0.5) * ah;
    }
    // overlap misfit: K copies of (Z - mean target) / sigma_b^2
    if (MODE != 1) {
      const double eh = MODE == 3 ? double(tg.h) : double(C.h) - double(tg.h);
      const double eu = MODE == 3 ? double(tg.u) : double(C.u) - double(tg.u);
      const double ev = MODE == 3 ? double(tg.v) : double(C.v) - double(tg.v);
      const double mk = D.mu * double(K);
      fh += mk * eh * D.isb2[0];
      fu += mk * eu * D.isb2[1];
      fv += mk * ev * D.isb2[2];
      if (MODE != 3)
        jloc += 0.5 * mk * (eh * eh * D.isb2[0] + eu * eu * D.isb2[1] + ev * ev * D.isb2[2]);
    }
    const double bh = fh + double(ah) + double(l2.h);
    const double bu = fu + double(au) + double(l2.u);
    const double bv = fv + double(av) + double(l2.v);
    if (n > 0) {
      T* B = A + int64_t(n % 3) * 3 * plane;
      B[m] = T(bh);
      B[plane + m] = T(bu);
      B[2 * plane + m] = T(bv);
    } else if (MODE == 0) {
      const int64_t o = S.ctrl_off + m;
      const double wb = D.weight_mode ? 1.0 : 1.0 / double(D.cover[S.cell_off + m]);
      const double dh = x[o] - xb[o];
      const double du = x[o + plane] - xb[o + plane];
      const double dv = x[o + 2 * plane] - xb[o + 2 * plane];
      const double gh = wb * dh * D.isb2[0] + bh;
      const double gu = wb * du * D.isb2[1] + bu;
      const double gv = wb * dv * D.isb2[2] + bv;
      out[o] = gh;
      out[o + plane] = gu;
      out[o + 2 * plane] = gv;
      flag_nonfinite(D.nonfinite, !(isfinite(gh) && isfinite(gu) && isfinite(gv)));
      jloc += 0.5 * wb * (dh * dh * D.isb2[0] + du * du * D.isb2[1] + dv * dv * D.isb2[2]);
    } else {
      const int64_t o = S.ctrl_off + m;
      out[o] = bh;
      out[o + plane] = bu;
      out[o + 2 * plane] = bv;
      flag_nonfinite(D.nonfinite, !(isfinite(bh) && isfinite(bu) && isfinite(bv)));
    }
  }
  if (MODE == 0 || MODE == 2) {
    const double tot = block_sum(jloc, red);
    if (threadIdx.x == 0) D.jpart[w] = (n == L) ? tot : D.jpart[w] + tot;
  }
}

#if DD4DVAR_SWEEP_PRIMARY
// J[s] = sum of tile partials + constant overlap part, one wave per box: lane
// l sums tiles l, l + 64, ... in order, then a butterfly whose pairs add the
// same two values in either order (a fixed order, whatever the box size: a
// box of thousands of tiles is not left to one thread)
__global__ __launch_bounds__(256) void k_reduce_j(const SubDev* __restrict__ subs, int count,
                                                  const int32_t* __restrict__ ids,
                                                  const double* __restrict__ jpart,
                                                  const double* __restrict__ jconst,
                                                  double* __restrict__ J,
                                                  uint32_t* __restrict__ nonfinite) {
  const int i = int(blockIdx.x) * 4 + int(threadIdx.x >> 6);
  if (i >= count) return;                   // uniform over the wave
  const int s = ids ? ids[i] : i;
  const SubDev S = subs[s];
  double acc = 0.0;
  for (int t = int(threadIdx.x & 63); t < S.ntile; t += 64) acc += jpart[S.tile0 + t];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) != 0) return;
  acc += jconst[s];
  J[s] = acc;
  if (!isfinite(acc)) atomicOr(nonfinite, 1u);
}
#endif

// packed FP64 trajectory output (h + h_ref): every level (level < 0) or one
template <typename T>
__global__ __launch_bounds__(kTile) void k_traj_out(Dom<T> D, double* __restrict__ out, int tile_base,
                                                    int level) {
  const int2 wt = D.tiles[tile_base + xcd_tile(blockIdx.x, gridDim.x)];
  const SubDev S = D.subs[wt.x];
  const int m = wt.y * kTile + threadIdx.x;
  if (m >= S.ncell) return;
  const int64_t plane = S.ncell;
  const int n0 = level < 0 ? 0 : level, n1 = level < 0 ? S.nlev : (level < S.nlev ? level + 1 : level);
  for (int n = n0; n < n1; ++n) {
    const T* Z = zlevel(D, S, n);
    double* o = out + S.traj_off + int64_t(n) * 3 * plane;
    o[m] = double(Z[m]) + double(D.h0);
    o[plane + m] = double(Z[plane + m]);
    o[2 * plane + m] = double(Z[2 * plane + m]);
  }
}

// ---- launchers --------------------------------------------------------------
template <typename T>
void launch_init(const Dom<T>& D, const double* x, int tile_base, int ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_init<T>, dim3(ntiles), dim3(kTile), 0, st, D, x, tile_base);
}
template <typename T>
void launch_fwd(const Dom<T>& D, int n, int tile_base, int ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_fwd<T>, dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base);
}
template <typename T>
void launch_adj(const Dom<T>& D, int n, int tile_base, int ntiles, int mode, const double* x,
                const double* xb, const double* forcing, double* out, hipStream_t st) {
  if (mode == 0)
    hipLaunchKernelGGL((k_adj<T, 0>), dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base, x, xb,
                       forcing, out);
  else if (mode == 1)
    hipLaunchKernelGGL((k_adj<T, 1>), dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base, x, xb,
                       forcing, out);
  else if (mode == 2)
    hipLaunchKernelGGL((k_adj<T, 2>), dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base, x, xb,
                       forcing, out);
  else
    hipLaunchKernelGGL((k_adj<T, 3>), dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base, x, xb,
                       forcing, out);
}
#if DD4DVAR_SWEEP_PRIMARY
void launch_reduce_j(const SubDev* subs, int count, const int32_t* ids, const double* jpart,
                     const double* jconst, double* J, uint32_t* nonfinite, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_j, dim3((count + 3) / 4), dim3(256), 0, st, subs, count, ids, jpart,
                     jconst, J, nonfinite);
}
#endif
template <typename T>
void launch_traj_out(const Dom<T>& D, double* out, int tile_base, int ntiles, int level,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_traj_out<T>, dim3(ntiles), dim3(kTile), 0, st, D, out, tile_base, level);
}

#define DD4DVAR_INST(T)                                                                        \
  template void launch_init<T>(const Dom<T>&, const double*, int, int, hipStream_t);          \
  template void launch_fwd<T>(const Dom<T>&, int, int, int, hipStream_t);                      \
  template void launch_adj<T>(const Dom<T>&, int, int, int, int, const double*, const double*, \
                              const double*, double*, hipStream_t);                            \
  template void launch_traj_out<T>(const Dom<T>&, double*, int, int, int, hipStream_t);
// This source is compiled once per state type: FP32 with the compiler's
// default contraction, FP64 with -ffp-contract=off so that FP64 results follow
// the rounding of the separate multiplies and adds of the reference.
DD4DVAR_INST(DD4DVAR_SWEEP_T)
#undef DD4DVAR_INST

}  // namespace dd4dvar
