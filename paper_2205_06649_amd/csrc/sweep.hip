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

namespace dd4dvar {

namespace {

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
// position (encoded as -1 - k), plus the sign applied to u, v.
struct NbrIdx {
  int64_t e, w, n, s;
  int8_t sn, ss;       // -1 across a pole
};

__device__ __forceinline__ NbrIdx nbr_index(const SubDev& S, int r, int c, int half) {
  NbrIdx q;
  const int64_t m = int64_t(r) * S.nx + c;
  q.sn = 1;
  q.ss = 1;
  if (c + 1 < S.nx) q.e = m + 1;
  else if (S.span) q.e = m + 1 - S.nx;
  else q.e = -1 - (2 * S.nx + S.ny + r);
  if (c > 0) q.w = m - 1;
  else if (S.span) q.w = m - 1 + S.nx;
  else q.w = -1 - (2 * S.nx + r);
  if (r + 1 < S.ny) q.n = m + S.nx;
  else if (S.pole_n) { q.n = int64_t(r) * S.nx + (c + half) % S.nx; q.sn = -1; }
  else q.n = -1 - (S.nx + c);
  if (r > 0) q.s = m - S.nx;
  else if (S.pole_s) { q.s = (c + half) % S.nx; q.ss = -1; }
  else q.s = -1 - c;
  return q;
}

template <typename T>
__device__ __forceinline__ V3<T> ld_nbr(const T* Z, const T* R, int64_t plane, int nring,
                                        int64_t idx, int sgn) {
  if (idx >= 0) return ld_box(Z, plane, idx, T(sgn));
  return ld_ring(R, nring, int(-1 - idx));
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

}  // namespace

// Z^0 = x - (h_ref, 0, 0)
template <typename T>
__global__ __launch_bounds__(kTile) void k_init(Dom<T> D, const double* __restrict__ x,
                                                int tile_base) {
  const int2 wt = D.tiles[tile_base + blockIdx.x];
  const SubDev S = D.subs[wt.x];
  const int m = wt.y * kTile + threadIdx.x;
  if (m >= S.ncell) return;
  const double* xs = x + S.ctrl_off;
  T* Z = D.traj + S.traj_off;
  Z[m] = T(xs[m] - double(D.h0));
  Z[S.ncell + m] = T(xs[S.ncell + m]);
  Z[2 * S.ncell + m] = T(xs[2 * S.ncell + m]);
}

template <typename T>
__global__ __launch_bounds__(kTile) void k_fwd(Dom<T> D, int n, int tile_base) {
  const int2 wt = D.tiles[tile_base + blockIdx.x];
  const SubDev S = D.subs[wt.x];
  if (n >= S.nlev - 1) return;
  const int m = wt.y * kTile + threadIdx.x;
  if (m >= S.ncell) return;
  const int r = m / S.nx, c = m - r * S.nx;
  const int64_t plane = S.ncell;
  const T* Z = D.traj + S.traj_off + int64_t(n) * 3 * plane;
  const T* R = D.ring + S.ring_off + int64_t(n) * 3 * S.nring;
  const NbrIdx q = nbr_index(S, r, c, D.half);
  const V3<T> C = ld_box(Z, plane, m, T(1));
  const V3<T> E = ld_nbr(Z, R, plane, S.nring, q.e, 1);
  const V3<T> W = ld_nbr(Z, R, plane, S.nring, q.w, 1);
  const V3<T> N = ld_nbr(Z, R, plane, S.nring, q.n, q.sn);
  const V3<T> Sv = ld_nbr(Z, R, plane, S.nring, q.s, q.ss);
  const int j = S.row0 + r;
  const RowCoef<T> rc = D.rows[j];
  const T cN = D.cosx[j + 2], cS = D.cosx[j];
  const T st = D.st, stg = D.stg, h0 = D.h0;
  const T cor = rc.cf + rc.ct * C.u;
  const T U = -rc.a1 * C.u * (E.u - W.u) - st * C.v * (N.u - Sv.u) - rc.a2 * (E.h - W.h) + cor * C.v;
  const T V = -rc.a1 * C.u * (E.v - W.v) - st * C.v * (N.v - Sv.v) - stg * (N.h - Sv.h) - cor * C.u;
  const T H = -rc.a1 * (h0 * (E.u - W.u) + (E.h * E.u - W.h * W.u))
              - rc.a3 * (h0 * (N.v * cN - Sv.v * cS) + (N.h * N.v * cN - Sv.h * Sv.v * cS));
  T* out = const_cast<T*>(Z) + 3 * plane;
  if (n == 0) {
    out[m] = C.h + T(0.5) * H;
    out[plane + m] = C.u + T(0.5) * U;
    out[2 * plane + m] = C.v + T(0.5) * V;
  } else {
    const T* P = Z - 3 * plane;
    out[m] = P[m] + H;
    out[plane + m] = P[plane + m] + U;
    out[2 * plane + m] = P[2 * plane + m] + V;
  }
}

// mode 0: cost forcing (observations + overlap), writes grad and J at level 0
// mode 1: caller forcing (packed FP64, trajectory layout), writes adj0
// mode 2: cost forcing, writes adj0 (no background term)
template <typename T, int MODE>
__global__ __launch_bounds__(kTile) void k_adj(Dom<T> D, int n, int tile_base,
                                               const double* __restrict__ x,
                                               const double* __restrict__ xb,
                                               const double* __restrict__ forcing,
                                               double* __restrict__ out) {
  __shared__ double fo[3][kTile];
  __shared__ double red[kTile / 64];
  const int w = tile_base + blockIdx.x;
  const int2 wt = D.tiles[w];
  const SubDev S = D.subs[wt.x];
  const int L = S.nlev - 1;
  if (n > L) return;                      // uniform over the block
  const int m = wt.y * kTile + threadIdx.x;
  const bool valid = m < S.ncell;
  const int64_t plane = S.ncell;
  const T* Z = D.traj + S.traj_off + int64_t(n) * 3 * plane;
  double jloc = 0.0;

  if (MODE != 1) {
    fo[0][threadIdx.x] = 0.0;
    fo[1][threadIdx.x] = 0.0;
    fo[2][threadIdx.x] = 0.0;
    __syncthreads();
    const int64_t key = int64_t(w) * D.maxlev + n;
    const int o0 = D.obs_ptr[key], o1 = D.obs_ptr[key + 1];
    for (int o = o0 + int(threadIdx.x); o < o1; o += kTile) {
      const int code = D.obs_code[o];
      const int loc = code >> 2, f = code & 3;
      const double r = double(Z[f * plane + loc]) - D.obs_val[o];
      const double qo = D.obs_q[o];
      jloc += 0.5 * qo * r * r;
      fo[f][loc - wt.y * kTile] = qo * r;
    }
    __syncthreads();
  }

  if (valid) {
    const int r = m / S.nx, c = m - r * S.nx;
    const T* R = D.ring + S.ring_off + int64_t(n) * 3 * S.nring;
    T* A = D.adj + S.adj_off;
    const NbrIdx q = nbr_index(S, r, c, D.half);
    const V3<T> C = ld_box(Z, plane, m, T(1));
    const V3<T> E = ld_nbr(Z, R, plane, S.nring, q.e, 1);
    const V3<T> W = ld_nbr(Z, R, plane, S.nring, q.w, 1);
    const V3<T> N = ld_nbr(Z, R, plane, S.nring, q.n, q.sn);
    const V3<T> Sv = ld_nbr(Z, R, plane, S.nring, q.s, q.ss);
    const int j = S.row0 + r;
    const RowCoef<T> rc = D.rows[j];
    const T st = D.st, stg = D.stg;
    const T hm = D.h0 + C.h;

    // J_F(Z^n)^T lambda^{n+1}
    T au = 0, av = 0, ah = 0;
    if (n + 1 <= L) {
      const T* L1 = A + int64_t((n + 1) % 3) * 3 * plane;
      const T lh = L1[m], lu = L1[plane + m], lv = L1[2 * plane + m];
      // self terms
      au += lu * (-rc.a1 * (E.u - W.u) + rc.ct * C.v) + lv * (-rc.a1 * (E.v - W.v) - rc.cf - T(2) * rc.ct * C.u);
      av += lu * (-st * (N.u - Sv.u) + rc.cf + rc.ct * C.u) + lv * (-st * (N.v - Sv.v));
      // east neighbour k (m is its west neighbour)
      if (q.e >= 0) {
        const T kh = L1[q.e], ku = L1[plane + q.e], kv = L1[2 * plane + q.e];
        au += rc.a1 * (ku * E.u + kh * hm);
        av += rc.a1 * kv * E.u;
        ah += rc.a2 * ku + rc.a1 * kh * C.u;
      }
      if (q.w >= 0) {
        const T kh = L1[q.w], ku = L1[plane + q.w], kv = L1[2 * plane + q.w];
        au -= rc.a1 * (ku * W.u + kh * hm);
        av -= rc.a1 * kv * W.u;
        ah -= rc.a2 * ku + rc.a1 * kh * C.u;
      }
      if (q.n >= 0) {
        const T kh = L1[q.n], ku = L1[plane + q.n], kv = L1[2 * plane + q.n];
        const T vk = T(q.sn) * N.v;                   // raw v at k
        const T a3k = D.rows[q.sn > 0 ? j + 1 : j].a3;
        au += ku * st * vk;
        av += kv * st * vk + kh * a3k * hm * rc.c;
        ah += T(q.sn) * kv * stg + kh * a3k * C.v * rc.c;
      }
      if (q.s >= 0) {
        const T kh = L1[q.s], ku = L1[plane + q.s], kv = L1[2 * plane + q.s];
        const T vk = T(q.ss) * Sv.v;
        const T a3k = D.rows[q.ss > 0 ? j - 1 : j].a3;
        au -= ku * st * vk;
        av -= kv * st * vk + kh * a3k * hm * rc.c;
        ah -= T(q.ss) * kv * stg + kh * a3k * C.v * rc.c;
      }
      if (n == 0) {
        au = lu + T(0.5) * au;
        av = lv + T(0.5) * av;
        ah = lh + T(0.5) * ah;
      }
    }
    // forcing
    double fh, fu, fv;
    if (MODE != 1) {
      fh = fo[0][threadIdx.x];
      fu = fo[1][threadIdx.x];
      fv = fo[2][threadIdx.x];
      const int cov = D.cover[S.cell_off + m];
      const int K = cov * D.tcount[S.lev0 + n] - 1;
      if (K > 0) {
        const T* Tg = D.targ + S.traj_off + int64_t(n) * 3 * plane;
        const double eh = double(C.h) - double(Tg[m]);
        const double eu = double(C.u) - double(Tg[plane + m]);
        const double ev = double(C.v) - double(Tg[2 * plane + m]);
        const double mk = D.mu * double(K);
        fh += mk * eh * D.isb2[0];
        fu += mk * eu * D.isb2[1];
        fv += mk * ev * D.isb2[2];
        jloc += 0.5 * mk * (eh * eh * D.isb2[0] + eu * eu * D.isb2[1] + ev * ev * D.isb2[2]);
      }
    } else {
      const double* Fz = forcing + S.traj_off + int64_t(n) * 3 * plane;
      fh = Fz[m];
      fu = Fz[plane + m];
      fv = Fz[2 * plane + m];
    }
    double bh = fh + double(ah), bu = fu + double(au), bv = fv + double(av);
    if (n + 2 <= L) {
      const T* L2 = A + int64_t((n + 2) % 3) * 3 * plane;
      bh += double(L2[m]);
      bu += double(L2[plane + m]);
      bv += double(L2[2 * plane + m]);
    }
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
      out[o] = wb * dh * D.isb2[0] + bh;
      out[o + plane] = wb * du * D.isb2[1] + bu;
      out[o + 2 * plane] = wb * dv * D.isb2[2] + bv;
      jloc += 0.5 * wb * (dh * dh * D.isb2[0] + du * du * D.isb2[1] + dv * dv * D.isb2[2]);
    } else {
      const int64_t o = S.ctrl_off + m;
      out[o] = bh;
      out[o + plane] = bu;
      out[o + 2 * plane] = bv;
    }
  }
  if (MODE != 1) {
    const double tot = block_sum(jloc, red);
    if (threadIdx.x == 0) D.jpart[w] = (n == L) ? tot : D.jpart[w] + tot;
  }
}

// J[s] = sum of tile partials (fixed order) + constant overlap part
__global__ void k_reduce_j(const SubDev* __restrict__ subs, int count, const int32_t* __restrict__ ids,
                           const double* __restrict__ jpart, const double* __restrict__ jconst,
                           double* __restrict__ J, uint32_t* __restrict__ nonfinite) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int s = ids ? ids[i] : i;
  const SubDev S = subs[s];
  double acc = 0.0;
  for (int t = 0; t < S.ntile; ++t) acc += jpart[S.tile0 + t];
  acc += jconst[s];
  J[s] = acc;
  if (!isfinite(acc)) atomicOr(nonfinite, 1u);
}

// packed FP64 trajectory output (h + h_ref)
template <typename T>
__global__ __launch_bounds__(kTile) void k_traj_out(Dom<T> D, double* __restrict__ out, int tile_base) {
  const int2 wt = D.tiles[tile_base + blockIdx.x];
  const SubDev S = D.subs[wt.x];
  const int m = wt.y * kTile + threadIdx.x;
  if (m >= S.ncell) return;
  const int64_t plane = S.ncell;
  for (int n = 0; n < S.nlev; ++n) {
    const T* Z = D.traj + S.traj_off + int64_t(n) * 3 * plane;
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
  else
    hipLaunchKernelGGL((k_adj<T, 2>), dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base, x, xb,
                       forcing, out);
}
void launch_reduce_j(const SubDev* subs, int count, const int32_t* ids, const double* jpart,
                     const double* jconst, double* J, uint32_t* nonfinite, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_j, dim3((count + 255) / 256), dim3(256), 0, st, subs, count, ids,
                     jpart, jconst, J, nonfinite);
}
template <typename T>
void launch_traj_out(const Dom<T>& D, double* out, int tile_base, int ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_traj_out<T>, dim3(ntiles), dim3(kTile), 0, st, D, out, tile_base);
}

#define DD4DVAR_INST(T)                                                                        \
  template void launch_init<T>(const Dom<T>&, const double*, int, int, hipStream_t);          \
  template void launch_fwd<T>(const Dom<T>&, int, int, int, hipStream_t);                      \
  template void launch_adj<T>(const Dom<T>&, int, int, int, int, const double*, const double*, \
                              const double*, double*, hipStream_t);                            \
  template void launch_traj_out<T>(const Dom<T>&, double*, int, int, hipStream_t);
DD4DVAR_INST(float)
DD4DVAR_INST(double)
#undef DD4DVAR_INST

}  // namespace dd4dvar
