// Turkel-Zwas variant of the local sweeps (Sec. 7 discrete U, V, H with
// coarse offsets p, q and averaging alpha), for boxes that cover the whole
// sphere (time decompositions): step kernels over every box, one workgroup
// per 256-cell tile.
//
// The scheme reads 13 points: the cell, its four neighbours, (i +- p, j),
// (i, j +- q) and the corners (i +- p, j +- q).  Rows beyond a pole are the
// rows on the other side of it (same latitude, half a circle further, u and v
// negated, that row's coefficients).  Readings: H with leading -sigma, the
// latitude divergence with h / cos, advective form; the alpha-averaged
// Coriolis terms take u, v, f, tan at the neighbour; 2 dt on the Coriolis
// bracket; v differences for the meridional advection of v.
//
// Adjoint, deterministic and without atomics: for every cell k a first
// kernel writes the transposed contribution of its increment to each of the
// 13 points it reads (the partial derivatives of the increment at k with
// respect to the state there, applied to lambda^{n+1}(k)) into one slot
// plane per offset; for a given offset the map from k to the point read is
// one-to-one, except that a row within q of a pole is reached both directly
// and across the pole, so contributions that cross a pole go to separate
// planes.  A second kernel sums, for every cell, the planes that some cell's
// offset reaches there, in a fixed order, and adds the forcing and
// lambda^{n+2} (gather form of the same transpose).
#include "kernels.h"
#include "launch.h"
#include "stencil.h"

#ifndef DD4DVAR_TZ_T
#error "compile with -DDD4DVAR_TZ_T=float or double"
#endif

namespace dd4dvar {

using namespace stencil;

namespace {
// offsets: the cell, E1, W1, N1, S1, Ep, Wp, Nq, Sq, EpNq, WpNq, EpSq, WpSq;
// planes 13.. hold the across-pole contributions of N1, S1, Nq, Sq and the
// four corners
constexpr int kOffs = 13;
constexpr int kPlanes = tz_slot_planes();

struct Pt {
  int idx;   // cell of the box
  int sg;    // +1, or -1 across a pole (u, v)
  int row;   // its row (coefficients)
  bool across;
};

// point (r + dr, c + dc) of a box covering the sphere
__device__ __forceinline__ Pt point(const SubDev& S, int r, int c, int dr, int dc, int half) {
  int rr = r + dr, cc = c + dc, sg = 1;
  bool across = false;
  if (rr >= S.ny) {
    rr = 2 * S.ny - 1 - rr;
    cc += half;
    sg = -1;
    across = true;
  } else if (rr < 0) {
    rr = -1 - rr;
    cc += half;
    sg = -1;
    across = true;
  }
  cc %= S.nx;
  if (cc < 0) cc += S.nx;
  return {rr * S.nx + cc, sg, rr, across};
}

template <typename T>
__device__ __forceinline__ V3<T> ld_pt(const T* Z, int64_t plane, const Pt& p) {
  const T s = T(p.sg);
  return {Z[p.idx], s * Z[plane + p.idx], s * Z[2 * plane + p.idx]};
}

// the 13 points of cell (r, c): offsets in the order of the slot planes
__device__ __forceinline__ void points(const SubDev& S, int r, int c, int p, int q, int half,
                                       Pt* P) {
  P[0] = point(S, r, c, 0, 0, half);
  P[1] = point(S, r, c, 0, 1, half);
  P[2] = point(S, r, c, 0, -1, half);
  P[3] = point(S, r, c, 1, 0, half);
  P[4] = point(S, r, c, -1, 0, half);
  P[5] = point(S, r, c, 0, p, half);
  P[6] = point(S, r, c, 0, -p, half);
  P[7] = point(S, r, c, q, 0, half);
  P[8] = point(S, r, c, -q, 0, half);
  P[9] = point(S, r, c, q, p, half);
  P[10] = point(S, r, c, q, -p, half);
  P[11] = point(S, r, c, -q, p, half);
  P[12] = point(S, r, c, -q, -p, half);
}

// across-pole plane of offset o (o = 3, 4, 7 .. 12), else -1
__device__ __forceinline__ int across_plane(int o) {
  if (o == 3 || o == 4) return 13 + (o - 3);
  if (o >= 7) return 15 + (o - 7);
  return -1;
}

template <typename T>
struct State13 {
  V3<T> C, E, W, N, Sv, Ep, Wp, Nq, Sq, EN, WN, ES, WS;
};

template <typename T>
__device__ __forceinline__ State13<T> load13(const T* Z, int64_t plane, const Pt* P) {
  State13<T> s;
  s.C = ld_pt(Z, plane, P[0]);
  s.E = ld_pt(Z, plane, P[1]);
  s.W = ld_pt(Z, plane, P[2]);
  s.N = ld_pt(Z, plane, P[3]);
  s.Sv = ld_pt(Z, plane, P[4]);
  s.Ep = ld_pt(Z, plane, P[5]);
  s.Wp = ld_pt(Z, plane, P[6]);
  s.Nq = ld_pt(Z, plane, P[7]);
  s.Sq = ld_pt(Z, plane, P[8]);
  s.EN = ld_pt(Z, plane, P[9]);
  s.WN = ld_pt(Z, plane, P[10]);
  s.ES = ld_pt(Z, plane, P[11]);
  s.WS = ld_pt(Z, plane, P[12]);
  return s;
}
}  // namespace

// Z^{n+1} = Z^{n-1} + F(Z^n) (Z^1 = Z^0 + F(Z^0)/2) with the Turkel-Zwas F
template <typename T>
__global__ __launch_bounds__(kTile) void k_fwd_tz(Dom<T> D, int n, int tile_base, int p, int q,
                                                  T alpha) {
  const int2 wt = D.tiles[tile_base + xcd_tile(blockIdx.x, gridDim.x)];
  if (D.active && !D.active[wt.x]) return;
  const SubDev S = D.subs[wt.x];
  if (n >= S.nlev - 1) return;
  const int m = wt.y * kTile + threadIdx.x;
  if (m >= S.ncell) return;
  const int r = m / S.nx, c = m - r * S.nx;
  const int64_t plane = S.ncell;
  const T* Z = zlevel(D, S, n);
  const T* B0 = n >= 1 ? zlevel(D, S, n - 1) : Z;
  Pt P[kOffs];
  points(S, r, c, p, q, D.half, P);
  const State13<T> z = load13(Z, plane, P);
  const V3<T> B = ld_box(B0, plane, m, T(1));
  const RowCoef<T> rc = D.rows[S.row0 + r];
  const RowCoef<T> rN = D.rows[S.row0 + P[7].row], rS = D.rows[S.row0 + P[8].row];
  const T st = D.st, stg = D.stg, h0 = D.h0, al = alpha, one = T(1), half = T(0.5);
  const T tp = T(p), tq = T(q);
  const V3<T>& C = z.C;
  const T hh = h0 + C.h;
  const T U = -rc.a1 * C.u * (z.E.u - z.W.u) - st * C.v * (z.N.u - z.Sv.u) -
              rc.a2 / tp * (z.Ep.h - z.Wp.h) +
              ((one - al) * (rc.cf + rc.ct * C.u) * C.v + half * al * (rc.cf + rc.ct * z.Ep.u) * z.Ep.v +
               half * al * (rc.cf + rc.ct * z.Wp.u) * z.Wp.v);
  const T V = -rc.a1 * C.u * (z.E.v - z.W.v) - st * C.v * (z.N.v - z.Sv.v) -
              stg / tq * (z.Nq.h - z.Sq.h) -
              ((one - al) * (rc.cf + rc.ct * C.u) * C.u + half * al * (rN.cf + rN.ct * z.Nq.u) * z.Nq.u +
               half * al * (rS.cf + rS.ct * z.Sq.u) * z.Sq.u);
  const T Dl = ((one - al) * (z.Ep.u - z.Wp.u) + half * al * (z.EN.u - z.WN.u + z.ES.u - z.WS.u)) / tp;
  const T Dt = ((one - al) * (z.Nq.v * rN.c - z.Sq.v * rS.c) + half * al * (z.EN.v * rN.c - z.ES.v * rS.c) +
                half * al * (z.WN.v * rN.c - z.WS.v * rS.c)) / tq;
  const T H = -rc.a1 * (C.u * (z.E.h - z.W.h) + hh * Dl) - (st * C.v * (z.N.h - z.Sv.h) + rc.a3 * hh * Dt);
  const T wgt = n == 0 ? T(0.5) : T(1);
  T* out = zlevel(D, S, n + 1);
  out[m] = B.h + wgt * H;
  out[plane + m] = B.u + wgt * U;
  out[2 * plane + m] = B.v + wgt * V;
}

// first adjoint kernel: the transposed contributions of cell k's increment
// at level n applied to lambda^{n+1}(k), one slot plane per offset
template <typename T>
__global__ __launch_bounds__(kTile) void k_adj_tz_scatter(Dom<T> D, int n, int tile_base, int p,
                                                          int q, T alpha, T* __restrict__ slots) {
  const int2 wt = D.tiles[tile_base + xcd_tile(blockIdx.x, gridDim.x)];
  if (D.active && !D.active[wt.x]) return;
  const SubDev S = D.subs[wt.x];
  if (n + 1 > S.nlev - 1) return;
  const int m = wt.y * kTile + threadIdx.x;
  if (m >= S.ncell) return;
  const int r = m / S.nx, c = m - r * S.nx;
  const int64_t plane = S.ncell;
  const T* Z = zlevel(D, S, n);
  const T* L1 = D.adj + S.adj_off + int64_t((n + 1) % 3) * 3 * plane;
  Pt P[kOffs];
  points(S, r, c, p, q, D.half, P);
  const State13<T> z = load13(Z, plane, P);
  const V3<T> lam = ld_box(L1, plane, m, T(1));
  const RowCoef<T> rc = D.rows[S.row0 + r];
  const RowCoef<T> rN = D.rows[S.row0 + P[7].row], rS = D.rows[S.row0 + P[8].row];
  const T st = D.st, stg = D.stg, h0 = D.h0, al = alpha, one = T(1), half = T(0.5);
  const T tp = T(p), tq = T(q);
  const V3<T>& C = z.C;
  const T hh = h0 + C.h;
  const T lH = lam.h, lU = lam.u, lV = lam.v;
  const T Dl = ((one - al) * (z.Ep.u - z.Wp.u) + half * al * (z.EN.u - z.WN.u + z.ES.u - z.WS.u)) / tp;
  const T Dt = ((one - al) * (z.Nq.v * rN.c - z.Sq.v * rS.c) + half * al * (z.EN.v * rN.c - z.ES.v * rS.c) +
                half * al * (z.WN.v * rN.c - z.WS.v * rS.c)) / tq;
  const T a1u = rc.a1 * C.u, stv = st * C.v;
  const T dn = half * al * rc.a1 * hh / tp;          // corner weight of u in H
  const T cqN = rc.a3 * hh * rN.c / tq, cqS = rc.a3 * hh * rS.c / tq;
  V3<T> g[kOffs];
  // the cell itself
  g[0].h = -lH * (rc.a1 * Dl + rc.a3 * Dt);
  g[0].u = lU * (-rc.a1 * (z.E.u - z.W.u) + (one - al) * rc.ct * C.v) +
           lV * (-rc.a1 * (z.E.v - z.W.v) - (one - al) * (rc.cf + T(2) * rc.ct * C.u)) -
           lH * rc.a1 * (z.E.h - z.W.h);
  g[0].v = lU * (-st * (z.N.u - z.Sv.u) + (one - al) * (rc.cf + rc.ct * C.u)) - lV * st * (z.N.v - z.Sv.v) -
           lH * st * (z.N.h - z.Sv.h);
  // advection neighbours (offset one)
  g[1] = {-lH * a1u, -lU * a1u, -lV * a1u};
  g[2] = {lH * a1u, lU * a1u, lV * a1u};
  g[3] = {-lH * stv, -lU * stv, -lV * stv};
  g[4] = {lH * stv, lU * stv, lV * stv};
  // (i +- p, j): pressure gradient and averaged Coriolis of U, divergence of H
  g[5] = {-lU * rc.a2 / tp, lU * half * al * rc.ct * z.Ep.v - lH * (one - al) * rc.a1 * hh / tp,
          lU * half * al * (rc.cf + rc.ct * z.Ep.u)};
  g[6] = {lU * rc.a2 / tp, lU * half * al * rc.ct * z.Wp.v + lH * (one - al) * rc.a1 * hh / tp,
          lU * half * al * (rc.cf + rc.ct * z.Wp.u)};
  // (i, j +- q): pressure gradient and averaged Coriolis of V, divergence of H
  g[7] = {-lV * stg / tq, -lV * half * al * (rN.cf + T(2) * rN.ct * z.Nq.u), -lH * (one - al) * cqN};
  g[8] = {lV * stg / tq, -lV * half * al * (rS.cf + T(2) * rS.ct * z.Sq.u), lH * (one - al) * cqS};
  // corners: the averaged divergence of H
  g[9] = {T(0), -lH * dn, -lH * half * al * cqN};
  g[10] = {T(0), lH * dn, -lH * half * al * cqN};
  g[11] = {T(0), -lH * dn, lH * half * al * cqS};
  g[12] = {T(0), lH * dn, lH * half * al * cqS};
  T* base = slots + S.ctrl_off * kPlanes;
#pragma unroll
  for (int o = 0; o < kOffs; ++o) {
    const int pl = P[o].across ? across_plane(o) : o;
    const T sg = T(P[o].sg);
    T* sp = base + int64_t(pl) * 3 * plane;
    sp[P[o].idx] = g[o].h;
    sp[plane + P[o].idx] = sg * g[o].u;
    sp[2 * plane + P[o].idx] = sg * g[o].v;
  }
}

// second adjoint kernel: lambda^n (or the gradient) at every cell from the
// slot planes that reach it, the forcing and lambda^{n+2}
template <typename T, int MODE>
__global__ __launch_bounds__(kTile) void k_adj_tz_gather(Dom<T> D, int n, int tile_base, int q,
                                                         const T* __restrict__ slots,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ xb,
                                                         const double* __restrict__ forcing,
                                                         double* __restrict__ out) {
  __shared__ double fo[3][kTile];
  __shared__ double red[kTile / 64];
  const int w = tile_base + xcd_tile(blockIdx.x, gridDim.x);
  const int2 wt = D.tiles[w];
  if (D.active && !D.active[wt.x]) return;
  const SubDev S = D.subs[wt.x];
  const int L = S.nlev - 1;
  if (n > L) return;
  const int m = wt.y * kTile + threadIdx.x;
  const bool valid = m < S.ncell;
  const int mm = valid ? m : 0;
  const int64_t plane = S.ncell;
  const T* Z = zlevel(D, S, n);
  T* A = D.adj + S.adj_off;
  const bool has1 = n + 1 <= L, has2 = n + 2 <= L;
  const T* L1 = A + int64_t((n + 1) % 3) * 3 * plane;
  const T* L2 = A + int64_t((n + 2) % 3) * 3 * plane;
  const int r = mm / S.nx, ny = S.ny;
  double jloc = 0.0;
  // J_F(Z^n)^T lambda^{n+1}: the planes whose offset reaches this row
  double ah = 0, au = 0, av = 0;
  if (has1) {
    const T* base = slots + S.ctrl_off * kPlanes;
    // rows reached directly by an offset of +k rows: r >= k; of -k: r + k < ny;
    // across a pole by +k: r >= ny - k; by -k: r < k
    const bool dir[kOffs] = {true, true, true, r >= 1, r + 1 < ny, true, true, r >= q, r + q < ny,
                             r >= q, r >= q, r + q < ny, r + q < ny};
    const bool acr[8] = {r >= ny - 1, r < 1, r >= ny - q, r < q, r >= ny - q, r >= ny - q, r < q, r < q};
#pragma unroll
    for (int o = 0; o < kOffs; ++o) {
      if (!dir[o]) continue;
      const T* sp = base + int64_t(o) * 3 * plane;
      ah += double(sp[mm]);
      au += double(sp[plane + mm]);
      av += double(sp[2 * plane + mm]);
    }
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      if (!acr[o]) continue;
      const T* sp = base + int64_t(13 + o) * 3 * plane;
      ah += double(sp[mm]);
      au += double(sp[plane + mm]);
      av += double(sp[2 * plane + mm]);
    }
  }
  V3<T> l0 = {T(0), T(0), T(0)}, l2 = {T(0), T(0), T(0)};
  if (has1) l0 = ld_box(L1, plane, mm, T(1));
  if (has2) l2 = ld_box(L2, plane, mm, T(1));
  double fh = 0, fu = 0, fv = 0;
  int K = 0;
  if (MODE != 1) K = int(D.cover[S.cell_off + mm]) * D.tcount[S.lev0 + n] - 1;
  if (MODE == 1) {
    const double* Fz = forcing + S.traj_off + int64_t(n) * 3 * plane;
    fh = Fz[mm];
    fu = Fz[plane + mm];
    fv = Fz[2 * plane + mm];
  } else {
    const int64_t key = int64_t(w) * D.maxlev + n;
    const int o0 = D.obs_ptr[key], o1 = D.obs_ptr[key + 1];
    if (o1 > o0) {
      fo[0][threadIdx.x] = 0.0;
      fo[1][threadIdx.x] = 0.0;
      fo[2][threadIdx.x] = 0.0;
      __syncthreads();
      for (int o = o0 + int(threadIdx.x); o < o1; o += kTile) {
        const int code = D.obs_code[o];
        const int loc = code >> 2, f = code & 3;
        const double rr = double(Z[f * plane + loc]) - D.obs_val[o];
        const double qo = D.obs_q[o];
        jloc += 0.5 * qo * rr * rr;
        fo[f][loc - wt.y * kTile] = qo * rr;
      }
      __syncthreads();
      fh = fo[0][threadIdx.x];
      fu = fo[1][threadIdx.x];
      fv = fo[2][threadIdx.x];
    }
  }
  if (valid) {
    if (n == 0) {
      ah = double(l0.h) + 0.5 * ah;
      au = double(l0.u) + 0.5 * au;
      av = double(l0.v) + 0.5 * av;
    }
    if (MODE != 1) {
      const V3<T> C = ld_box(Z, plane, m, T(1));
      const V3<T> tg = ld_box(D.targ + S.traj_off + int64_t(n) * 3 * plane, plane, K > 0 ? m : 0, T(1));
      const double eh = double(C.h) - double(tg.h);
      const double eu = double(C.u) - double(tg.u);
      const double ev = double(C.v) - double(tg.v);
      const double mk = D.mu * double(K);
      fh += mk * eh * D.isb2[0];
      fu += mk * eu * D.isb2[1];
      fv += mk * ev * D.isb2[2];
      jloc += 0.5 * mk * (eh * eh * D.isb2[0] + eu * eu * D.isb2[1] + ev * ev * D.isb2[2]);
    }
    const double bh = fh + ah + double(l2.h);
    const double bu = fu + au + double(l2.u);
    const double bv = fv + av + double(l2.v);
    if (n > 0) {
      T* Bn = A + int64_t(n % 3) * 3 * plane;
      Bn[m] = T(bh);
      Bn[plane + m] = T(bu);
      Bn[2 * plane + m] = T(bv);
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
  if (MODE == 0 || MODE == 2) {
    const double tot = block_sum(jloc, red);
    if (threadIdx.x == 0) D.jpart[w] = (n == L) ? tot : D.jpart[w] + tot;
  }
}

template <typename T>
void launch_fwd_tz(const Dom<T>& D, int n, int tile_base, int ntiles, int p, int q, double alpha,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_fwd_tz<T>, dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base, p, q, T(alpha));
}
template <typename T>
void launch_adj_tz(const Dom<T>& D, int n, int tile_base, int ntiles, int mode, int p, int q,
                   double alpha, T* slots, const double* x, const double* xb,
                   const double* forcing, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_tz_scatter<T>, dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base, p, q,
                     T(alpha), slots);
  if (mode == 0)
    hipLaunchKernelGGL((k_adj_tz_gather<T, 0>), dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base, q,
                       slots, x, xb, forcing, out);
  else if (mode == 1)
    hipLaunchKernelGGL((k_adj_tz_gather<T, 1>), dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base, q,
                       slots, x, xb, forcing, out);
  else
    hipLaunchKernelGGL((k_adj_tz_gather<T, 2>), dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base, q,
                       slots, x, xb, forcing, out);
}

#define DD4DVAR_INST(T)                                                                         \
  template void launch_fwd_tz<T>(const Dom<T>&, int, int, int, int, int, double, hipStream_t); \
  template void launch_adj_tz<T>(const Dom<T>&, int, int, int, int, int, int, double, T*,      \
                                 const double*, const double*, const double*, double*,         \
                                 hipStream_t);
DD4DVAR_INST(DD4DVAR_TZ_T)
#undef DD4DVAR_INST

}  // namespace dd4dvar
