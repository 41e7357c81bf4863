// Turkel-Zwas variant of the local sweeps (Sec. 7 discrete U, V, H with
// coarse offsets p, q and averaging alpha): step kernels over every box, one
// workgroup per 256-cell tile.
//
// The scheme reads 13 points: the cell, its four neighbours, (i +- p, j),
// (i, j +- q) and the corners (i +- p, j +- q).  Rows beyond a pole are the
// rows on the other side of it (same latitude, half a circle further, u and v
// negated, that row's coefficients).  Readings: H with leading -sigma, the
// latitude divergence with h / cos, advective form; the alpha-averaged
// Coriolis terms take u, v, f, tan at the neighbour; 2 dt on the Coriolis
// bracket; v differences for the meridional advection of v.
//
// Points outside the box (restricted model, eq. restricted) come from the
// box's frozen pad, q rows and p columns wide with corners, whose values the
// exchange writes with their signs applied: for a box of several pieces every
// position of the frame [-q, ny+q) x [-p, nx+p) outside the box, numbered
// south block, north block (row-major over columns -p..nx+p-1), west block,
// east block (row-major); for a box spanning the circle, whose columns wrap
// onto itself, the south and north blocks over columns 0..nx-1, and a point
// beyond a pole that maps into the box itself is read there (u, v negated).
//
// Adjoint (adjoint definition of Sec. 2, eq. adjProd), gather form, one
// launch per level: every cell x sums the transposed contributions of the
// in-box cells k whose increment reads it, the partial derivative of the
// increment at k with respect to the state at x applied to lambda^{n+1}(k),
// evaluated from k's state, lambda and row coefficients: the cell itself
// (its whole 13-point neighbourhood), the readers k = x - offset of the other
// 12 offsets, and in a box spanning the circle the readers whose offset
// reaches x across a pole (u, v components negated).  Frozen pad values get
// nothing.  The sum runs in a fixed order (deterministic, no atomics).
#include "kernels.h"
#include "launch.h"
#include "stencil.h"

#ifndef DD4DVAR_TZ_T
#error "compile with -DDD4DVAR_TZ_T=float or double"
#endif

namespace dd4dvar {

using namespace stencil;

namespace {
// offsets: the cell, E1, W1, N1, S1, Ep, Wp, Nq, Sq, EpNq, WpNq, EpSq, WpSq
constexpr int kOffs = 13;

struct Pt {
  int idx;      // cell of the box, or position in the frozen pad
  int sg;       // -1 for an in-box point reached across a pole (u, v)
  int grow;     // global row whose coefficients apply
  bool pad;     // frozen pad value (signs already applied)
  bool across;  // in-box point reached across a pole
};

// row offset and column offset of each of the 13 points
__device__ __forceinline__ int off_r(int o, int q) {
  return o == 3 ? 1 : o == 4 ? -1 : (o == 7 || o == 9 || o == 10) ? q : (o == 8 || o == 11 || o == 12) ? -q : 0;
}
__device__ __forceinline__ int off_c(int o, int p) {
  return o == 1 ? 1 : o == 2 ? -1 : (o == 5 || o == 9 || o == 11) ? p : (o == 6 || o == 10 || o == 12) ? -p : 0;
}

// point (r + dr, c + dc) of box cell (r, c)
__device__ __forceinline__ Pt point(const SubDev& S, int r, int c, int dr, int dc, int p, int q,
                                    int half, int nlat) {
  const int rr = r + dr;
  int cc = c + dc;
  const int g = S.row0 + rr;
  const bool cross = g < 0 || g >= nlat;
  Pt P;
  P.grow = g < 0 ? -1 - g : (g >= nlat ? 2 * nlat - 1 - g : g);
  P.sg = 1;
  P.pad = false;
  P.across = false;
  if (S.span) {
    cc = cc < 0 ? cc + S.nx : (cc >= S.nx ? cc - S.nx : cc);
    if (rr >= 0 && rr < S.ny) {
      P.idx = rr * S.nx + cc;
    } else if (cross && P.grow >= S.row0 && P.grow < S.row0 + S.ny) {
      int ca = cc + half;
      ca = ca >= S.nx ? ca - S.nx : ca;
      P.idx = (P.grow - S.row0) * S.nx + ca;
      P.sg = -1;
      P.across = true;
    } else {
      P.pad = true;
      P.idx = (rr < 0 ? rr + q : q + rr - S.ny) * S.nx + cc;
    }
    return P;
  }
  if (rr >= 0 && rr < S.ny && cc >= 0 && cc < S.nx) {
    P.idx = rr * S.nx + cc;
    return P;
  }
  P.pad = true;
  const int w = S.nx + 2 * p;
  if (rr < 0)
    P.idx = (rr + q) * w + cc + p;
  else if (rr >= S.ny)
    P.idx = (q + rr - S.ny) * w + cc + p;
  else if (cc < 0)
    P.idx = 2 * q * w + rr * p + cc + p;
  else
    P.idx = 2 * q * w + S.ny * p + rr * p + cc - S.nx;
  return P;
}

// value at a point: the box state (sign across a pole) or the frozen pad
template <typename T>
__device__ __forceinline__ V3<T> ld_pt(const T* Z, const T* R, int64_t plane, int nring, const Pt& P) {
  const T* base = P.pad ? R : Z;
  const int64_t st = P.pad ? int64_t(nring) : plane;
  const T s = T(P.sg);
  return {base[P.idx], s * base[st + P.idx], s * base[2 * st + P.idx]};
}

// the 13 points of cell (r, c): plain index arithmetic for cells whose
// neighbourhood lies inside the box (nearly all), the general mapping else
__device__ __forceinline__ void points(const SubDev& S, int r, int c, int p, int q, int half,
                                       int nlat, Pt* P) {
  const bool inner = r >= q && r + q < S.ny && c >= p && c + p < S.nx;
  if (inner) {
    const int m = r * S.nx + c;
#pragma unroll
    for (int o = 0; o < kOffs; ++o) {
      P[o].idx = m + off_r(o, q) * S.nx + off_c(o, p);
      P[o].sg = 1;
      P[o].grow = S.row0 + r + off_r(o, q);
      P[o].pad = false;
      P[o].across = false;
    }
    return;
  }
#pragma unroll
  for (int o = 0; o < kOffs; ++o) P[o] = point(S, r, c, off_r(o, q), off_c(o, p), p, q, half, nlat);
}

// perturbation at a point: the box value (sign across a pole), zero on a
// frozen pad position (the pad does not depend on the control)
template <typename T>
__device__ __forceinline__ V3<T> ld_dpt(const T* dZ, int64_t plane, int m, const Pt& P) {
  const int i = P.pad ? m : P.idx;
  const T s = T(P.sg);
  const T h = dZ[i], u = dZ[plane + i], v = dZ[2 * plane + i];
  return {P.pad ? T(0) : h, P.pad ? T(0) : s * u, P.pad ? T(0) : s * v};
}

template <typename T>
struct State13 {
  V3<T> C, E, W, N, Sv, Ep, Wp, Nq, Sq, EN, WN, ES, WS;
};

template <typename T>
__device__ __forceinline__ State13<T> load13(const T* Z, const T* R, int64_t plane, int nring,
                                             const Pt* P) {
  State13<T> s;
  s.C = ld_pt(Z, R, plane, nring, P[0]);
  s.E = ld_pt(Z, R, plane, nring, P[1]);
  s.W = ld_pt(Z, R, plane, nring, P[2]);
  s.N = ld_pt(Z, R, plane, nring, P[3]);
  s.Sv = ld_pt(Z, R, plane, nring, P[4]);
  s.Ep = ld_pt(Z, R, plane, nring, P[5]);
  s.Wp = ld_pt(Z, R, plane, nring, P[6]);
  s.Nq = ld_pt(Z, R, plane, nring, P[7]);
  s.Sq = ld_pt(Z, R, plane, nring, P[8]);
  s.EN = ld_pt(Z, R, plane, nring, P[9]);
  s.WN = ld_pt(Z, R, plane, nring, P[10]);
  s.ES = ld_pt(Z, R, plane, nring, P[11]);
  s.WS = ld_pt(Z, R, plane, nring, P[12]);
  return s;
}
}  // namespace

// Z^{n+1} = Z^{n-1} + F(Z^n) (Z^1 = Z^0 + F(Z^0)/2) with the Turkel-Zwas F
template <typename T>
__global__ __launch_bounds__(kTile) void k_fwd_tz(Dom<T> D, int n, int tile_base, int p, int q,
                                                  T alpha, int nlat) {
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
  const T* R = D.ring + S.ring_off + int64_t(n) * 3 * S.nring;
  Pt P[kOffs];
  points(S, r, c, p, q, D.half, nlat, P);
  const State13<T> z = load13(Z, R, plane, S.nring, P);
  const V3<T> B = ld_box(B0, plane, m, T(1));
  const RowCoef<T> rc = D.rows[S.row0 + r];
  const RowCoef<T> rN = D.rows[P[7].grow], rS = D.rows[P[8].grow];
  const T st = D.st, stg = D.stg, h0 = D.h0, al = alpha, one = T(1), half = T(0.5);
  // 1/p, 1/q: multiplying by them equals dividing when p, q are powers of two
  const T itp = one / T(p), itq = one / T(q);
  const V3<T>& C = z.C;
  const T hh = h0 + C.h;
  const T U = -rc.a1 * C.u * (z.E.u - z.W.u) - st * C.v * (z.N.u - z.Sv.u) -
              rc.a2 * itp * (z.Ep.h - z.Wp.h) +
              ((one - al) * (rc.cf + rc.ct * C.u) * C.v + half * al * (rc.cf + rc.ct * z.Ep.u) * z.Ep.v +
               half * al * (rc.cf + rc.ct * z.Wp.u) * z.Wp.v);
  const T V = -rc.a1 * C.u * (z.E.v - z.W.v) - st * C.v * (z.N.v - z.Sv.v) -
              stg * itq * (z.Nq.h - z.Sq.h) -
              ((one - al) * (rc.cf + rc.ct * C.u) * C.u + half * al * (rN.cf + rN.ct * z.Nq.u) * z.Nq.u +
               half * al * (rS.cf + rS.ct * z.Sq.u) * z.Sq.u);
  const T Dl = ((one - al) * (z.Ep.u - z.Wp.u) + half * al * (z.EN.u - z.WN.u + z.ES.u - z.WS.u)) * itp;
  const T Dt = ((one - al) * (z.Nq.v * rN.c - z.Sq.v * rS.c) + half * al * (z.EN.v * rN.c - z.ES.v * rS.c) +
                half * al * (z.WN.v * rN.c - z.WS.v * rS.c)) * itq;
  const T H = -rc.a1 * (C.u * (z.E.h - z.W.h) + hh * Dl) - (st * C.v * (z.N.h - z.Sv.h) + rc.a3 * hh * Dt);
  const T wgt = n == 0 ? T(0.5) : T(1);
  T* out = zlevel(D, S, n + 1);
  out[m] = B.h + wgt * H;
  out[plane + m] = B.u + wgt * U;
  out[2 * plane + m] = B.v + wgt * V;
}

// tangent linear (the TLM step of Alg. 6):
// dZ^{n+1} = dZ^{n-1} + F'(Z^n) dZ^n (dZ^1 = dZ^0 + F'(Z^0) dZ^0 / 2)
template <typename T>
__global__ __launch_bounds__(kTile) void k_tlm_tz(Dom<T> D, int n, int tile_base, int p, int q,
                                                  T alpha, int nlat) {
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
  const T* dZ = D.dz + S.zoff + int64_t(n) * 3 * plane;
  const T* dB = n >= 1 ? D.dz + S.zoff + int64_t(n - 1) * 3 * plane : dZ;
  Pt P[kOffs];
  points(S, r, c, p, q, D.half, nlat, P);
  const State13<T> z = load13(Z, R, plane, S.nring, P);
  V3<T> d[kOffs];
#pragma unroll
  for (int o = 0; o < kOffs; ++o) d[o] = ld_dpt(dZ, plane, m, P[o]);
  const V3<T> B = ld_box(dB, plane, m, T(1));
  const RowCoef<T> rc = D.rows[S.row0 + r];
  const RowCoef<T> rN = D.rows[P[7].grow], rS = D.rows[P[8].grow];
  const T st = D.st, stg = D.stg, h0 = D.h0, al = alpha, one = T(1), half = T(0.5);
  // 1/p, 1/q: multiplying by them equals dividing when p, q are powers of two
  const T itp = one / T(p), itq = one / T(q);
  const V3<T>& C = z.C;
  const V3<T>& dC = d[0];
  const T hh = h0 + C.h;
  const T dU = -rc.a1 * (dC.u * (z.E.u - z.W.u) + C.u * (d[1].u - d[2].u)) -
               st * (dC.v * (z.N.u - z.Sv.u) + C.v * (d[3].u - d[4].u)) - rc.a2 * itp * (d[5].h - d[6].h) +
               ((one - al) * (rc.ct * dC.u * C.v + (rc.cf + rc.ct * C.u) * dC.v) +
                half * al * (rc.ct * d[5].u * z.Ep.v + (rc.cf + rc.ct * z.Ep.u) * d[5].v) +
                half * al * (rc.ct * d[6].u * z.Wp.v + (rc.cf + rc.ct * z.Wp.u) * d[6].v));
  const T dV = -rc.a1 * (dC.u * (z.E.v - z.W.v) + C.u * (d[1].v - d[2].v)) -
               st * (dC.v * (z.N.v - z.Sv.v) + C.v * (d[3].v - d[4].v)) - stg * itq * (d[7].h - d[8].h) -
               ((one - al) * (rc.cf + T(2) * rc.ct * C.u) * dC.u +
                half * al * (rN.cf + T(2) * rN.ct * z.Nq.u) * d[7].u +
                half * al * (rS.cf + T(2) * rS.ct * z.Sq.u) * d[8].u);
  const T Dl = ((one - al) * (z.Ep.u - z.Wp.u) + half * al * (z.EN.u - z.WN.u + z.ES.u - z.WS.u)) * itp;
  const T Dt = ((one - al) * (z.Nq.v * rN.c - z.Sq.v * rS.c) + half * al * (z.EN.v * rN.c - z.ES.v * rS.c) +
                half * al * (z.WN.v * rN.c - z.WS.v * rS.c)) * itq;
  const T dDl = ((one - al) * (d[5].u - d[6].u) + half * al * (d[9].u - d[10].u + d[11].u - d[12].u)) * itp;
  const T dDt = ((one - al) * (d[7].v * rN.c - d[8].v * rS.c) + half * al * (d[9].v * rN.c - d[11].v * rS.c) +
                 half * al * (d[10].v * rN.c - d[12].v * rS.c)) * itq;
  const T dH = -rc.a1 * (dC.u * (z.E.h - z.W.h) + C.u * (d[1].h - d[2].h) + dC.h * Dl + hh * dDl) -
               (st * (dC.v * (z.N.h - z.Sv.h) + C.v * (d[3].h - d[4].h)) + rc.a3 * (dC.h * Dt + hh * dDt));
  const T wgt = n == 0 ? T(0.5) : T(1);
  T* out = D.dz + S.zoff + int64_t(n + 1) * 3 * plane;
  out[m] = B.h + wgt * dH;
  out[plane + m] = B.u + wgt * dU;
  out[2 * plane + m] = B.v + wgt * dV;
}

// transposed contribution of reader k through offset o (1 .. 12) to the
// point x it reads there: lk = lambda^{n+1}(k), hk, uk, vk its state (h as
// the anomaly), K its row coefficients, X those of x's row, ux, vx the
// values k reads at x (sign applied across a pole); itp, itq = 1/p, 1/q
// (a multiply instead of a division per term)
template <typename T>
__device__ __forceinline__ V3<T> reader_term(int o, const V3<T>& lk, T hk, T uk, T vk,
                                             const RowCoef<T>& K, const RowCoef<T>& X, T ux,
                                             T vx, T st, T stg, T h0, T al, T itp, T itq) {
  const T one = T(1), half = T(0.5), hh = h0 + hk;
  switch (o) {
    case 1: case 2: {
      const T a = (o == 1 ? -K.a1 : K.a1) * uk;
      return {lk.h * a, lk.u * a, lk.v * a};
    }
    case 3: case 4: {
      const T a = (o == 3 ? -st : st) * vk;
      return {lk.h * a, lk.u * a, lk.v * a};
    }
    case 5: case 6: {
      const T sgn = o == 5 ? T(-1) : T(1);
      return {sgn * lk.u * K.a2 * itp, lk.u * half * al * K.ct * vx + sgn * lk.h * (one - al) * K.a1 * hh * itp,
              lk.u * half * al * (K.cf + K.ct * ux)};
    }
    case 7: case 8: {
      const T sgn = o == 7 ? T(-1) : T(1);
      return {sgn * lk.v * stg * itq, -lk.v * half * al * (X.cf + T(2) * X.ct * ux),
              sgn * lk.h * (one - al) * K.a3 * hh * X.c * itq};
    }
    default: {
      const T dn = half * al * K.a1 * hh * itp, cq = half * al * K.a3 * hh * X.c * itq;
      const T su = (o == 9 || o == 11) ? T(-1) : T(1), sv = (o == 9 || o == 10) ? T(-1) : T(1);
      return {T(0), su * lk.h * dn, sv * lk.h * cq};
    }
  }
}

// lambda^n (or the gradient at level 0) of every cell:
//   mode 0: cost forcing (observations + overlap), gradient and J at level 0
//   mode 1: caller forcing (packed FP64, trajectory layout), adj0 at level 0
//   mode 2: cost forcing, adj0 at level 0 (no background term)
//   mode 3: Gauss-Newton forcing W dZ^n from the tangent-linear trajectory
//           (eq. line5and7), adj0 at level 0, no cost
template <typename T, int MODE>
__global__ __launch_bounds__(kTile) void k_adj_tz(Dom<T> D, int n, int tile_base, int p, int q,
                                                  T alpha, int nlat, const double* __restrict__ x,
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
  const int r = mm / S.nx, c = mm - r * S.nx, ny = S.ny;
  double jloc = 0.0;
  // J_F(Z^n)^T lambda^{n+1} at this cell
  double ah = 0, au = 0, av = 0;
  if (has1 && valid) {
    const T* R = D.ring + S.ring_off + int64_t(n) * 3 * S.nring;
    Pt P[kOffs];
    points(S, r, c, p, q, D.half, nlat, P);
    const State13<T> z = load13(Z, R, plane, S.nring, P);
    const V3<T> lam = ld_box(L1, plane, mm, T(1));
    const RowCoef<T> rc = D.rows[S.row0 + r];
    const RowCoef<T> rN = D.rows[P[7].grow], rS = D.rows[P[8].grow];
    const T st = D.st, stg = D.stg, h0 = D.h0, al = alpha, one = T(1), half = T(0.5);
    // 1/p, 1/q: multiplying by them equals dividing when p, q are powers of two
    const T itp = one / T(p), itq = one / T(q);
    const V3<T>& C = z.C;
    // the cell itself
    {
      const T Dl = ((one - al) * (z.Ep.u - z.Wp.u) + half * al * (z.EN.u - z.WN.u + z.ES.u - z.WS.u)) * itp;
      const T Dt = ((one - al) * (z.Nq.v * rN.c - z.Sq.v * rS.c) + half * al * (z.EN.v * rN.c - z.ES.v * rS.c) +
                    half * al * (z.WN.v * rN.c - z.WS.v * rS.c)) * itq;
      ah += double(-lam.h * (rc.a1 * Dl + rc.a3 * Dt));
      au += double(lam.u * (-rc.a1 * (z.E.u - z.W.u) + (one - al) * rc.ct * C.v) +
                   lam.v * (-rc.a1 * (z.E.v - z.W.v) - (one - al) * (rc.cf + T(2) * rc.ct * C.u)) -
                   lam.h * rc.a1 * (z.E.h - z.W.h));
      av += double(lam.u * (-st * (z.N.u - z.Sv.u) + (one - al) * (rc.cf + rc.ct * C.u)) -
                   lam.v * st * (z.N.v - z.Sv.v) - lam.h * st * (z.N.h - z.Sv.h));
    }
    // in-box readers k = x - offset
#pragma unroll
    for (int o = 1; o < kOffs; ++o) {
      const int rk = r - off_r(o, q);
      int ck = c - off_c(o, p);
      if (rk < 0 || rk >= ny) continue;
      if (S.span) ck = ck < 0 ? ck + S.nx : (ck >= S.nx ? ck - S.nx : ck);
      else if (ck < 0 || ck >= S.nx) continue;
      const int k = rk * S.nx + ck;
      const V3<T> lk = ld_box(L1, plane, k, T(1));
      const V3<T> t = reader_term(o, lk, Z[k], Z[plane + k], Z[2 * plane + k], D.rows[S.row0 + rk], rc,
                                  C.u, C.v, st, stg, h0, al, itp, itq);
      ah += double(t.h);
      au += double(t.u);
      av += double(t.v);
    }
    // readers across a pole (a box spanning the circle): u, v negated
    if (S.span) {
      const int g = S.row0 + r;
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int o = a < 2 ? 3 + a : 5 + a;   // offsets 3, 4, 7 .. 12
        const int dr = off_r(o, q);
        const int gk = dr > 0 ? 2 * nlat - 1 - dr - g : -dr - 1 - g;
        const bool reach = dr > 0 ? g >= nlat - dr : g <= -dr - 1;
        if (!reach || gk < S.row0 || gk >= S.row0 + ny) continue;
        int ck = c - off_c(o, p) - D.half;
        ck = ((ck % S.nx) + S.nx) % S.nx;
        const int k = (gk - S.row0) * S.nx + ck;
        const V3<T> lk = ld_box(L1, plane, k, T(1));
        const V3<T> t = reader_term(o, lk, Z[k], Z[plane + k], Z[2 * plane + k], D.rows[gk], rc,
                                    -C.u, -C.v, st, stg, h0, al, itp, itq);
        ah += double(t.h);
        au -= double(t.u);
        av -= double(t.v);
      }
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
    if (n == 0) {
      ah = double(l0.h) + 0.5 * ah;
      au = double(l0.u) + 0.5 * au;
      av = double(l0.v) + 0.5 * av;
    }
    if (MODE != 1) {
      // overlap misfit, or in mode 3 the perturbation in its place
      const V3<T> C = ld_box(Z, plane, m, T(1));
      const V3<T> tg = MODE == 3 ? ld_box(D.dz + S.zoff + int64_t(n) * 3 * plane, plane, m, T(1))
                                 : ld_box(D.targ + S.traj_off + int64_t(n) * 3 * plane, plane,
                                          K > 0 ? m : 0, T(1));
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

// ---------------------------------------------------------------------------
// Column-walk adjoint for the q = 2 offset.  One wave owns the columns
// c0 - p .. c0 + 63 - p of one box (its outputs are the columns of the box
// among lanes p .. 63 - p) and walks the rows r0 .. r1 - 1.  Every lane keeps,
// for its column, the state and lambda^{n+1} of the rows r - 2 .. r + 2 in
// registers: the values the 13-point stencil reads there (box cells, frozen
// pad values, or box cells across a pole with u, v negated), and lambda only
// at box cells (zero elsewhere: no reader lives there).  It loads one new row
// per step, one step ahead, and takes the other columns from the lanes p
// (through the LDS crossbar) and 1 (DPP wave shifts) to either side; the
// forcing's loads of a step (lambda^{n+2}, the overlap target) are issued
// before its arithmetic, with the coverage byte fetched one step ahead.  The
// 12 in-box readers of a cell are the points of its
// own stencil at the opposite offsets, so the window serves both, and a
// reader outside the box contributes zero.  Arithmetic and its order as in
// k_adj_tz (own terms, readers 1 .. 12, readers across a pole, summed in
// FP64); the observation forcing is added afterwards by k_obs_tz, and each
// wave's share of J goes to its own slot of the box's tile accumulators.
constexpr int kColQ = 2;
constexpr int kColThreads = 256;

template <typename T>
struct WinRow {
  V3<T> z, l;
};

// window entry of box row rr (-2 .. ny + 1) and column col (wrapped into the
// box for a box spanning the circle, -p .. nx + p - 1 otherwise; a lane with
// no such column reads column 0 and serves no output), as loaded: the
// stencil's state, and lambda^{n+1} read at a box cell in any case, with the
// flag that it is one (zero otherwise).  Every load is issued without a
// branch around it, so that none is waited for before the row enters the
// window one step later (win_take applies the flag then).
template <typename T>
struct WinLoad {
  V3<T> z, l;
  bool lin;
};
template <typename T>
__device__ __forceinline__ WinLoad<T> win_issue(const SubDev& S, const T* Z, const T* R, const T* L1,
                                                int64_t plane, int rr, int col, bool col_ok,
                                                bool has1, int p, int half, int nlat) {
  const Pt P = point(S, rr, col_ok ? col : 0, 0, 0, p, kColQ, half, nlat);
  WinLoad<T> w;
  w.z = ld_pt(Z, R, plane, S.nring, P);
  const bool in_box = !P.pad && !P.across;
  w.l = ld_box(L1, plane, in_box ? P.idx : 0, T(1));
  w.lin = col_ok && has1 && in_box;
  return w;
}

// per lane a (lanes in mask) or b, as one v_cndmask per 32 bits written out
// (a select left to the compiler can become a branch that waits for a)
__device__ __forceinline__ float pick_lane(float a, float b, uint64_t mask) {
  float r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(b), "v"(a), "s"(mask));
  return r;
}
__device__ __forceinline__ double pick_lane(double a, double b, uint64_t mask) {
  const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
  const float lo = pick_lane(__builtin_bit_cast(float, uint32_t(ua)), __builtin_bit_cast(float, uint32_t(ub)), mask);
  const float hi = pick_lane(__builtin_bit_cast(float, uint32_t(ua >> 32)),
                             __builtin_bit_cast(float, uint32_t(ub >> 32)), mask);
  return __builtin_bit_cast(double, (uint64_t(__builtin_bit_cast(uint32_t, hi)) << 32) |
                                        __builtin_bit_cast(uint32_t, lo));
}
template <typename T>
__device__ __forceinline__ V3<T> pick3_lane(const V3<T>& a, uint64_t mask) {
  return {pick_lane(a.h, T(0), mask), pick_lane(a.u, T(0), mask), pick_lane(a.v, T(0), mask)};
}
template <typename T>
__device__ __forceinline__ WinRow<T> win_take(const WinLoad<T>& w) {
  return {w.z, pick3_lane(w.l, __builtin_amdgcn_ballot_w64(w.lin))};
}

template <typename T>
__device__ __forceinline__ WinRow<T> win_shfl(const WinRow<T>& w, int src) {
  WinRow<T> o;
  o.z = {__shfl(w.z.h, src, 64), __shfl(w.z.u, src, 64), __shfl(w.z.v, src, 64)};
  o.l = {__shfl(w.l.h, src, 64), __shfl(w.l.u, src, 64), __shfl(w.l.v, src, 64)};
  return o;
}


// value of the lane one above (wave_shl:1) or one below (wave_shr:1) in the wave
template <typename T>
__device__ __forceinline__ T lane_next(T v) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, false));
  } else {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, int(b), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), 0x130, 0xf, 0xf, false);
    return __builtin_bit_cast(T, (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
  }
}
template <typename T>
__device__ __forceinline__ T lane_prev(T v) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
  } else {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, int(b), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), 0x138, 0xf, 0xf, false);
    return __builtin_bit_cast(T, (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
  }
}
template <typename T>
__device__ __forceinline__ WinRow<T> win_next(const WinRow<T>& w) {
  return {{lane_next(w.z.h), lane_next(w.z.u), lane_next(w.z.v)}, {lane_next(w.l.h), lane_next(w.l.u), lane_next(w.l.v)}};
}
template <typename T>
__device__ __forceinline__ WinRow<T> win_prev(const WinRow<T>& w) {
  return {{lane_prev(w.z.h), lane_prev(w.z.u), lane_prev(w.z.v)}, {lane_prev(w.l.h), lane_prev(w.l.u), lane_prev(w.l.v)}};
}
// coefficient row of box row rr, mirrored across a pole
__device__ __forceinline__ int grow_of(const SubDev& S, int rr, int nlat) {
  const int g = S.row0 + rr;
  return g < 0 ? -1 - g : (g >= nlat ? 2 * nlat - 1 - g : g);
}

// (occupancy: four waves per SIMD in FP32, two in FP64, each within its
// register budget)
template <typename T, int MODE>
__global__ __launch_bounds__(kColThreads, sizeof(T) == 4 ? 4 : 2) void k_adj_tz_col(Dom<T> D, int n,
                                                            const TzWork* __restrict__ work,
                                                            int nwork, int p, T alpha, int nlat,
                                                            const double* __restrict__ x,
                                                            const double* __restrict__ xb,
                                                            const double* __restrict__ forcing,
                                                            double* __restrict__ out) {
  // consecutive work items (the strips of one box column) on one XCD
  // (uniform over the wave: its work item, box and rows live in scalar registers)
  const int wv = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * (kColThreads / 64) +
                                                int(threadIdx.x >> 6));
  if (wv >= nwork) return;                 // whole waves; no workgroup barrier below
  const TzWork wk = work[wv];
  if (D.active && !D.active[wk.box]) return;
  const SubDev S = D.subs[wk.box];
  const int L = S.nlev - 1;
  if (n > L) return;
  const int lane = int(threadIdx.x & 63);
  const int nx = S.nx, ny = S.ny;
  const int c = wk.c0 + lane - p;           // this lane's column
  const bool out_lane = lane >= p && lane < 64 - p && c < nx;
  const bool col_ok = S.span || c < nx + p;
  const int colw = S.span ? ((c % nx) + nx) % nx : c;
  const int64_t plane = S.ncell;
  const T* Z = zlevel(D, S, n);
  const T* R = D.ring + S.ring_off + int64_t(n) * 3 * S.nring;
  T* A = D.adj + S.adj_off;
  const bool has1 = n + 1 <= L, has2 = n + 2 <= L;
  const T* L1 = A + int64_t((n + 1) % 3) * 3 * plane;
  const T* L2 = A + int64_t((n + 2) % 3) * 3 * plane;
  const T st = D.st, stg = D.stg, h0 = D.h0, al = alpha, one = T(1), half = T(0.5);
  const T itp = one / T(p), itq = one / T(kColQ);
  const int q = kColQ;
  const int hl = D.half;
  const int lEp = min(lane + p, 63), lWp = max(lane - p, 0);
  double jloc = 0.0;

  WinRow<T> w[5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
    w[i] = win_take(win_issue(S, Z, R, L1, plane, wk.r0 - 2 + i, colw, col_ok, has1, p, hl, nlat));
  WinLoad<T> pf;
  // coverage byte of the lane's cell in the step's row, one step ahead (a
  // lane without an output reads cell 0)
  const int tcn = MODE != 1 ? D.tcount[S.lev0 + n] : 0;
  int cov = MODE != 1 ? int(D.cover[S.cell_off + (out_lane ? wk.r0 * nx + c : 0)]) : 0;
  for (int r = wk.r0; r < wk.r1; ++r) {
    // coefficient rows of the step: own, pole-mirrored north and south, and
    // the readers' north and south rows clamped into the box (a reader
    // outside it has lambda zero), loaded first: the loads of a wave complete
    // in order, so that waiting for them leaves the later ones in flight
    const RowCoef<T> rc = D.rows[__builtin_amdgcn_readfirstlane(S.row0 + r)];
    const RowCoef<T> rN = D.rows[__builtin_amdgcn_readfirstlane(grow_of(S, r + q, nlat))];
    const RowCoef<T> rS = D.rows[__builtin_amdgcn_readfirstlane(grow_of(S, r - q, nlat))];
    const RowCoef<T> rKs = D.rows[__builtin_amdgcn_readfirstlane(S.row0 + max(r - q, 0))];
    const RowCoef<T> rKn = D.rows[__builtin_amdgcn_readfirstlane(S.row0 + min(r + q, ny - 1))];
    if (r > wk.r0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) w[i] = w[i + 1];
      w[4] = win_take(pf);
    }
    // this step's loads, by every lane and before any arithmetic: the
    // window's next row and coverage byte, lambda^{n+2} and the target (or
    // dZ) of the step's cell
    // (on the strip's last step they read rows the window never takes, kept
    // inside the pad and the box)
    const int cov_r = cov;
    pf = win_issue(S, Z, R, L1, plane, min(r + 3, ny + kColQ - 1), colw, col_ok, has1, p, hl, nlat);
    if (MODE != 1) cov = int(D.cover[S.cell_off + (out_lane ? min(r + 1, ny - 1) * nx + c : 0)]);
    const int m = out_lane ? r * nx + c : 0;
    const int K = cov_r * tcn - 1;
    const V3<T> l2raw = ld_box(L2, plane, m, T(1));
    V3<T> tg = {T(0), T(0), T(0)};
    if (MODE == 3) tg = ld_box(D.dz + S.zoff + int64_t(n) * 3 * plane, plane, m, T(1));
    else if (MODE != 1) tg = ld_box(D.targ + S.traj_off + int64_t(n) * 3 * plane, plane, K > 0 ? m : 0, T(1));
    // the other columns' values: row r at lanes +-1 and +-p, rows r +- q at
    // lanes +-p (every lane takes part in the exchange)
    const WinRow<T> E1 = win_next(w[2]), W1 = win_prev(w[2]);
    const WinRow<T> Ep = win_shfl(w[2], lEp), Wp = win_shfl(w[2], lWp);
    const WinRow<T> EN = win_shfl(w[4], lEp), WN = win_shfl(w[4], lWp);
    const WinRow<T> ES = win_shfl(w[0], lEp), WS = win_shfl(w[0], lWp);
    if (!out_lane) continue;
    const V3<T> C = w[2].z;
    double ah = 0, au = 0, av = 0;
    if (has1) {
      const V3<T> lam = w[2].l;
      {
        const T Dl = ((one - al) * (Ep.z.u - Wp.z.u) + half * al * (EN.z.u - WN.z.u + ES.z.u - WS.z.u)) * itp;
        const T Dt = ((one - al) * (w[4].z.v * rN.c - w[0].z.v * rS.c) +
                      half * al * (EN.z.v * rN.c - ES.z.v * rS.c) +
                      half * al * (WN.z.v * rN.c - WS.z.v * rS.c)) * itq;
        ah += double(-lam.h * (rc.a1 * Dl + rc.a3 * Dt));
        au += double(lam.u * (-rc.a1 * (E1.z.u - W1.z.u) + (one - al) * rc.ct * C.v) +
                     lam.v * (-rc.a1 * (E1.z.v - W1.z.v) - (one - al) * (rc.cf + T(2) * rc.ct * C.u)) -
                     lam.h * rc.a1 * (E1.z.h - W1.z.h));
        av += double(lam.u * (-st * (w[3].z.u - w[1].z.u) + (one - al) * (rc.cf + rc.ct * C.u)) -
                     lam.v * st * (w[3].z.v - w[1].z.v) - lam.h * st * (w[3].z.h - w[1].z.h));
      }
      // readers k = x - offset o: the stencil point at the opposite offset
#pragma unroll
      for (int o = 1; o < kOffs; ++o) {
        const WinRow<T>& k = o == 1 ? W1 : o == 2 ? E1 : o == 3 ? w[1] : o == 4 ? w[3]
                           : o == 5 ? Wp : o == 6 ? Ep : o == 7 ? w[0] : o == 8 ? w[4]
                           : o == 9 ? WS : o == 10 ? ES : o == 11 ? WN : EN;
        const RowCoef<T>& K = (o == 7 || o == 9 || o == 10) ? rKs : (o == 8 || o == 11 || o == 12) ? rKn : rc;
        const V3<T> t = reader_term(o, k.l, k.z.h, k.z.u, k.z.v, K, rc, C.u, C.v, st, stg, h0, al, itp, itq);
        ah += double(t.h);
        au += double(t.u);
        av += double(t.v);
      }
      // readers across a pole (a box spanning the circle): u, v negated
      if (S.span) {
        const int g = S.row0 + r;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const int o = a < 2 ? 3 + a : 5 + a;   // offsets 3, 4, 7 .. 12
          const int dr = off_r(o, q);
          const int gk = dr > 0 ? 2 * nlat - 1 - dr - g : -dr - 1 - g;
          const bool reach = dr > 0 ? g >= nlat - dr : g <= -dr - 1;
          if (!reach || gk < S.row0 || gk >= S.row0 + ny) continue;
          int ck = c - off_c(o, p) - hl;
          ck = ((ck % nx) + nx) % nx;
          const int kk = (gk - S.row0) * nx + ck;
          const V3<T> lk = ld_box(L1, plane, kk, T(1));
          const V3<T> t = reader_term(o, lk, Z[kk], Z[plane + kk], Z[2 * plane + kk], D.rows[gk], rc,
                                      -C.u, -C.v, st, stg, h0, al, itp, itq);
          ah += double(t.h);
          au -= double(t.u);
          av -= double(t.v);
        }
      }
    }
    const V3<T> l0 = w[2].l;
    const V3<T> l2 = has2 ? l2raw : V3<T>{T(0), T(0), T(0)};
    double fh = 0, fu = 0, fv = 0;
    if (MODE == 1) {
      const double* Fz = forcing + S.traj_off + int64_t(n) * 3 * plane;
      fh = Fz[m];
      fu = Fz[plane + m];
      fv = Fz[2 * plane + m];
    }
    if (n == 0) {
      ah = double(l0.h) + 0.5 * ah;
      au = double(l0.u) + 0.5 * au;
      av = double(l0.v) + 0.5 * av;
    }
    if (MODE != 1) {
      // overlap misfit, or in mode 3 the perturbation in its place
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
    // the wave's share of J (fixed reduction order) into its slot; at the
    // box's first level the slots of no wave are cleared
    double v = jloc;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) D.jpart[wk.slot] = (n == L) ? v : D.jpart[wk.slot] + v;
    if (n == L)
      for (int t = wk.zero0 + lane; t < wk.zero1; t += 64) D.jpart[t] = 0.0;
  }
}

// Column-walk forward step for the q = 2 offset: the waves of the adjoint's
// column walk (same blocks of columns and strips of rows), each lane keeping
// the state of the rows r - 2 .. r + 2 of its column as the 13-point stencil
// reads them (box cells, frozen pad values, or box cells across a pole with
// u, v negated), loading one new row per step, one step ahead, and taking
// the other columns from the lanes 1 (DPP) and p (LDS crossbar) to either
// side.  Arithmetic as in k_fwd_tz.
template <typename T>
__global__ __launch_bounds__(kColThreads) void k_fwd_tz_col(Dom<T> D, int n,
                                                            const TzWork* __restrict__ work,
                                                            int nwork, int p, T alpha, int nlat) {
  const int wv = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * (kColThreads / 64) +
                                                int(threadIdx.x >> 6));
  if (wv >= nwork) return;                 // whole waves; no workgroup barrier below
  const TzWork wk = work[wv];
  if (D.active && !D.active[wk.box]) return;
  const SubDev S = D.subs[wk.box];
  if (n >= S.nlev - 1) return;
  const int lane = int(threadIdx.x & 63);
  const int nx = S.nx, ny = S.ny;
  const int c = wk.c0 + lane - p;
  const bool out_lane = lane >= p && lane < 64 - p && c < nx;
  const bool col_ok = S.span || c < nx + p;
  const int colw = S.span ? ((c % nx) + nx) % nx : c;
  const int64_t plane = S.ncell;
  const T* Z = zlevel(D, S, n);
  const T* B0 = n >= 1 ? zlevel(D, S, n - 1) : Z;
  const T* R = D.ring + S.ring_off + int64_t(n) * 3 * S.nring;
  T* out = zlevel(D, S, n + 1);
  const T st = D.st, stg = D.stg, h0 = D.h0, al = alpha, one = T(1), half = T(0.5);
  const T itp = one / T(p), itq = one / T(kColQ);
  const int q = kColQ;
  const int hl = D.half;
  const int lEp = min(lane + p, 63), lWp = max(lane - p, 0);
  const T wgt = n == 0 ? T(0.5) : T(1);
  auto zload = [&](int rr) {
    const Pt P = point(S, rr, col_ok ? colw : 0, 0, 0, p, kColQ, hl, nlat);
    return ld_pt(Z, R, plane, S.nring, P);
  };
  V3<T> w[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) w[i] = zload(wk.r0 - 2 + i);
  V3<T> pf;
  for (int r = wk.r0; r < wk.r1; ++r) {
    // coefficient rows first (the loads of a wave complete in order)
    const RowCoef<T> rc = D.rows[__builtin_amdgcn_readfirstlane(S.row0 + r)];
    const RowCoef<T> rN = D.rows[__builtin_amdgcn_readfirstlane(grow_of(S, r + q, nlat))];
    const RowCoef<T> rS = D.rows[__builtin_amdgcn_readfirstlane(grow_of(S, r - q, nlat))];
    if (r > wk.r0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) w[i] = w[i + 1];
      w[4] = pf;
    }
    pf = zload(min(r + 3, ny + kColQ - 1));
    const int m = out_lane ? r * nx + c : 0;
    const V3<T> B = ld_box(B0, plane, m, T(1));
    const V3<T> E = {lane_next(w[2].h), lane_next(w[2].u), lane_next(w[2].v)};
    const V3<T> W = {lane_prev(w[2].h), lane_prev(w[2].u), lane_prev(w[2].v)};
    const V3<T> Ep = {__shfl(w[2].h, lEp, 64), __shfl(w[2].u, lEp, 64), __shfl(w[2].v, lEp, 64)};
    const V3<T> Wp = {__shfl(w[2].h, lWp, 64), __shfl(w[2].u, lWp, 64), __shfl(w[2].v, lWp, 64)};
    const T ENu = __shfl(w[4].u, lEp, 64), ENv = __shfl(w[4].v, lEp, 64);
    const T WNu = __shfl(w[4].u, lWp, 64), WNv = __shfl(w[4].v, lWp, 64);
    const T ESu = __shfl(w[0].u, lEp, 64), ESv = __shfl(w[0].v, lEp, 64);
    const T WSu = __shfl(w[0].u, lWp, 64), WSv = __shfl(w[0].v, lWp, 64);
    if (!out_lane) continue;
    const V3<T>& C = w[2];
    const V3<T>& N = w[3];
    const V3<T>& Sv = w[1];
    const V3<T>& Nq = w[4];
    const V3<T>& Sq = w[0];
    const T hh = h0 + C.h;
    const T U = -rc.a1 * C.u * (E.u - W.u) - st * C.v * (N.u - Sv.u) -
                rc.a2 * itp * (Ep.h - Wp.h) +
                ((one - al) * (rc.cf + rc.ct * C.u) * C.v + half * al * (rc.cf + rc.ct * Ep.u) * Ep.v +
                 half * al * (rc.cf + rc.ct * Wp.u) * Wp.v);
    const T V = -rc.a1 * C.u * (E.v - W.v) - st * C.v * (N.v - Sv.v) -
                stg * itq * (Nq.h - Sq.h) -
                ((one - al) * (rc.cf + rc.ct * C.u) * C.u + half * al * (rN.cf + rN.ct * Nq.u) * Nq.u +
                 half * al * (rS.cf + rS.ct * Sq.u) * Sq.u);
    const T Dl = ((one - al) * (Ep.u - Wp.u) + half * al * (ENu - WNu + ESu - WSu)) * itp;
    const T Dt = ((one - al) * (Nq.v * rN.c - Sq.v * rS.c) + half * al * (ENv * rN.c - ESv * rS.c) +
                  half * al * (WNv * rN.c - WSv * rS.c)) * itq;
    const T H = -rc.a1 * (C.u * (E.h - W.h) + hh * Dl) - (st * C.v * (N.h - Sv.h) + rc.a3 * hh * Dt);
    out[m] = B.h + wgt * H;
    out[plane + m] = B.u + wgt * U;
    out[2 * plane + m] = B.v + wgt * V;
  }
}

// Column-walk tangent-linear step for the q = 2 offset (the TLM step of
// Alg. 6 under the variant): the forward's waves, each lane keeping the
// state and the perturbation of the rows r - 2 .. r + 2 of its column (the
// perturbation zero at frozen pad positions, whose values do not depend on
// the control, and negated in u, v across a pole), one new row per step.
// Arithmetic as in k_tlm_tz.
template <typename T>
__global__ __launch_bounds__(kColThreads) void k_tlm_tz_col(Dom<T> D, int n,
                                                            const TzWork* __restrict__ work,
                                                            int nwork, int p, T alpha, int nlat) {
  const int wv = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * (kColThreads / 64) +
                                                int(threadIdx.x >> 6));
  if (wv >= nwork) return;                 // whole waves; no workgroup barrier below
  const TzWork wk = work[wv];
  if (D.active && !D.active[wk.box]) return;
  const SubDev S = D.subs[wk.box];
  if (n >= S.nlev - 1) return;
  const int lane = int(threadIdx.x & 63);
  const int nx = S.nx, ny = S.ny;
  const int c = wk.c0 + lane - p;
  const bool out_lane = lane >= p && lane < 64 - p && c < nx;
  const bool col_ok = S.span || c < nx + p;
  const int colw = S.span ? ((c % nx) + nx) % nx : c;
  const int64_t plane = S.ncell;
  const T* Z = zlevel(D, S, n);
  const T* R = D.ring + S.ring_off + int64_t(n) * 3 * S.nring;
  const T* dZ = D.dz + S.zoff + int64_t(n) * 3 * plane;
  const T* dB = n >= 1 ? D.dz + S.zoff + int64_t(n - 1) * 3 * plane : dZ;
  T* out = D.dz + S.zoff + int64_t(n + 1) * 3 * plane;
  const T st = D.st, stg = D.stg, h0 = D.h0, al = alpha, one = T(1), half = T(0.5);
  const T itp = one / T(p), itq = one / T(kColQ);
  const int q = kColQ;
  const int hl = D.half;
  const int lEp = min(lane + p, 63), lWp = max(lane - p, 0);
  const T wgt = n == 0 ? T(0.5) : T(1);
  // the state and the perturbation as loaded (no branch around the loads);
  // the perturbation's pad flag and pole sign are applied when the row
  // enters the window
  struct TLoad {
    V3<T> z, d;
    bool din;
    T sg;
  };
  auto issue = [&](int rr) {
    const Pt P = point(S, rr, col_ok ? colw : 0, 0, 0, p, kColQ, hl, nlat);
    TLoad t;
    t.z = ld_pt(Z, R, plane, S.nring, P);
    t.d = ld_box(dZ, plane, P.pad ? 0 : P.idx, T(1));
    t.din = !P.pad;
    t.sg = T(P.sg);
    return t;
  };
  auto take = [&](const TLoad& t) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(t.din);
    WinRow<T> w;
    w.z = t.z;
    w.l = {pick_lane(t.d.h, T(0), m), t.sg * pick_lane(t.d.u, T(0), m), t.sg * pick_lane(t.d.v, T(0), m)};
    return w;
  };
  WinRow<T> w[5];                          // .z the state, .l the perturbation
#pragma unroll
  for (int i = 0; i < 5; ++i) w[i] = take(issue(wk.r0 - 2 + i));
  TLoad pf;
  for (int r = wk.r0; r < wk.r1; ++r) {
    const RowCoef<T> rc = D.rows[__builtin_amdgcn_readfirstlane(S.row0 + r)];
    const RowCoef<T> rN = D.rows[__builtin_amdgcn_readfirstlane(grow_of(S, r + q, nlat))];
    const RowCoef<T> rS = D.rows[__builtin_amdgcn_readfirstlane(grow_of(S, r - q, nlat))];
    if (r > wk.r0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) w[i] = w[i + 1];
      w[4] = take(pf);
    }
    pf = issue(min(r + 3, ny + kColQ - 1));
    const int m = out_lane ? r * nx + c : 0;
    const V3<T> B = ld_box(dB, plane, m, T(1));
    const WinRow<T> E1 = win_next(w[2]), W1 = win_prev(w[2]);
    const WinRow<T> Ep = win_shfl(w[2], lEp), Wp = win_shfl(w[2], lWp);
    const WinRow<T> EN = win_shfl(w[4], lEp), WN = win_shfl(w[4], lWp);
    const WinRow<T> ES = win_shfl(w[0], lEp), WS = win_shfl(w[0], lWp);
    if (!out_lane) continue;
    const V3<T>& C = w[2].z;
    const V3<T>& dC = w[2].l;
    const T hh = h0 + C.h;
    const T dU = -rc.a1 * (dC.u * (E1.z.u - W1.z.u) + C.u * (E1.l.u - W1.l.u)) -
                 st * (dC.v * (w[3].z.u - w[1].z.u) + C.v * (w[3].l.u - w[1].l.u)) -
                 rc.a2 * itp * (Ep.l.h - Wp.l.h) +
                 ((one - al) * (rc.ct * dC.u * C.v + (rc.cf + rc.ct * C.u) * dC.v) +
                  half * al * (rc.ct * Ep.l.u * Ep.z.v + (rc.cf + rc.ct * Ep.z.u) * Ep.l.v) +
                  half * al * (rc.ct * Wp.l.u * Wp.z.v + (rc.cf + rc.ct * Wp.z.u) * Wp.l.v));
    const T dV = -rc.a1 * (dC.u * (E1.z.v - W1.z.v) + C.u * (E1.l.v - W1.l.v)) -
                 st * (dC.v * (w[3].z.v - w[1].z.v) + C.v * (w[3].l.v - w[1].l.v)) -
                 stg * itq * (w[4].l.h - w[0].l.h) -
                 ((one - al) * (rc.cf + T(2) * rc.ct * C.u) * dC.u +
                  half * al * (rN.cf + T(2) * rN.ct * w[4].z.u) * w[4].l.u +
                  half * al * (rS.cf + T(2) * rS.ct * w[0].z.u) * w[0].l.u);
    const T Dl = ((one - al) * (Ep.z.u - Wp.z.u) + half * al * (EN.z.u - WN.z.u + ES.z.u - WS.z.u)) * itp;
    const T Dt = ((one - al) * (w[4].z.v * rN.c - w[0].z.v * rS.c) +
                  half * al * (EN.z.v * rN.c - ES.z.v * rS.c) +
                  half * al * (WN.z.v * rN.c - WS.z.v * rS.c)) * itq;
    const T dDl = ((one - al) * (Ep.l.u - Wp.l.u) + half * al * (EN.l.u - WN.l.u + ES.l.u - WS.l.u)) * itp;
    const T dDt = ((one - al) * (w[4].l.v * rN.c - w[0].l.v * rS.c) +
                   half * al * (EN.l.v * rN.c - ES.l.v * rS.c) +
                   half * al * (WN.l.v * rN.c - WS.l.v * rS.c)) * itq;
    const T dH = -rc.a1 * (dC.u * (E1.z.h - W1.z.h) + C.u * (E1.l.h - W1.l.h) + dC.h * Dl + hh * dDl) -
                 (st * (dC.v * (w[3].z.h - w[1].z.h) + C.v * (w[3].l.h - w[1].l.h)) +
                  rc.a3 * (dC.h * Dt + hh * dDt));
    out[m] = B.h + wgt * dH;
    out[plane + m] = B.u + wgt * dU;
    out[2 * plane + m] = B.v + wgt * dV;
  }
}

// observation forcing of the column-walk adjoint at level n: for every entry
// of a (tile, level) bin, q_o (Z - y) (or q_o dZ in mode 3) added to
// lambda^n, or at level 0 to the gradient / adj0; its share of J added to
// the tile's accumulator.  A cell and field occur at most once per level.
template <typename T, int MODE>
__global__ __launch_bounds__(kTile) void k_obs_tz(Dom<T> D, int n, const int32_t* __restrict__ tiles,
                                                  int tile_base, int ntiles,
                                                  double* __restrict__ out) {
  __shared__ double red[kTile / 64];
  // one tile of the level's list (the tiles with entries at level n), if it
  // belongs to the launched boxes
  const int w = tiles[blockIdx.x];
  if (w < tile_base || w >= tile_base + ntiles) return;
  const int2 wt = D.tiles[w];
  if (D.active && !D.active[wt.x]) return;
  const SubDev S = D.subs[wt.x];
  if (n > S.nlev - 1) return;
  const int64_t key = obs_key(S.tile0, S.ntile, D.maxlev, wt.y, n);
  const int o0 = D.obs_ptr[key], o1 = D.obs_ptr[key + 1];
  if (o1 <= o0) return;                    // uniform over the block
  const int64_t plane = S.ncell;
  const T* Z = zlevel(D, S, n);
  T* An = D.adj + S.adj_off + int64_t(n % 3) * 3 * plane;
  double jloc = 0.0;
  for (int o = o0 + int(threadIdx.x); o < o1; o += kTile) {
    const int code = D.obs_code[o];
    const int loc = code >> 2, f = code & 3;
    const double rr = MODE == 3 ? double(D.dz[S.zoff + int64_t(n) * 3 * plane + f * plane + loc])
                                : double(Z[f * plane + loc]) - D.obs_val[o];
    const double qo = D.obs_q[o];
    if (MODE != 3) jloc += 0.5 * qo * rr * rr;
    if (n > 0) {
      T* a = An + f * plane + loc;
      *a = T(double(*a) + qo * rr);
    } else {
      out[S.ctrl_off + f * plane + loc] += qo * rr;
    }
  }
  if (MODE == 0 || MODE == 2) {
    const double tot = block_sum(jloc, red);
    if (threadIdx.x == 0) D.jpart[w] += tot;
  }
}

template <typename T>
void launch_fwd_tz(const Dom<T>& D, int n, int tile_base, int ntiles, int p, int q, double alpha,
                   int nlat, const TzWork* work, int nwork, hipStream_t st) {
  if (work) {
    const int nb = (nwork + kColThreads / 64 - 1) / (kColThreads / 64);
    if (nb > 0)
      hipLaunchKernelGGL(k_fwd_tz_col<T>, dim3(nb), dim3(kColThreads), 0, st, D, n, work, nwork, p,
                         T(alpha), nlat);
    return;
  }
  hipLaunchKernelGGL(k_fwd_tz<T>, dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base, p, q, T(alpha),
                     nlat);
}
template <typename T>
void launch_adj_tz(const Dom<T>& D, int n, int tile_base, int ntiles, int mode, int p, int q,
                   double alpha, int nlat, const double* x, const double* xb,
                   const double* forcing, double* out, const TzWork* work, int nwork,
                   const int32_t* obs_tiles, int nobs_tiles, hipStream_t st) {
  if (work) {
    // column walk (q = 2), then the observation forcing of the level over
    // the tiles that have entries there
    const int nb = (nwork + kColThreads / 64 - 1) / (kColThreads / 64);
    if (nb == 0) return;
    if (mode == 0)
      hipLaunchKernelGGL((k_adj_tz_col<T, 0>), dim3(nb), dim3(kColThreads), 0, st, D, n, work, nwork,
                         p, T(alpha), nlat, x, xb, forcing, out);
    else if (mode == 1)
      hipLaunchKernelGGL((k_adj_tz_col<T, 1>), dim3(nb), dim3(kColThreads), 0, st, D, n, work, nwork,
                         p, T(alpha), nlat, x, xb, forcing, out);
    else if (mode == 2)
      hipLaunchKernelGGL((k_adj_tz_col<T, 2>), dim3(nb), dim3(kColThreads), 0, st, D, n, work, nwork,
                         p, T(alpha), nlat, x, xb, forcing, out);
    else
      hipLaunchKernelGGL((k_adj_tz_col<T, 3>), dim3(nb), dim3(kColThreads), 0, st, D, n, work, nwork,
                         p, T(alpha), nlat, x, xb, forcing, out);
    if (nobs_tiles == 0) return;
    if (mode == 0)
      hipLaunchKernelGGL((k_obs_tz<T, 0>), dim3(nobs_tiles), dim3(kTile), 0, st, D, n, obs_tiles,
                         tile_base, ntiles, out);
    else if (mode == 2)
      hipLaunchKernelGGL((k_obs_tz<T, 2>), dim3(nobs_tiles), dim3(kTile), 0, st, D, n, obs_tiles,
                         tile_base, ntiles, out);
    else if (mode == 3)
      hipLaunchKernelGGL((k_obs_tz<T, 3>), dim3(nobs_tiles), dim3(kTile), 0, st, D, n, obs_tiles,
                         tile_base, ntiles, out);
    return;
  }
  if (mode == 0)
    hipLaunchKernelGGL((k_adj_tz<T, 0>), dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base, p, q,
                       T(alpha), nlat, x, xb, forcing, out);
  else if (mode == 1)
    hipLaunchKernelGGL((k_adj_tz<T, 1>), dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base, p, q,
                       T(alpha), nlat, x, xb, forcing, out);
  else if (mode == 2)
    hipLaunchKernelGGL((k_adj_tz<T, 2>), dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base, p, q,
                       T(alpha), nlat, x, xb, forcing, out);
  else
    hipLaunchKernelGGL((k_adj_tz<T, 3>), dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base, p, q,
                       T(alpha), nlat, x, xb, forcing, out);
}
template <typename T>
void launch_tlm_tz(const Dom<T>& D, int n, int tile_base, int ntiles, int p, int q, double alpha,
                   int nlat, const TzWork* work, int nwork, hipStream_t st) {
  if (work) {
    const int nb = (nwork + kColThreads / 64 - 1) / (kColThreads / 64);
    if (nb > 0)
      hipLaunchKernelGGL(k_tlm_tz_col<T>, dim3(nb), dim3(kColThreads), 0, st, D, n, work, nwork, p,
                         T(alpha), nlat);
    return;
  }
  hipLaunchKernelGGL(k_tlm_tz<T>, dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base, p, q, T(alpha),
                     nlat);
}

#define DD4DVAR_INST(T)                                                                        \
  template void launch_fwd_tz<T>(const Dom<T>&, int, int, int, int, int, double, int,         \
                                 const TzWork*, int, hipStream_t);                            \
  template void launch_adj_tz<T>(const Dom<T>&, int, int, int, int, int, int, double, int,     \
                                 const double*, const double*, const double*, double*,        \
                                 const TzWork*, int, const int32_t*, int, hipStream_t);       \
  template void launch_tlm_tz<T>(const Dom<T>&, int, int, int, int, int, double, int,         \
                                 const TzWork*, int, hipStream_t);
DD4DVAR_INST(DD4DVAR_TZ_T)
#undef DD4DVAR_INST

}  // namespace dd4dvar
