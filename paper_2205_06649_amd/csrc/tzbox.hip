// Persistent forward sweep of the Turkel-Zwas variant (Sec. 7 discrete U, V,
// H with offsets p, q and averaging alpha), FP32 state: one 1024-thread
// workgroup per box for the whole interval, the box's level in an LDS frame
// q rows and p columns wider than the box on each side, the level before it
// in registers, each new level written to memory once.  The frame's border
// holds the level's frozen pad values (the ring arena of the variant),
// refreshed at every step.  Boxes that span the circle (whose points reach
// across a pole into the box itself) are not taken here.
#include "kernels.h"
#include "launch.h"
#include "stencil.h"

namespace dd4dvar {

using namespace stencil;

namespace {
constexpr int kTzThreads = 1024;
constexpr int kTzKMax = 11;                   // passes: boxes of up to 11 x 1024 cells
constexpr int kTzRingMax = 2;                 // pad positions per thread: up to 2048
constexpr int kTzRowWords = 12;               // row table entry

// global row of box row rr, mirrored across a pole
__device__ __forceinline__ int tz_grow(const SubDev& S, int rr, int nlat) {
  const int g = S.row0 + rr;
  return g < 0 ? -1 - g : (g >= nlat ? 2 * nlat - 1 - g : g);
}

// frame index of pad position k (the variant's ring layout: q rows above the
// box, q rows below, each nx + 2p wide, then p columns west and p columns
// east of every box row)
__device__ __forceinline__ int tz_pad_frame(int k, int nx, int ny, int p, int q) {
  const int w = nx + 2 * p;
  int rr, cc;
  if (k < q * w) {
    rr = k / w - q;
    cc = k % w - p;
  } else if (k < 2 * q * w) {
    const int k2 = k - q * w;
    rr = ny + k2 / w;
    cc = k2 % w - p;
  } else if (k < 2 * q * w + ny * p) {
    const int k3 = k - 2 * q * w;
    rr = k3 / p;
    cc = k3 % p - p;
  } else {
    const int k4 = k - 2 * q * w - ny * p;
    rr = k4 / p;
    cc = nx + k4 % p;
  }
  return (rr + q) * w + cc + p;
}

// a thread's cell in the current pass: index, row, column; the next pass is
// 1024 cells on
struct TzCell {
  int m, r, c;
};
__device__ __forceinline__ void tz_next(TzCell& e, int nx, int dr, int dc) {
  e.m += kTzThreads;
  e.c += dc;
  e.r += dr;
  const bool wrap = e.c >= nx;
  e.c = wrap ? e.c - nx : e.c;
  e.r = wrap ? e.r + 1 : e.r;
}
}  // namespace

// Z^{n+1} = Z^{n-1} + F(Z^n) (Z^1 = Z^0 + F(Z^0)/2) with the Turkel-Zwas F,
// for every level of box order[blockIdx.x]; the arithmetic of k_fwd_tz
template <int K>
__global__ __launch_bounds__(kTzThreads) void k_fwd_tz_box(Dom<float> D, const double* __restrict__ x,
                                                           const int32_t* __restrict__ order, int p,
                                                           int q, float alpha, int nlat) {
  extern __shared__ float lds[];
  const int s = order[blockIdx.x];
  if (D.active && !D.active[s]) return;
  const SubDev S = D.subs[s];
  const int nx = S.nx, ny = S.ny, fx = nx + 2 * p, fy = ny + 2 * q;
  const int ncell = S.ncell, nring = S.nring;
  const int L = S.nlev - 1;
  const int tid = threadIdx.x;
  float* F = lds;                               // [fy][fx][3]: the level and its pad
  float* rt = lds + 3 * fy * fx;                // [ny][12]: row coefficients
  const float st = D.st, stg = D.stg, h0 = D.h0, al = alpha, one = 1.0f, half = 0.5f;
  const float itp = one / float(p), itq = one / float(q);
  const int64_t plane = ncell;
  float* Zb = D.traj + S.zoff;                  // level n at Zb + 3 n plane
  const float* ring = D.ring + S.ring_off;

  for (int r = tid; r < ny; r += kTzThreads) {
    const RowCoef<float> rc = D.rows[S.row0 + r];
    const RowCoef<float> rN = D.rows[tz_grow(S, r + q, nlat)];
    const RowCoef<float> rS = D.rows[tz_grow(S, r - q, nlat)];
    float* t = rt + kTzRowWords * r;
    t[0] = rc.a1; t[1] = rc.a2; t[2] = rc.a3; t[3] = rc.cf; t[4] = rc.ct;
    t[5] = rN.c; t[6] = rS.c; t[7] = rN.cf; t[8] = rN.ct; t[9] = rS.cf; t[10] = rS.ct;
  }
  // this thread's pad positions and their frame indices
  int padf[kTzRingMax];
#pragma unroll
  for (int j = 0; j < kTzRingMax; ++j) {
    const int k = tid + j * kTzThreads;
    padf[j] = k < nring ? tz_pad_frame(k, nx, ny, p, q) : -1;
  }
  // level 0 from the FP64 control, and its pad
  const double* xs = x + S.ctrl_off;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int m = tid + k * kTzThreads;
    if (m < ncell) {
      const int r = m / nx, c = m - r * nx;
      float* Fc = F + 3 * ((r + q) * fx + c + p);
      const float h = float(xs[m] - double(h0)), u = float(xs[ncell + m]), v = float(xs[2 * ncell + m]);
      Fc[0] = h; Fc[1] = u; Fc[2] = v;
      Zb[m] = h; Zb[plane + m] = u; Zb[2 * plane + m] = v;
    }
  }
#pragma unroll
  for (int j = 0; j < kTzRingMax; ++j) {
    if (padf[j] < 0) continue;
    const int k = tid + j * kTzThreads;
    float* Fp = F + 3 * padf[j];
    Fp[0] = ring[k]; Fp[1] = ring[nring + k]; Fp[2] = ring[2 * nring + k];
  }
  __syncthreads();

  const int dr = kTzThreads / nx, dc = kTzThreads - dr * nx;
  const TzCell e0 = {tid, tid / nx, tid - (tid / nx) * nx};
  // zr: this thread's cells of Z^{n-1}, the base of the leapfrog update
  float zr[3][K];
#pragma unroll
  for (int k = 0; k < K; ++k) zr[0][k] = zr[1][k] = zr[2][k] = 0.0f;
  for (int n = 0; n < L; ++n) {
    // pad of level n+1, fetched while this step computes
    float pv[kTzRingMax][3];
#pragma unroll
    for (int j = 0; j < kTzRingMax; ++j) {
      const int k = padf[j] < 0 ? 0 : tid + j * kTzThreads;
      const float* R1 = ring + int64_t(n + 1) * 3 * nring;
      pv[j][0] = R1[k]; pv[j][1] = R1[nring + k]; pv[j][2] = R1[2 * nring + k];
    }
    const bool euler = n == 0;
    float* Zn = Zb + int64_t(n + 1) * 3 * plane;
    // an opaque copy of the start cell: the per-pass positions are rebuilt
    // at every step instead of being hoisted (and spilled) out of the loop
    TzCell e = e0;
    asm volatile("" : "+v"(e.m), "+v"(e.r), "+v"(e.c));
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int m = e.m, r = e.r, c = e.c;
      if (k * kTzThreads < ncell && m < ncell) {
        const float* t = rt + kTzRowWords * r;
        const float a1 = t[0], a2 = t[1], a3 = t[2], cf = t[3], ct = t[4];
        const float cN = t[5], cS = t[6], cfN = t[7], ctN = t[8], cfS = t[9], ctS = t[10];
        const float* Fc = F + 3 * ((r + q) * fx + c + p);
        const int rq = 3 * q * fx, cp = 3 * p;
        const V3<float> C = {Fc[0], Fc[1], Fc[2]};
        const V3<float> E = {Fc[3], Fc[4], Fc[5]}, W = {Fc[-3], Fc[-2], Fc[-1]};
        const V3<float> N = {Fc[3 * fx], Fc[3 * fx + 1], Fc[3 * fx + 2]};
        const V3<float> Sv = {Fc[-3 * fx], Fc[-3 * fx + 1], Fc[-3 * fx + 2]};
        const V3<float> Ep = {Fc[cp], Fc[cp + 1], Fc[cp + 2]}, Wp = {Fc[-cp], Fc[-cp + 1], Fc[-cp + 2]};
        const V3<float> Nq = {Fc[rq], Fc[rq + 1], Fc[rq + 2]};
        const V3<float> Sq = {Fc[-rq], Fc[-rq + 1], Fc[-rq + 2]};
        const float ENu = Fc[rq + cp + 1], ENv = Fc[rq + cp + 2];
        const float WNu = Fc[rq - cp + 1], WNv = Fc[rq - cp + 2];
        const float ESu = Fc[-rq + cp + 1], ESv = Fc[-rq + cp + 2];
        const float WSu = Fc[-rq - cp + 1], WSv = Fc[-rq - cp + 2];
        const float hh = h0 + C.h;
        const float U = -a1 * C.u * (E.u - W.u) - st * C.v * (N.u - Sv.u) - a2 * itp * (Ep.h - Wp.h) +
                        ((one - al) * (cf + ct * C.u) * C.v + half * al * (cf + ct * Ep.u) * Ep.v +
                         half * al * (cf + ct * Wp.u) * Wp.v);
        const float V = -a1 * C.u * (E.v - W.v) - st * C.v * (N.v - Sv.v) - stg * itq * (Nq.h - Sq.h) -
                        ((one - al) * (cf + ct * C.u) * C.u + half * al * (cfN + ctN * Nq.u) * Nq.u +
                         half * al * (cfS + ctS * Sq.u) * Sq.u);
        const float Dl = ((one - al) * (Ep.u - Wp.u) + half * al * (ENu - WNu + ESu - WSu)) * itp;
        const float Dt = ((one - al) * (Nq.v * cN - Sq.v * cS) + half * al * (ENv * cN - ESv * cS) +
                          half * al * (WNv * cN - WSv * cS)) * itq;
        const float H = -a1 * (C.u * (E.h - W.h) + hh * Dl) - (st * C.v * (N.h - Sv.h) + a3 * hh * Dt);
        const float wgt = euler ? 0.5f : 1.0f;
        const float bh = euler ? C.h : zr[0][k], bu = euler ? C.u : zr[1][k], bv = euler ? C.v : zr[2][k];
        zr[0][k] = bh + wgt * H;
        zr[1][k] = bu + wgt * U;
        zr[2][k] = bv + wgt * V;
        Zn[m] = zr[0][k];
        Zn[plane + m] = zr[1][k];
        Zn[2 * plane + m] = zr[2][k];
      }
      // keep each pass's frame reads within its own iteration: hoisting them
      // ahead of the unrolled loop exhausts the register file
      __builtin_amdgcn_sched_barrier(0);
      tz_next(e, nx, dr, dc);
    }
    __syncthreads();                            // every read of level n done
    // level n+1 and its pad into the frame; level n into the registers
    e = e0;
    asm volatile("" : "+v"(e.m), "+v"(e.r), "+v"(e.c));
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int m = e.m, r = e.r, c = e.c;
      tz_next(e, nx, dr, dc);
      if (m < ncell) {
        float* Fc = F + 3 * ((r + q) * fx + c + p);
        const float th = Fc[0], tu = Fc[1], tv = Fc[2];
        Fc[0] = zr[0][k]; Fc[1] = zr[1][k]; Fc[2] = zr[2][k];
        zr[0][k] = th; zr[1][k] = tu; zr[2][k] = tv;
      }
    }
#pragma unroll
    for (int j = 0; j < kTzRingMax; ++j) {
      if (padf[j] < 0) continue;
      float* Fp = F + 3 * padf[j];
      Fp[0] = pv[j][0]; Fp[1] = pv[j][1]; Fp[2] = pv[j][2];
    }
    __syncthreads();
  }
}

size_t tz_box_lds_bytes(int nx, int ny, int p, int q) {
  return size_t(3) * (ny + 2 * q) * (nx + 2 * p) * sizeof(float) + size_t(kTzRowWords) * ny * sizeof(float);
}

bool tz_box_fits(int ncell, int nring, size_t lds_bytes) {
  return ncell <= kTzKMax * kTzThreads && nring <= kTzRingMax * kTzThreads &&
         lds_bytes <= size_t(160 * 1024 - 1024);
}

namespace {
template <int K>
hipError_t fwd_tz_box_k(const Dom<float>& D, const double* x, const int32_t* order, int nboxes,
                        size_t lds_bytes, int p, int q, double alpha, int nlat, hipStream_t st) {
  hipLaunchKernelGGL(k_fwd_tz_box<K>, dim3(nboxes), dim3(kTzThreads), lds_bytes, st, D, x, order, p,
                     q, float(alpha), nlat);
  return hipGetLastError();
}
}  // namespace

hipError_t prepare_fwd_tz_box() {
  const int bytes = 160 * 1024 - 1024;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fwd_tz_box<10>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fwd_tz_box<kTzKMax>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return e;
}

hipError_t launch_fwd_tz_box(const Dom<float>& D, const double* x, const int32_t* order, int nboxes,
                             size_t lds_bytes, int max_cells, int p, int q, double alpha, int nlat,
                             hipStream_t st) {
  if (max_cells <= 10 * kTzThreads)
    return fwd_tz_box_k<10>(D, x, order, nboxes, lds_bytes, p, q, alpha, nlat, st);
  return fwd_tz_box_k<kTzKMax>(D, x, order, nboxes, lds_bytes, p, q, alpha, nlat, st);
}

}  // namespace dd4dvar
