// Persistent per-box sweeps (FP32 state): one workgroup owns one box for its
// whole time interval and keeps the current level in LDS and the level
// before it in registers, so that a forward step touches HBM only to store
// the trajectory and to read the frozen halo ring, and an adjoint step only
// to read the stored state, the overlap targets and the ring.
// Same arithmetic as the step kernels of sweep.hip (restricted model,
// eq. restricted; discrete U, V, H of Sec. 7; leapfrog with a forward-Euler
// half step).
//
// LDS holds the level on a padded (ny+2) x (nx+2) grid, the three fields of
// a cell side by side ([cell][h, u, v]), so that one base address and
// immediate offsets reach a cell and its east and west neighbours.  The
// one-cell frame carries the halo: frozen ring values (signs applied), or,
// for a box spanning the circle, copies of the box's own cells across the
// seam or the pole (u, v negated across a pole).  The stencil then needs no
// branches.  Per-row coefficients sit in LDS as well.
//
// Thread t handles cells t + 1024 k, k = 0 .. K-1 (K passes, row-major), and
// tracks the row and column of its cell incrementally from pass to pass.
// These kernels need every level stored (no checkpoints): level n of a box
// sits at slot n of its state arena.
#include <type_traits>

#include "kernels.h"
#include "launch.h"
#include "stencil.h"

namespace dd4dvar {

using namespace stencil;

namespace {
constexpr int kBoxThreads = 1024;
constexpr int kBoxKMax = 11;              // passes: boxes of up to 11 x 1024 cells
// dynamic LDS limit (160 KB per workgroup less the static reduction buffer)
constexpr size_t kBoxLdsMax = 160 * 1024 - 1024;

// padded-frame index of ring position k of a box
__device__ __forceinline__ int frame_index(int k, int nx, int ny) {
  const int nxp = nx + 2;
  if (k < nx) return k + 1;                             // south row
  if (k < 2 * nx) return (ny + 1) * nxp + (k - nx) + 1;  // north row
  if (k < 2 * nx + ny) return (k - 2 * nx + 1) * nxp;    // west column
  return (k - 2 * nx - ny + 1) * nxp + nx + 1;           // east column
}

// copy the internal (wrapped) frame positions from the box interior; state
// copies carry the across-pole sign of u, v, adjoint copies are raw (the
// adjoint gather applies the sign itself)
__device__ __forceinline__ void fill_wraps(float* P, const int32_t* hsrc, const int32_t* hoff,
                                           const int32_t* hsgn, int nring, int nx, int ny,
                                           bool signed_copy) {
  const int nxp = nx + 2;
  for (int k = threadIdx.x; k < nring; k += kBoxThreads) {
    if (hsrc[k] >= 0) continue;
    const int p = 3 * frame_index(k, nx, ny);
    const int o = hoff[k], sr = o / nx, sc = o - sr * nx;
    const int q = 3 * ((sr + 1) * nxp + sc + 1);
    const float sg = signed_copy ? float(hsgn[k]) : 1.0f;
    P[p] = P[q];
    P[p + 1] = sg * P[q + 1];
    P[p + 2] = sg * P[q + 2];
  }
}

__device__ __forceinline__ void fill_rowtab(float* rowtab, const Dom<float>& D, const SubDev& S) {
  for (int r = threadIdx.x; r < S.ny; r += kBoxThreads) {
    const int j = S.row0 + r;
    const RowCoef<float> rc = D.rows[j];
    float* q = rowtab + 8 * r;
    q[0] = rc.a1; q[1] = rc.a2; q[2] = rc.a3; q[3] = rc.cf; q[4] = rc.ct; q[5] = rc.c;
    q[6] = D.cosx[j + 2];
    q[7] = D.cosx[j];
  }
}

// Raw buffer access: a 32-bit byte offset per lane plus a wave-uniform one,
// against a range-checked resource, so neighbour and field addresses cost no
// 64-bit arithmetic.  Word 3 of the resource is the gfx9-family raw format.
constexpr int kRsrcWord3 = 0x00020000;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, kRsrcWord3);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ V3<float> bload3(__amdgpu_buffer_rsrc_t r, int voff, int soff, int fstride) {
  return {bload(r, voff, soff), bload(r, voff, soff + fstride), bload(r, voff, soff + 2 * fstride)};
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, float v, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
}

// per-lane choice a (lanes set in mask) or b, as one v_cndmask: written out
// so that the compiler cannot turn the choice into a branch around the load
// of b, which would make it wait for the load of a first
__device__ __forceinline__ float pick(float a, float b, uint64_t mask) {
  float r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(b), "v"(a), "s"(mask));
  return r;
}
__device__ __forceinline__ V3<float> pick3(const V3<float>& a, const V3<float>& b, uint64_t mask) {
  return {pick(a.h, b.h, mask), pick(a.u, b.u, mask), pick(a.v, b.v, mask)};
}

__device__ __forceinline__ V3<float> lds3(const float* P, int i) {
  return {P[i], P[i + 1], P[i + 2]};
}

// value of ring position k of a box at one level: the frozen ring value, or
// for a position that wraps inside the box the box's own cell (u, v with the
// across-pole sign)
__device__ __forceinline__ V3<float> ring_value(const Dom<float>& D, const SubDev& S, int k,
                                                int level) {
  const int nring = S.nring;
  const int64_t plane = S.ncell;
  if (D.hsrc[S.hmap_off + k] >= 0) {
    const float* R = D.ring + S.ring_off + int64_t(level) * 3 * nring;
    return {R[k], R[nring + k], R[2 * nring + k]};
  }
  const float* Z = D.traj + S.zoff + int64_t(level) * 3 * plane;
  const int o = D.hoff[S.hmap_off + k];
  const float sg = float(D.hsign[S.hmap_off + k]);
  return {Z[o], sg * Z[plane + o], sg * Z[2 * plane + o]};
}

// a thread's cell in the current pass: index, row, column
struct Cell {
  int m, r, c;
};
__device__ __forceinline__ Cell first_cell(int nx) {
  const int t = threadIdx.x, r = t / nx;
  return {t, r, t - r * nx};
}
// next pass: 1024 cells on = dr rows and dc columns on
__device__ __forceinline__ void next_cell(Cell& q, int nx, int dr, int dc) {
  q.m += kBoxThreads;
  q.c += dc;
  q.r += dr;
  const bool wrap = q.c >= nx;
  q.c = wrap ? q.c - nx : q.c;
  q.r = wrap ? q.r + 1 : q.r;
}

// per-row coefficients a cell's adjoint gather needs
struct RowK {
  float a1, a2, cf, ct, cc, a3n, a3s;
};

// transposed Jacobian of the increments of a cell and of its four neighbours
// applied to lambda^{n+1} (l0 at the cell, kE .. kS at the neighbours), grouped
// by shared factors; C .. Sv is the state of level n at the cell and its
// neighbours, sn / ss the across-pole signs.  Returns (h, u, v).
__device__ __forceinline__ V3<float> gather_cell(const RowK& k, float st, float stg, float h0,
                                                 const V3<float>& C, const V3<float>& E,
                                                 const V3<float>& W, const V3<float>& N,
                                                 const V3<float>& Sv, const V3<float>& l0,
                                                 const V3<float>& kE, const V3<float>& kW,
                                                 const V3<float>& kN, const V3<float>& kS, float sn,
                                                 float ss) {
  const float a1 = k.a1, a2 = k.a2, cf = k.cf, ct = k.ct, cc = k.cc, a3n = k.a3n, a3s = k.a3s;
  const float hm = h0 + C.h;
  const float ctu = ct * C.u;
  const float dh = kE.h - kW.h;                       // east - west height adjoints
  const float q = kN.h * a3n - kS.h * a3s;            // north - south, with cos factors
  const float vkn = sn * N.v, vks = ss * Sv.v;
  float au = l0.u * (ct * C.v - a1 * (E.u - W.u)) + l0.v * (-a1 * (E.v - W.v) - cf - 2.0f * ctu);
  au += a1 * ((kE.u * E.u - kW.u * W.u) + dh * hm) + st * (kN.u * vkn - kS.u * vks);
  float av = l0.u * (cf + ctu - st * (N.u - Sv.u)) - l0.v * (st * (N.v - Sv.v));
  av += a1 * (kE.v * E.u - kW.v * W.u) + st * (kN.v * vkn - kS.v * vks) + (hm * cc) * q;
  const float ah = a2 * (kE.u - kW.u) + (a1 * C.u) * dh + stg * (sn * kN.v - ss * kS.v) + (C.v * cc) * q;
  return {ah, au, av};
}

__device__ __forceinline__ double block_sum_box(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBoxThreads / 64; ++i) r += sh[i];
  return r;
}
}  // namespace

// forward sweep of box s by the whole workgroup (K passes of 1024 cells);
// SPAN: some box of the launch spans the circle (wrapped frame positions)
template <int K, bool SPAN>
__device__ __forceinline__ void fwd_box_body(const Dom<float>& D, const double* __restrict__ x,
                                             int s, float* lds) {
  const SubDev S = D.subs[s];
  const int nx = S.nx, ny = S.ny, nxp = nx + 2, npad = (ny + 2) * nxp;
  const int ncell = S.ncell, nring = S.nring;
  const int L = S.nlev - 1;
  const int tid = threadIdx.x;
  float* P = lds;                          // [npad][3]: the level
  float* rowtab = lds + 3 * npad;          // [ny][8]: a1 a2 a3 cf ct c cN cS
  const float h0 = D.h0, st = D.st, stg = D.stg;
  const float* ring = D.ring + S.ring_off;
  const int32_t* hsrc = D.hsrc + S.hmap_off;
  const int32_t* hoff = D.hoff + S.hmap_off;
  const int32_t* hsgn = D.hsign + S.hmap_off;
  const bool wraps = SPAN && S.span != 0;
  const int fp = ncell * 4, lvb = 3 * ncell * 4;   // byte strides: field, level
  const __amdgpu_buffer_rsrc_t zrs = make_rsrc(D.traj + S.zoff, S.nlev * lvb);
  const int dr = kBoxThreads / nx, dc = kBoxThreads - dr * nx;
  const int n3 = 3 * nxp;                  // one padded row, in floats

  fill_rowtab(rowtab, D, S);
  // level 0 from the FP64 control
  const double* xs = x + S.ctrl_off;
  {
    Cell q = first_cell(nx);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (q.m < ncell) {
        const int p = 3 * ((q.r + 1) * nxp + q.c + 1);
        const float h = float(xs[q.m] - double(h0)), u = float(xs[ncell + q.m]),
                    v = float(xs[2 * ncell + q.m]);
        P[p] = h; P[p + 1] = u; P[p + 2] = v;
        bstore(zrs, h, q.m * 4, 0);
        bstore(zrs, u, q.m * 4, fp);
        bstore(zrs, v, q.m * 4, 2 * fp);
      }
      next_cell(q, nx, dr, dc);
    }
  }
  for (int k = tid; k < nring; k += kBoxThreads) {
    if (hsrc[k] < 0) continue;
    const int p = 3 * frame_index(k, nx, ny);
    P[p] = ring[k]; P[p + 1] = ring[nring + k]; P[p + 2] = ring[2 * nring + k];
  }
  __syncthreads();
  if (wraps) {
    fill_wraps(P, hsrc, hoff, hsgn, nring, nx, ny, true);
    __syncthreads();
  }

  // zr holds this thread's cells of Z^{n-1} on entry to step n >= 1 (the
  // level before the one in LDS), so the base of the leapfrog update never
  // comes back from memory; the new level replaces it in place and goes to
  // LDS, and the thread's cells of level n, kept in cz from the step's own
  // reads, become the next base (no second read of the frame).
  float zr[3][K], cz[3][K];
#pragma unroll
  for (int k = 0; k < K; ++k) zr[0][k] = zr[1][k] = zr[2][k] = cz[0][k] = cz[1][k] = cz[2][k] = 0.0f;
  const Cell q0 = first_cell(nx);
  // this thread's frozen ring position, if any (decided once: a load that a
  // branch waits on at every step would hold up the thread's first pass)
  const bool ring_pos = tid < nring && hsrc[tid] >= 0;
  for (int n = 0; n < L; ++n) {
    // frozen ring of level n+1, fetched while this step computes
    float rh = 0.f, ru = 0.f, rv = 0.f;
    if (ring_pos) {
      const float* R1 = ring + int64_t(n + 1) * 3 * nring;
      rh = R1[tid]; ru = R1[nring + tid]; rv = R1[2 * nring + tid];
    }
    const bool euler = n == 0;
    const int so = __builtin_amdgcn_readfirstlane((n + 1) * lvb);   // level n+1, field h
    // an opaque copy of the start cell: the per-pass positions are rebuilt
    // every step instead of being hoisted (and spilled) out of the time loop
    Cell q = q0;
    asm volatile("" : "+v"(q.m), "+v"(q.r), "+v"(q.c));
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (k * kBoxThreads < ncell) {                   // uniform
        // lanes past the box read a valid frame position and compute nothing
        const bool act = q.m < ncell;
        const int rr = act ? q.r : 0, cc = act ? q.c : 0;
        const float* rw = rowtab + 8 * rr;
        const float a1 = rw[0], a2 = rw[1], a3 = rw[2], cf = rw[3], ct = rw[4], cN = rw[6], cS = rw[7];
        const float* Pc = P + 3 * ((rr + 1) * nxp + cc + 1);
        const V3<float> C = lds3(Pc, 0), E = lds3(Pc, 3), W = lds3(Pc, -3);
        const V3<float> N = lds3(Pc, n3), Sv = lds3(Pc, -n3);
        cz[0][k] = C.h;
        cz[1][k] = C.u;
        cz[2][k] = C.v;
        if (act) {
          const float cor = cf + ct * C.u;
          const float U = -a1 * C.u * (E.u - W.u) - st * C.v * (N.u - Sv.u) - a2 * (E.h - W.h) + cor * C.v;
          const float V = -a1 * C.u * (E.v - W.v) - st * C.v * (N.v - Sv.v) - stg * (N.h - Sv.h) - cor * C.u;
          const float H = -a1 * (h0 * (E.u - W.u) + (E.h * E.u - W.h * W.u)) -
                          a3 * (h0 * (N.v * cN - Sv.v * cS) + (N.h * N.v * cN - Sv.h * Sv.v * cS));
          // Z^1 = Z^0 + F(Z^0)/2 (Euler start), else Z^{n+1} = Z^{n-1} + F(Z^n)
          if (euler) {
            zr[0][k] = C.h + 0.5f * H;
            zr[1][k] = C.u + 0.5f * U;
            zr[2][k] = C.v + 0.5f * V;
          } else {
            zr[0][k] += H;
            zr[1][k] += U;
            zr[2][k] += V;
          }
          bstore(zrs, zr[0][k], q.m * 4, so);
          bstore(zrs, zr[1][k], q.m * 4, so + fp);
          bstore(zrs, zr[2][k], q.m * 4, so + 2 * fp);
        }
      }
      // keep each pass's loads within its own iteration: hoisting them all
      // ahead of the unrolled loop exhausts the register file
      __builtin_amdgcn_sched_barrier(0);
      next_cell(q, nx, dr, dc);
    }
    __syncthreads();                                    // every read of level n done
    // level n+1 into LDS; level n (kept from the reads above) into the
    // registers, the base of the next step
    q = q0;
    asm volatile("" : "+v"(q.m), "+v"(q.r), "+v"(q.c));
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (q.m < ncell) {
        float* Pc = P + 3 * ((q.r + 1) * nxp + q.c + 1);
        Pc[0] = zr[0][k]; Pc[1] = zr[1][k]; Pc[2] = zr[2][k];
        zr[0][k] = cz[0][k]; zr[1][k] = cz[1][k]; zr[2][k] = cz[2][k];
      }
      next_cell(q, nx, dr, dc);
    }
    if (ring_pos) {
      const int p = 3 * frame_index(tid, nx, ny);
      P[p] = rh; P[p + 1] = ru; P[p + 2] = rv;
    }
    __syncthreads();
    if (wraps) {
      fill_wraps(P, hsrc, hoff, hsgn, nring, nx, ny, true);
      __syncthreads();
    }
  }
}

// Tangent-linear sweep of box s (the TLM step of Alg. 6, linearized about
// the stored trajectory; frozen ring unperturbed): the perturbation level
// dZ^n lives in the LDS frame (frozen ring entries zero, wrapped entries
// copies of the box's own cells with the across-pole sign) and dZ^{n-1} in
// registers, as the forward keeps Z^n and Z^{n-1}; the state Z^n comes from
// the stored trajectory through buffer loads issued a pass ahead, its
// out-of-box neighbours from the level's ring staged in LDS one level ahead
// (as in the adjoint); each new level dZ^{n+1} is written once.  Derivative
// of the increments of fwd_box_body, with the flux terms linearized as
// (h_ref + h) du + dh u.
template <int K, bool SPAN>
__device__ __forceinline__ void tlm_box_body(const Dom<float>& D, const double* __restrict__ dx,
                                             int s, float* lds) {
  const SubDev S = D.subs[s];
  const int nx = S.nx, ny = S.ny, nxp = nx + 2, npad = (ny + 2) * nxp;
  const int ncell = S.ncell, nring = S.nring;
  const int L = S.nlev - 1;
  const int tid = threadIdx.x;
  float* P = lds;                          // [npad][3]: dZ^n
  float* rowtab = lds + 3 * npad;          // [ny][8]
  float* zring = rowtab + 8 * ny;          // [2 levels][nring][3]: Z on the ring
  const int64_t plane = ncell;
  const int32_t* hsrc = D.hsrc + S.hmap_off;
  const int32_t* hoff = D.hoff + S.hmap_off;
  const int32_t* hsgn = D.hsign + S.hmap_off;
  const bool wraps = SPAN && S.span != 0;
  const float h0 = D.h0, st = D.st, stg = D.stg;
  const int fp = ncell * 4, nx4 = nx * 4, lvb = 3 * ncell * 4;   // byte strides
  const __amdgpu_buffer_rsrc_t zrs = make_rsrc(D.traj + S.zoff, S.nlev * lvb);
  const __amdgpu_buffer_rsrc_t drs = make_rsrc(D.dz + S.zoff, S.nlev * lvb);
  const int dr = kBoxThreads / nx, dc = kBoxThreads - dr * nx;
  const int n3 = 3 * nxp;

  fill_rowtab(rowtab, D, S);
  for (int i = tid; i < 3 * npad; i += kBoxThreads) P[i] = 0.0f;
  for (int k = tid; k < nring; k += kBoxThreads) {
    const V3<float> g = ring_value(D, S, k, 0);
    float* Zr = zring + 3 * k;
    Zr[0] = g.h; Zr[1] = g.u; Zr[2] = g.v;
  }
  __syncthreads();                         // frame cleared before the level-0 cells
  // level 0 = dx
  const double* dxs = dx + S.ctrl_off;
  {
    Cell q = first_cell(nx);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (q.m < ncell) {
        const int p = 3 * ((q.r + 1) * nxp + q.c + 1);
        const float h = float(dxs[q.m]), u = float(dxs[ncell + q.m]), v = float(dxs[2 * ncell + q.m]);
        P[p] = h; P[p + 1] = u; P[p + 2] = v;
        bstore(drs, h, q.m * 4, 0);
        bstore(drs, u, q.m * 4, fp);
        bstore(drs, v, q.m * 4, 2 * fp);
      }
      next_cell(q, nx, dr, dc);
    }
  }
  // this thread's ring position and its source for every level
  const bool ring_thread0 = tid < nring;
  bool rfrozen = true;
  int roff = 0;
  float rsg = 1.0f;
  if (ring_thread0) {
    rfrozen = hsrc[tid] >= 0;
    roff = rfrozen ? tid : hoff[tid];
    rsg = rfrozen ? 1.0f : float(hsgn[tid]);
  }
  __syncthreads();
  if (wraps) {
    fill_wraps(P, hsrc, hoff, hsgn, nring, nx, ny, true);
    __syncthreads();
  }

  float zr[3][K];                          // dZ^{n-1} of this thread's cells
#pragma unroll
  for (int k = 0; k < K; ++k) zr[0][k] = zr[1][k] = zr[2][k] = 0.0f;
  const Cell q0 = first_cell(nx);
  for (int n = 0; n < L; ++n) {
    const int so = __builtin_amdgcn_readfirstlane(n * lvb);        // Z^n
    const int sw = __builtin_amdgcn_readfirstlane((n + 1) * lvb);  // dZ^{n+1}
    const float* Zr = zring + (n & 1) * 3 * nring;
    // ring of level n+1, fetched now and staged after this level's reads
    V3<float> gnext = {0.f, 0.f, 0.f};
    if (ring_thread0) {
      const float* src = rfrozen ? D.ring + S.ring_off + int64_t(n + 1) * 3 * nring + roff
                                 : D.traj + S.zoff + int64_t(n + 1) * 3 * plane + roff;
      const int64_t fs = rfrozen ? int64_t(nring) : plane;
      gnext = {src[0], rsg * src[fs], rsg * src[2 * fs]};
    }
    const bool euler = n == 0;
    struct PassLoads {
      V3<float> C, E, W, N, Sv;
    };
    auto issue = [&](const Cell& cq, bool edge) {
      PassLoads Q;
      const int v0 = cq.m * 4;
      const bool e_in = cq.c + 1 < nx, w_in = cq.c > 0;
      const bool n_in = !edge || cq.r + 1 < ny, s_in = !edge || cq.r > 0;
      Q.C = bload3(zrs, v0, so, fp);
      Q.E = bload3(zrs, e_in ? v0 + 4 : v0, so, fp);
      Q.W = bload3(zrs, w_in ? v0 - 4 : v0, so, fp);
      Q.N = bload3(zrs, n_in ? v0 + nx4 : v0, so, fp);
      Q.Sv = bload3(zrs, s_in ? v0 - nx4 : v0, so, fp);
      return Q;
    };
    Cell q = q0;
    asm volatile("" : "+v"(q.m), "+v"(q.r), "+v"(q.c));
    PassLoads cur = issue(q, true);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const bool edge_rows = k == 0 || (k + 1) * kBoxThreads > ncell - nx;
      const Cell qc = q;
      next_cell(q, nx, dr, dc);
      // issued whether or not the next pass holds cells of this box (an
      // in-range read past the end is never used): a conditional issue would
      // first copy this pass's loads, waiting for them
      PassLoads nxt = cur;
      if (k + 1 < K) nxt = issue(q, (k + 2) * kBoxThreads > ncell - nx);
      __builtin_amdgcn_sched_barrier(0);
      if (k * kBoxThreads < ncell && qc.m < ncell) {
        const int m = qc.m, r = qc.r, c = qc.c;
        const bool e_in = c + 1 < nx, w_in = c > 0;
        const bool n_in = !edge_rows || r + 1 < ny, s_in = !edge_rows || r > 0;
        const float* rw = rowtab + 8 * r;
        const float a1 = rw[0], a2 = rw[1], a3 = rw[2], cf = rw[3], ct = rw[4], cN = rw[6], cS = rw[7];
        const V3<float> C = cur.C;
        const V3<float> rE = lds3(Zr, e_in ? 0 : 3 * (2 * nx + ny + r));
        const V3<float> rW = lds3(Zr, w_in ? 0 : 3 * (2 * nx + r));
        const V3<float> E = pick3(cur.E, rE, __builtin_amdgcn_ballot_w64(e_in));
        const V3<float> W = pick3(cur.W, rW, __builtin_amdgcn_ballot_w64(w_in));
        V3<float> N = cur.N, Sv = cur.Sv;
        if (edge_rows) {
          N = pick3(N, lds3(Zr, n_in ? 0 : 3 * (nx + c)), __builtin_amdgcn_ballot_w64(n_in));
          Sv = pick3(Sv, lds3(Zr, s_in ? 0 : 3 * c), __builtin_amdgcn_ballot_w64(s_in));
        }
        const float* Pc = P + 3 * ((r + 1) * nxp + c + 1);
        const V3<float> dC = lds3(Pc, 0), dE = lds3(Pc, 3), dW = lds3(Pc, -3);
        const V3<float> dN = lds3(Pc, n3), dS = lds3(Pc, -n3);
        const float cor = cf + ct * C.u;
        const float dU = -a1 * (dC.u * (E.u - W.u) + C.u * (dE.u - dW.u)) -
                         st * (dC.v * (N.u - Sv.u) + C.v * (dN.u - dS.u)) - a2 * (dE.h - dW.h) +
                         (cor * dC.v + ct * dC.u * C.v);
        const float dV = -a1 * (dC.u * (E.v - W.v) + C.u * (dE.v - dW.v)) -
                         st * (dC.v * (N.v - Sv.v) + C.v * (dN.v - dS.v)) - stg * (dN.h - dS.h) -
                         (cor * dC.u + ct * dC.u * C.u);
        const float dH = -a1 * (((h0 + E.h) * dE.u + dE.h * E.u) - ((h0 + W.h) * dW.u + dW.h * W.u)) -
                         a3 * (((h0 + N.h) * dN.v + dN.h * N.v) * cN -
                               ((h0 + Sv.h) * dS.v + dS.h * Sv.v) * cS);
        if (euler) {
          zr[0][k] = dC.h + 0.5f * dH;
          zr[1][k] = dC.u + 0.5f * dU;
          zr[2][k] = dC.v + 0.5f * dV;
        } else {
          zr[0][k] += dH;
          zr[1][k] += dU;
          zr[2][k] += dV;
        }
        bstore(drs, zr[0][k], m * 4, sw);
        bstore(drs, zr[1][k], m * 4, sw + fp);
        bstore(drs, zr[2][k], m * 4, sw + 2 * fp);
      }
      __builtin_amdgcn_sched_barrier(0);
      cur = nxt;
    }
    __syncthreads();                                    // every read of dZ^n and the ring done
    // dZ^{n+1} into LDS; dZ^n into the registers (base of the next step)
    q = q0;
    asm volatile("" : "+v"(q.m), "+v"(q.r), "+v"(q.c));
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (q.m < ncell) {
        float* Pc = P + 3 * ((q.r + 1) * nxp + q.c + 1);
        const float th = Pc[0], tu = Pc[1], tv = Pc[2];
        Pc[0] = zr[0][k]; Pc[1] = zr[1][k]; Pc[2] = zr[2][k];
        zr[0][k] = th; zr[1][k] = tu; zr[2][k] = tv;
      }
      next_cell(q, nx, dr, dc);
    }
    if (ring_thread0) {
      float* Zq = zring + ((n + 1) & 1) * 3 * nring + 3 * tid;
      Zq[0] = gnext.h; Zq[1] = gnext.u; Zq[2] = gnext.v;
    }
    __syncthreads();
    if (wraps) {
      fill_wraps(P, hsrc, hoff, hsgn, nring, nx, ny, true);
      __syncthreads();
    }
  }
}

// Persistent adjoint sweep: lambda^{n+1} of the box lives in LDS on the
// padded grid (frozen ring entries of the frame stay zero: those increments
// are not part of the local model; wrapped entries hold raw copies), and
// each thread keeps its own cells of lambda^{n+2} in registers, where
// lambda^n replaces it; after the level the register and LDS copies are
// swapped.  Only Z^n, the overlap targets and the ring come from global
// memory: Z^n and the targets through buffer loads with clamped offsets, and
// neighbours outside the box from a copy of the level's ring (frozen values
// or wrapped cells, signs applied) staged in LDS one level ahead.  Only the
// passes that hold the box's first or last row look beyond it to the south
// or north.  Gather form and forcing as in k_adj (sweep.hip).
// MODE 0: cost forcing, gradient + J out; 1: caller forcing, adjoint out;
// 2: cost forcing, adjoint out; 3: Gauss-Newton forcing (the observation and
// overlap weights applied to the tangent-linear trajectory), adjoint out.
template <int K, int MODE, bool SPAN>
__device__ __forceinline__ void adj_box_body(const Dom<float>& D, const double* __restrict__ x,
                                             const double* __restrict__ xb,
                                             const double* __restrict__ forcing,
                                             double* __restrict__ out, int s, float* lds,
                                             double* red) {
  const SubDev S = D.subs[s];
  const int nx = S.nx, ny = S.ny, nxp = nx + 2, npad = (ny + 2) * nxp;
  const int ncell = S.ncell, nring = S.nring;
  const int L = S.nlev - 1;
  const int tid = threadIdx.x;
  float* Lm = lds;                         // [npad][3]: lambda^{n+1}
  float* rowtab = lds + 3 * npad;          // [ny][8]
  float* zring = rowtab + 8 * ny;          // [2 levels][nring][3]: state on the ring
  uint8_t* covl = reinterpret_cast<uint8_t*>(zring + 6 * nring);   // [ny*nx] coverage
  // per level: intervals covering it, and where the box's observation
  // entries of the level start ([nlev + 1]: level n's are lvl_ob[n] ..
  // lvl_ob[n + 1] - 1, one contiguous range of the bins)
  int* lvl_tc = reinterpret_cast<int*>(covl + ((ncell + 3) & ~3));
  int* lvl_ob = lvl_tc + S.nlev;
  const int64_t plane = ncell;
  const int32_t* hsrc = D.hsrc + S.hmap_off;
  const int32_t* hoff = D.hoff + S.hmap_off;
  const int32_t* hsgn = D.hsign + S.hmap_off;
  const bool wraps = SPAN && S.span != 0;
  const float st = D.st, stg = D.stg;
  const int fp = ncell * 4, nx4 = nx * 4, lvb = 3 * ncell * 4;   // byte strides
  const __amdgpu_buffer_rsrc_t zrs = make_rsrc(D.traj + S.zoff, S.nlev * lvb);
  // overlap targets, or (MODE 3) the tangent-linear trajectory: both read
  // only where the cell is covered by another box
  const __amdgpu_buffer_rsrc_t trs =
      make_rsrc(MODE == 3 ? D.dz + S.zoff : D.targ + S.traj_off, S.nlev * lvb);
  const float mu_f = float(D.mu);
  const float ib_h = float(D.isb2[0]), ib_u = float(D.isb2[1]), ib_v = float(D.isb2[2]);
  const int dr = kBoxThreads / nx, dc = kBoxThreads - dr * nx;
  const int n3 = 3 * nxp;

  fill_rowtab(rowtab, D, S);
  for (int i = tid; i < 3 * npad; i += kBoxThreads) Lm[i] = 0.0f;   // lambda^{L+1} = 0
  for (int k = tid; k < nring; k += kBoxThreads) {
    const V3<float> g = ring_value(D, S, k, L);
    float* Zr = zring + (L & 1) * 3 * nring + 3 * k;
    Zr[0] = g.h; Zr[1] = g.u; Zr[2] = g.v;
  }
  // coverage counts (the same at every level), kept in LDS so that the
  // target loads wait on an LDS read only
  for (int i = tid; i < ncell; i += kBoxThreads) covl[i] = D.cover[S.cell_off + i];
  // per-level tables, so that no level waits on a global load at its start
  // or before its barrier
  for (int n = tid; n <= S.nlev; n += kBoxThreads) {
    if (n < S.nlev) lvl_tc[n] = (MODE != 1) ? D.tcount[S.lev0 + n] : 0;
    lvl_ob[n] = (MODE != 1) ? D.obs_ptr[obs_key(S.tile0, S.ntile, D.maxlev, 0, n)] : 0;
  }
  // this thread's ring position: the source of its value at every level
  // (frozen ring entry, or the box's own cell with the across-pole sign)
  const bool ring_thread0 = tid < nring;
  bool rfrozen = true;
  int roff = 0;
  float rsg = 1.0f;
  if (ring_thread0) {
    rfrozen = hsrc[tid] >= 0;
    roff = rfrozen ? tid : hoff[tid];
    rsg = rfrozen ? 1.0f : float(hsgn[tid]);
  }
  __syncthreads();
  double jloc = 0.0;
  // this thread's cells of lambda^{n+2} (zero above the window)
  float ln[3][K];
#pragma unroll
  for (int k = 0; k < K; ++k) ln[0][k] = ln[1][k] = ln[2][k] = 0.0f;
  const Cell q0 = first_cell(nx);

  for (int n = L; n >= 0; --n) {
    const float* Z = D.traj + S.zoff + int64_t(n) * 3 * plane;
    // level n, field h (wave-uniform: kept in a scalar register, as the
    // buffer loads need it there)
    const int so = __builtin_amdgcn_readfirstlane(n * lvb);
    const float* Zr = zring + (n & 1) * 3 * nring;
    const int tcount = lvl_tc[n];
    // ring of level n-1, fetched now and staged after this level's reads
    V3<float> gnext = {0.f, 0.f, 0.f};
    const bool ring_thread = ring_thread0 && n > 0;
    if (ring_thread) {
      const float* src = rfrozen ? D.ring + S.ring_off + int64_t(n - 1) * 3 * nring + roff
                                 : D.traj + S.zoff + int64_t(n - 1) * 3 * plane + roff;
      const int64_t fs = rfrozen ? int64_t(nring) : plane;
      gnext = {src[0], rsg * src[fs], rsg * src[2 * fs]};
    }
    // Global loads of one pass (the state of level n at the cell and at its
    // neighbours inside the box, offsets clamped to the cell itself at the
    // box edge, and the overlap target), issued one pass ahead of their use
    // so that their latency overlaps the arithmetic of the pass before.
    // Loads for cells past the box end stay inside the range-checked buffer
    // (or read as zero) and are never used.
    struct PassLoads {
      V3<float> C, E, W, N, Sv, tg;
      int Kc;
    };
    auto issue = [&](const Cell& cq, bool edge) {
      PassLoads L;
      const int v0 = cq.m * 4;
      const bool e_in = cq.c + 1 < nx, w_in = cq.c > 0;
      const bool n_in = !edge || cq.r + 1 < ny, s_in = !edge || cq.r > 0;
      L.Kc = 0;
      L.tg = {0.f, 0.f, 0.f};
      if (MODE != 1) {
        L.Kc = int(covl[cq.m < ncell ? cq.m : ncell - 1]) * tcount - 1;
        L.tg = bload3(trs, L.Kc > 0 ? v0 : 0, so, fp);
      }
      L.C = bload3(zrs, v0, so, fp);
      L.E = bload3(zrs, e_in ? v0 + 4 : v0, so, fp);
      L.W = bload3(zrs, w_in ? v0 - 4 : v0, so, fp);
      L.N = bload3(zrs, n_in ? v0 + nx4 : v0, so, fp);
      L.Sv = bload3(zrs, s_in ? v0 - nx4 : v0, so, fp);
      return L;
    };
    // opaque per-step copy of the start cell (see the forward)
    Cell q = q0;
    asm volatile("" : "+v"(q.m), "+v"(q.r), "+v"(q.c));
    PassLoads cur = issue(q, true);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      // passes holding the box's first or last row (wave-uniform)
      const bool edge_rows = k == 0 || (k + 1) * kBoxThreads > ncell - nx;
      const Cell qc = q;
      next_cell(q, nx, dr, dc);
      PassLoads nxt = cur;
      if (k + 1 < K && (k + 1) * kBoxThreads < ncell)
        nxt = issue(q, (k + 2) * kBoxThreads > ncell - nx);
      // the next pass's loads are in flight before this pass computes
      __builtin_amdgcn_sched_barrier(0);
      if (k * kBoxThreads < ncell && qc.m < ncell) {
        const int m = qc.m, r = qc.r, c = qc.c;
        const bool e_in = c + 1 < nx, w_in = c > 0;
        const bool n_in = !edge_rows || r + 1 < ny, s_in = !edge_rows || r > 0;
        const float* rw = rowtab + 8 * r;
        const float a1 = rw[0], a2 = rw[1], cf = rw[3], ct = rw[4], cc = rw[5];
        const float a3n = rowtab[8 * (n_in ? r + 1 : r) + 2];
        const float a3s = rowtab[8 * (s_in ? r - 1 : r) + 2];
        const int Kc = cur.Kc;
        const V3<float> tg = cur.tg, C = cur.C;
        V3<float> E = cur.E, W = cur.W, N = cur.N, Sv = cur.Sv;
        // the caller's forcing (adjoint_integrate)
        float fh = 0.f, fu = 0.f, fv = 0.f;
        if (MODE == 1) {
          const double* Fz = forcing + S.traj_off + int64_t(n) * 3 * plane;
          fh = float(Fz[m]);
          fu = float(Fz[plane + m]);
          fv = float(Fz[2 * plane + m]);
        }
        // neighbours outside the box, from the staged ring (every lane reads
        // a valid position and keeps it only at the edge)
        const int iE = e_in ? 0 : 3 * (2 * nx + ny + r), iW = w_in ? 0 : 3 * (2 * nx + r);
        const V3<float> rE = lds3(Zr, iE), rW = lds3(Zr, iW);
        V3<float> rN = {0.f, 0.f, 0.f}, rS = {0.f, 0.f, 0.f};
        if (edge_rows) {
          rN = lds3(Zr, n_in ? 0 : 3 * (nx + c));
          rS = lds3(Zr, s_in ? 0 : 3 * c);
        }
        E = pick3(E, rE, __builtin_amdgcn_ballot_w64(e_in));
        W = pick3(W, rW, __builtin_amdgcn_ballot_w64(w_in));
        if (edge_rows) {
          N = pick3(N, rN, __builtin_amdgcn_ballot_w64(n_in));
          Sv = pick3(Sv, rS, __builtin_amdgcn_ballot_w64(s_in));
        }
        // across a pole (boxes spanning the circle) the adjoint of a wrapped
        // neighbour carries the sign of u, v
        const float sn = (SPAN && !n_in && S.pole_n) ? -1.0f : 1.0f;
        const float ss = (SPAN && !s_in && S.pole_s) ? -1.0f : 1.0f;
        const V3<float> l2 = {ln[0][k], ln[1][k], ln[2][k]};
        // lambda^{n+1} from LDS (zero in frozen frame entries)
        const float* Lc = Lm + 3 * ((r + 1) * nxp + c + 1);
        const V3<float> l0 = lds3(Lc, 0), kE = lds3(Lc, 3), kW = lds3(Lc, -3);
        const V3<float> kN = lds3(Lc, n3), kS = lds3(Lc, -n3);
        const V3<float> gth = gather_cell({a1, a2, cf, ct, cc, a3n, a3s}, st, stg, D.h0, C, E, W, N,
                                          Sv, l0, kE, kW, kN, kS, sn, ss);
        float ah = gth.h, au = gth.u, av = gth.v;
        if (n == 0) {
          au = l0.u + 0.5f * au;
          av = l0.v + 0.5f * av;
          ah = l0.h + 0.5f * ah;
        }
        if (MODE != 1) {
          // overlap residual (the FP32 difference is the correctly rounded
          // exact one), its forcing in FP32 like the adjoint state, and the
          // cell's term of J accumulated in FP64
          const float eh = MODE == 3 ? tg.h : C.h - tg.h;
          const float eu = MODE == 3 ? tg.u : C.u - tg.u;
          const float ev = MODE == 3 ? tg.v : C.v - tg.v;
          const float mk = mu_f * float(Kc);
          fh = mk * ib_h * eh;
          fu = mk * ib_u * eu;
          fv = mk * ib_v * ev;
          if (MODE != 3)
            jloc += 0.5 * double(mk) * double(ib_h * eh * eh + ib_u * eu * eu + ib_v * ev * ev);
        }
        const float bh = fh + ah + l2.h;
        const float bu = fu + au + l2.u;
        const float bv = fv + av + l2.v;
        if (n > 0) {
          ln[0][k] = bh;
          ln[1][k] = bu;
          ln[2][k] = bv;
        } else {
          const int64_t o = S.ctrl_off + m;
          if (MODE == 0) {
            const double wb = D.weight_mode ? 1.0 : 1.0 / double(covl[m]);
            const double dh = x[o] - xb[o];
            const double du = x[o + plane] - xb[o + plane];
            const double dv = x[o + 2 * plane] - xb[o + 2 * plane];
            const double gh = wb * dh * D.isb2[0] + double(bh);
            const double gu = wb * du * D.isb2[1] + double(bu);
            const double gv = wb * dv * D.isb2[2] + double(bv);
            out[o] = gh;
            out[o + plane] = gu;
            out[o + 2 * plane] = gv;
            flag_nonfinite(D.nonfinite, !(isfinite(gh) && isfinite(gu) && isfinite(gv)));
            jloc += 0.5 * wb * (dh * dh * D.isb2[0] + du * du * D.isb2[1] + dv * dv * D.isb2[2]);
          } else {
            out[o] = double(bh);
            out[o + plane] = double(bu);
            out[o + 2 * plane] = double(bv);
            flag_nonfinite(D.nonfinite, !(isfinite(bh) && isfinite(bu) && isfinite(bv)));
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      cur = nxt;
    }
    // observations of this box at level n
    const int ob0 = lvl_ob[n], ob1 = lvl_ob[n + 1];
    const bool any_obs = MODE != 1 && ob1 > ob0;
    __syncthreads();                                   // all reads of lambda^{n+1} done
    if (ring_thread) {
      float* Zq = zring + ((n - 1) & 1) * 3 * nring + 3 * tid;
      Zq[0] = gnext.h; Zq[1] = gnext.u; Zq[2] = gnext.v;
    }
    if (n > 0) {
      // lambda^n into LDS; lambda^{n+1} into the registers (the lambda^{n+2}
      // of the next level)
      q = q0;
      asm volatile("" : "+v"(q.m), "+v"(q.r), "+v"(q.c));
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (q.m < ncell) {
          float* Lc = Lm + 3 * ((q.r + 1) * nxp + q.c + 1);
          const float th = Lc[0], tu = Lc[1], tv = Lc[2];
          Lc[0] = ln[0][k];
          Lc[1] = ln[1][k];
          Lc[2] = ln[2][k];
          ln[0][k] = th;
          ln[1][k] = tu;
          ln[2][k] = tv;
        }
        next_cell(q, nx, dr, dc);
      }
    }
    if (MODE != 1 && any_obs) {
      __syncthreads();                                   // lambda^n (or the gradient) complete
      // the level's entries of every tile of the box in one range; a cell
      // and field occur at most once per level (duplicate observations are
      // rejected), so the updates of the frame never collide
      for (int o = ob0 + tid; o < ob1; o += kBoxThreads) {
        const int code = D.obs_code[o];
        const int loc = code >> 2, f = code & 3;
        const double rr = MODE == 3 ? double(D.dz[S.zoff + int64_t(n) * 3 * plane + f * plane + loc])
                                    : double(Z[f * plane + loc]) - D.obs_val[o];
        const double qo = D.obs_q[o];
        if (MODE != 3) jloc += 0.5 * qo * rr * rr;
        if (n > 0) {
          const int lr = loc / nx, lc = loc - lr * nx;
          float* Lf = Lm + 3 * ((lr + 1) * nxp + lc + 1) + f;
          *Lf = float(double(*Lf) + qo * rr);
        } else {
          out[S.ctrl_off + f * plane + loc] += qo * rr;
        }
      }
    }
    __syncthreads();
    if (wraps && n > 0) {
      fill_wraps(Lm, hsrc, hoff, hsgn, nring, nx, ny, false);
      __syncthreads();
    }
  }
  if (MODE == 0 || MODE == 2) {
    // the box total goes to its first tile slot, the others are cleared, so
    // the per-subdomain reduction of the step path applies unchanged
    const double tot = block_sum_box(jloc, red);
    for (int t = tid + 1; t < S.ntile; t += kBoxThreads) D.jpart[S.tile0 + t] = 0.0;
    if (tid == 0) D.jpart[S.tile0] = tot;
  }
}

template <int K, bool SPAN>
__global__ __launch_bounds__(kBoxThreads) void k_fwd_box(Dom<float> D, const double* __restrict__ x,
                                                         const int32_t* __restrict__ order) {
  extern __shared__ float lds[];
  const int s = order[blockIdx.x];
  if (D.active && !D.active[s]) return;
  fwd_box_body<K, SPAN>(D, x, s, lds);
}

// Persistent adjoint sweep with column strips: thread t owns column
// c = t mod nx of the rows g R .. g R + R - 1 of its strip g = t div nx
// (G = 1024 div nx strips side by side, R = ceil(ny / G) <= K rows each) and
// walks them one row per pass.  The state of row r+1, loaded for the north
// neighbour of row r, is the centre of the next pass and the south
// neighbour of the one after, and the same holds for lambda^{n+1} in LDS, so
// a cell costs 10 buffer loads (its north state, east and west u, v, the
// overlap target) instead of 14 and 9 LDS reads of lambda instead of 15; a
// thread's column and its east/west edge masks are fixed for the whole
// sweep.  Waves none of whose lanes has a row left skip the loads of the
// remaining passes.  Arithmetic, forcing, ring staging, observations and
// outputs as in adj_box_body.
template <int K, int MODE, bool SPAN>
__device__ __forceinline__ void adj_strip_body(const Dom<float>& D, const double* __restrict__ x,
                                               const double* __restrict__ xb,
                                               const double* __restrict__ forcing,
                                               double* __restrict__ out, int s, float* lds,
                                               double* red) {
  const SubDev S = D.subs[s];
  const int nx = S.nx, ny = S.ny, nxp = nx + 2, npad = (ny + 2) * nxp;
  const int ncell = S.ncell, nring = S.nring;
  const int L = S.nlev - 1;
  const int tid = threadIdx.x;
  float* Lm = lds;                         // [npad][3]: lambda^{n+1}
  float* rowtab = lds + 3 * npad;          // [ny][8], see below
  float* zring = rowtab + 8 * ny;          // [2 levels][nring][3]: state on the ring
  uint8_t* covl = reinterpret_cast<uint8_t*>(zring + 6 * nring);   // [ny*nx] coverage
  int* lvl_tc = reinterpret_cast<int*>(covl + ((ncell + 3) & ~3));
  int* lvl_ob = lvl_tc + S.nlev;           // [nlev + 1], as in the box mapping
  const int64_t plane = ncell;
  const int32_t* hsrc = D.hsrc + S.hmap_off;
  const int32_t* hoff = D.hoff + S.hmap_off;
  const int32_t* hsgn = D.hsign + S.hmap_off;
  const bool wraps = SPAN && S.span != 0;
  const float st = D.st, stg = D.stg;
  const int fp = ncell * 4, nx4 = nx * 4, lvb = 3 * ncell * 4;   // byte strides
  const __amdgpu_buffer_rsrc_t zrs = make_rsrc(D.traj + S.zoff, S.nlev * lvb);
  const __amdgpu_buffer_rsrc_t trs =
      make_rsrc(MODE == 3 ? D.dz + S.zoff : D.targ + S.traj_off, S.nlev * lvb);
  const float mu_f = float(D.mu);
  const float ib_h = float(D.isb2[0]), ib_u = float(D.isb2[1]), ib_v = float(D.isb2[2]);
  const int n3 = 3 * nxp;
  // this thread's strip
  const int G = kBoxThreads / nx;
  const int R = (ny + G - 1) / G;
  const int c = tid % nx, g = tid / nx;
  const int r0 = g * R;
  // rows this thread owns (none beyond the last strip or past the box end)
  const int nrows = g < G ? max(0, min(R, ny - r0)) : 0;
  // LDS addressing stays on the thread's own rows (a row of the box for the
  // threads without rows), so every frame read is inside the frame
  const int ra = nrows > 0 ? r0 : ny - 1;
  const int kl = nrows > 0 ? nrows - 1 : 0;
  const bool w_in = c > 0, e_in = c + 1 < nx;
  const uint64_t mw = __builtin_amdgcn_ballot_w64(w_in), me = __builtin_amdgcn_ballot_w64(e_in);

  // per-row coefficients of the gather: a1, a2, a3, cf, ct, c, and a3 of the
  // rows the north and south terms take (the row itself at the box edge)
  for (int r = tid; r < ny; r += kBoxThreads) {
    const int j = S.row0 + r;
    const RowCoef<float> rc = D.rows[j];
    float* q = rowtab + 8 * r;
    q[0] = rc.a1; q[1] = rc.a2; q[2] = rc.a3; q[3] = rc.cf; q[4] = rc.ct; q[5] = rc.c;
    q[6] = D.rows[r + 1 < ny ? j + 1 : j].a3;
    q[7] = D.rows[r > 0 ? j - 1 : j].a3;
  }
  for (int i = tid; i < 3 * npad; i += kBoxThreads) Lm[i] = 0.0f;   // lambda^{L+1} = 0
  for (int k = tid; k < nring; k += kBoxThreads) {
    const V3<float> gv = ring_value(D, S, k, L);
    float* Zr = zring + (L & 1) * 3 * nring + 3 * k;
    Zr[0] = gv.h; Zr[1] = gv.u; Zr[2] = gv.v;
  }
  for (int i = tid; i < ncell; i += kBoxThreads) covl[i] = D.cover[S.cell_off + i];
  for (int n = tid; n <= S.nlev; n += kBoxThreads) {
    if (n < S.nlev) lvl_tc[n] = (MODE != 1) ? D.tcount[S.lev0 + n] : 0;
    lvl_ob[n] = (MODE != 1) ? D.obs_ptr[obs_key(S.tile0, S.ntile, D.maxlev, 0, n)] : 0;
  }
  const bool ring_thread0 = tid < nring;
  bool rfrozen = true;
  int roff = 0;
  float rsg = 1.0f;
  if (ring_thread0) {
    rfrozen = hsrc[tid] >= 0;
    roff = rfrozen ? tid : hoff[tid];
    rsg = rfrozen ? 1.0f : float(hsgn[tid]);
  }
  __syncthreads();
  double jloc = 0.0;
  float ln[3][K];                          // lambda^{n+2} of rows r0 .. r0+K-1
#pragma unroll
  for (int k = 0; k < K; ++k) ln[0][k] = ln[1][k] = ln[2][k] = 0.0f;
  // byte offset of (r0, c) and LDS frame index of (ra, c)
  const int v00 = (r0 * nx + c) * 4, f00 = 3 * ((ra + 1) * nxp + c + 1);
  // staged ring positions (float index) of the thread's column to the south
  // (north: nx positions on) and of its first row to the west (east: ny
  // positions on).  Every lane reads them for its rows inside the box, all
  // valid positions; lanes inside the box discard the values.
  const int zS = 3 * c, zW = 3 * (2 * nx + r0);

  // one level of the sweep; the first level of the window (n = 0: the
  // adjoint of the forward start's half step, and the gradient output) is a
  // copy of its own, so that the passes of the other levels test nothing
  auto level = [&](const int n, auto last_tag) {
    constexpr bool LAST = decltype(last_tag)::value;
    const float* Z = D.traj + S.zoff + int64_t(n) * 3 * plane;
    const int so = __builtin_amdgcn_readfirstlane(n * lvb);
    const float* Zr = zring + (n & 1) * 3 * nring;
    // overlap weight mu K of a cell with coverage byte cov: K = cov tcount - 1
    // other boxes hold it at this level (exact in FP32, as K is an integer
    // below 2^24)
    const float tcf = float(lvl_tc[n]);
    V3<float> gnext = {0.f, 0.f, 0.f};
    const bool ring_thread = ring_thread0 && !LAST;
    if (ring_thread) {
      const float* src = rfrozen ? D.ring + S.ring_off + int64_t(n - 1) * 3 * nring + roff
                                 : D.traj + S.zoff + int64_t(n - 1) * 3 * plane + roff;
      const int64_t fs = rfrozen ? int64_t(nring) : plane;
      gnext = {src[0], rsg * src[fs], rsg * src[2 * fs]};
    }
    // loads of the pass for the row at byte offset v: the state of the row
    // to the north, east and west u, v, and the overlap target where covered.
    // The neighbour offsets ride on the scalar offset (one row on, one cell
    // either way); a neighbour outside the box (north of the last row, east
    // of the last column, west of the first) is read at the position those
    // offsets reach inside the arena and replaced by the staged ring.  Rows
    // past the box are read the same way and discarded.
    struct RowLoads {
      V3<float> Cn, tg;
      float Eu, Ev, Wu, Wv, mk;
    };
    auto issue = [&](int v) {
      RowLoads Q;
      Q.Cn = bload3(zrs, v, so + nx4, fp);
      Q.Eu = bload(zrs, v, so + fp + 4);
      Q.Ev = bload(zrs, v, so + 2 * fp + 4);
      Q.Wu = bload(zrs, v, so + fp - 4);
      Q.Wv = bload(zrs, v, so + 2 * fp - 4);
      Q.mk = 0.f;
      Q.tg = {0.f, 0.f, 0.f};
      if (MODE != 1) {
        const int mc = v >> 2;
        Q.mk = mu_f * __builtin_fmaf(float(covl[mc < ncell ? mc : ncell - 1]), tcf, -1.0f);
        Q.tg = bload3(trs, Q.mk > 0.f ? v : 0, so, fp);
      }
      return Q;
    };
    // opaque per-level copies of the thread's start offsets and row range:
    // every per-pass offset is rebuilt from them at each level instead of
    // being hoisted out of the level loop (which would spill)
    int v0 = v00, fb = f00, rb = r0, nr = nrows, kk = kl;
    asm volatile("" : "+v"(v0), "+v"(fb), "+v"(rb), "+v"(nr), "+v"(kk));
    // rows r0-1 and r0 (row -1: the cell itself, replaced from the ring)
    V3<float> Cs = bload3(zrs, rb > 0 ? v0 - nx4 : v0, so, fp);
    V3<float> Cc = bload3(zrs, v0, so, fp);
    const float* L0 = Lm + fb;
    V3<float> lp = lds3(L0, -n3), lc = lds3(L0, 0);   // lambda^{n+1} of rows r0-1, r0
    // waves none of whose lanes has a row left issue no loads
    RowLoads cur{};
    if (__builtin_amdgcn_ballot_w64(0 < nr) != 0) cur = issue(v0);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int r = rb + k;
      const int v = v0 + k * nx4;
      // (zero in a wave without rows left: never used there)
      RowLoads nxt{};
      if (k + 1 < K && __builtin_amdgcn_ballot_w64(k + 1 < nr) != 0) nxt = issue(v + nx4);
      __builtin_amdgcn_sched_barrier(0);
      const float* Lc = L0 + (k < kk ? k : kk) * n3;
      const V3<float> ln1 = lds3(Lc, n3);            // lambda^{n+1} of row r+1
      if (k < nr) {
        const int m = v >> 2;
        const bool n_in = r + 1 < ny, s_in = r > 0;
        const float* rw = rowtab + 8 * r;
        const RowK rk = {rw[0], rw[1], rw[3], rw[4], rw[5], rw[6], rw[7]};
        const V3<float> C = Cc;
        const V3<float> rE = lds3(Zr + 3 * ny, zW + 3 * k);
        const V3<float> rW = lds3(Zr, zW + 3 * k);
        const V3<float> E = pick3({0.f, cur.Eu, cur.Ev}, rE, me);
        const V3<float> W = pick3({0.f, cur.Wu, cur.Wv}, rW, mw);
        V3<float> N = cur.Cn, Sv = Cs;
        // rows at the box's south or north edge (wave-uniform test)
        if (__builtin_amdgcn_ballot_w64(!n_in || !s_in) != 0) {
          N = pick3(N, lds3(Zr + 3 * nx, zS), __builtin_amdgcn_ballot_w64(n_in));
          Sv = pick3(Sv, lds3(Zr, zS), __builtin_amdgcn_ballot_w64(s_in));
        }
        const float sn = (SPAN && !n_in && S.pole_n) ? -1.0f : 1.0f;
        const float ss = (SPAN && !s_in && S.pole_s) ? -1.0f : 1.0f;
        const V3<float> l0 = lc, kE = lds3(Lc, 3), kW = lds3(Lc, -3);
        const V3<float> gth = gather_cell(rk, st, stg, D.h0, C, E, W, N, Sv, l0, kE, kW, ln1, lp,
                                          sn, ss);
        float ah = gth.h, au = gth.u, av = gth.v;
        if (LAST) {
          au = l0.u + 0.5f * au;
          av = l0.v + 0.5f * av;
          ah = l0.h + 0.5f * ah;
        }
        float fh = 0.f, fu = 0.f, fv = 0.f;
        if (MODE == 1) {
          const double* Fz = forcing + S.traj_off + int64_t(n) * 3 * plane;
          fh = float(Fz[m]);
          fu = float(Fz[plane + m]);
          fv = float(Fz[2 * plane + m]);
        } else {
          const V3<float> tg = cur.tg;
          const float eh = MODE == 3 ? tg.h : C.h - tg.h;
          const float eu = MODE == 3 ? tg.u : C.u - tg.u;
          const float ev = MODE == 3 ? tg.v : C.v - tg.v;
          const float mk = cur.mk;
          fh = mk * ib_h * eh;
          fu = mk * ib_u * eu;
          fv = mk * ib_v * ev;
          if (MODE != 3)
            jloc += 0.5 * double(mk) * double(ib_h * eh * eh + ib_u * eu * eu + ib_v * ev * ev);
        }
        const float bh = fh + ah + ln[0][k];
        const float bu = fu + au + ln[1][k];
        const float bv = fv + av + ln[2][k];
        if (!LAST) {
          ln[0][k] = bh;
          ln[1][k] = bu;
          ln[2][k] = bv;
        } else {
          const int64_t o = S.ctrl_off + m;
          if (MODE == 0) {
            const double wb = D.weight_mode ? 1.0 : 1.0 / double(covl[m]);
            const double dh = x[o] - xb[o];
            const double du = x[o + plane] - xb[o + plane];
            const double dv = x[o + 2 * plane] - xb[o + 2 * plane];
            const double gh = wb * dh * D.isb2[0] + double(bh);
            const double gu = wb * du * D.isb2[1] + double(bu);
            const double gv = wb * dv * D.isb2[2] + double(bv);
            out[o] = gh;
            out[o + plane] = gu;
            out[o + 2 * plane] = gv;
            flag_nonfinite(D.nonfinite, !(isfinite(gh) && isfinite(gu) && isfinite(gv)));
            jloc += 0.5 * wb * (dh * dh * D.isb2[0] + du * du * D.isb2[1] + dv * dv * D.isb2[2]);
          } else {
            out[o] = double(bh);
            out[o + plane] = double(bu);
            out[o + 2 * plane] = double(bv);
            flag_nonfinite(D.nonfinite, !(isfinite(bh) && isfinite(bu) && isfinite(bv)));
          }
        }
      }
      // roll rows: r becomes the south row, r+1 the centre
      Cs = Cc;
      Cc = cur.Cn;
      lp = lc;
      lc = ln1;
      __builtin_amdgcn_sched_barrier(0);
      cur = nxt;
    }
    const int ob0 = lvl_ob[n], ob1 = lvl_ob[n + 1];
    const bool any_obs = MODE != 1 && ob1 > ob0;
    __syncthreads();                                   // all reads of lambda^{n+1} done
    if (ring_thread) {
      float* Zq = zring + ((n - 1) & 1) * 3 * nring + 3 * tid;
      Zq[0] = gnext.h; Zq[1] = gnext.u; Zq[2] = gnext.v;
    }
    if (!LAST) {
      // lambda^n into LDS; lambda^{n+1} into the registers
      int fs = f00, ns = nrows;
      asm volatile("" : "+v"(fs), "+v"(ns));
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (k < ns) {
          float* Lc = Lm + fs + k * n3;
          const float th = Lc[0], tu = Lc[1], tv = Lc[2];
          Lc[0] = ln[0][k];
          Lc[1] = ln[1][k];
          Lc[2] = ln[2][k];
          ln[0][k] = th;
          ln[1][k] = tu;
          ln[2][k] = tv;
        }
      }
    }
    if (MODE != 1 && any_obs) {
      __syncthreads();
      // the level's entries of every tile of the box in one range; a cell
      // and field occur at most once per level (duplicate observations are
      // rejected), so the updates of the frame never collide
      for (int o = ob0 + tid; o < ob1; o += kBoxThreads) {
        const int code = D.obs_code[o];
        const int loc = code >> 2, f = code & 3;
        const double rr = MODE == 3 ? double(D.dz[S.zoff + int64_t(n) * 3 * plane + f * plane + loc])
                                    : double(Z[f * plane + loc]) - D.obs_val[o];
        const double qo = D.obs_q[o];
        if (MODE != 3) jloc += 0.5 * qo * rr * rr;
        if (!LAST) {
          const int lr = loc / nx, lcc = loc - lr * nx;
          float* Lf = Lm + 3 * ((lr + 1) * nxp + lcc + 1) + f;
          *Lf = float(double(*Lf) + qo * rr);
        } else {
          out[S.ctrl_off + f * plane + loc] += qo * rr;
        }
      }
    }
    __syncthreads();
    if (wraps && !LAST) {
      fill_wraps(Lm, hsrc, hoff, hsgn, nring, nx, ny, false);
      __syncthreads();
    }
  };
  for (int n = L; n > 0; --n) level(n, std::false_type{});
  level(0, std::true_type{});
  if (MODE == 0 || MODE == 2) {
    const double tot = block_sum_box(jloc, red);
    for (int t = tid + 1; t < S.ntile; t += kBoxThreads) D.jpart[S.tile0 + t] = 0.0;
    if (tid == 0) D.jpart[S.tile0] = tot;
  }
}

template <int K, int MODE, bool SPAN>
__global__ __launch_bounds__(kBoxThreads) void k_adj_strip(Dom<float> D, const double* __restrict__ x,
                                                           const double* __restrict__ xb,
                                                           const double* __restrict__ forcing,
                                                           double* __restrict__ out,
                                                           const int32_t* __restrict__ order) {
  extern __shared__ float lds[];
  __shared__ double red[kBoxThreads / 64];
  const int s = order[blockIdx.x];
  if (D.active && !D.active[s]) return;
  adj_strip_body<K, MODE, SPAN>(D, x, xb, forcing, out, s, lds, red);
}

template <int K, bool SPAN>
__global__ __launch_bounds__(kBoxThreads) void k_tlm_box(Dom<float> D, const double* __restrict__ dx,
                                                         const int32_t* __restrict__ order) {
  extern __shared__ float lds[];
  const int s = order[blockIdx.x];
  if (D.active && !D.active[s]) return;
  tlm_box_body<K, SPAN>(D, dx, s, lds);
}

template <int K, int MODE, bool SPAN>
__global__ __launch_bounds__(kBoxThreads) void k_adj_box(Dom<float> D, const double* __restrict__ x,
                                                         const double* __restrict__ xb,
                                                         const double* __restrict__ forcing,
                                                         double* __restrict__ out,
                                                         const int32_t* __restrict__ order) {
  extern __shared__ float lds[];
  __shared__ double red[kBoxThreads / 64];
  const int s = order[blockIdx.x];
  if (D.active && !D.active[s]) return;
  adj_box_body<K, MODE, SPAN>(D, x, xb, forcing, out, s, lds, red);
}

// one whole local cost/gradient evaluation of box s in one workgroup: the
// forward sweep, then the adjoint sweep with the cost forcing (the levels the
// adjoint reads first are the ones the forward wrote last, still in the
// last-level cache)
template <int K, bool SPAN>
__global__ __launch_bounds__(kBoxThreads) void k_eval_box(Dom<float> D, const double* __restrict__ x,
                                                          const double* __restrict__ xb,
                                                          double* __restrict__ grad,
                                                          const int32_t* __restrict__ order) {
  extern __shared__ float lds[];
  __shared__ double red[kBoxThreads / 64];
  const int s = order[blockIdx.x];
  if (D.active && !D.active[s]) return;
  fwd_box_body<K, SPAN>(D, x, s, lds);
  __syncthreads();
  // an opaque copy of the box index: the adjoint recomputes its own indices
  // instead of keeping the forward's alive (which would spill)
  int sa = s;
  asm volatile("" : "+s"(sa));
  adj_box_body<K, 0, SPAN>(D, x, xb, nullptr, grad, sa, lds, red);
}

// dynamic LDS of the persistent kernels: padded level frame, per-row
// coefficients, and (adjoint) the state on the ring for two levels, the
// coverage byte of every cell and two ints per level
size_t box_lds_bytes(int ny, int nx, int nring, int nlev) {
  return size_t(3 * (ny + 2) * (nx + 2) + 8 * ny + 6 * nring) * sizeof(float) +
         ((size_t(ny) * nx + 3) & ~size_t(3)) + (2 * size_t(nlev) + 1) * sizeof(int);
}

// passes of 1024 cells the persistent kernels run for a box (0 when the box
// does not fit one workgroup: too many cells, ring positions or LDS bytes)
int box_passes(int ny, int nx, int nring, int nlev) {
  if (nring > kBoxThreads || nx + 2 > kBoxThreads) return 0;
  if (box_lds_bytes(ny, nx, nring, nlev) > kBoxLdsMax) return 0;
  const int k = (ny * nx + kBoxThreads - 1) / kBoxThreads;
  return k <= kBoxKMax ? k : 0;
}

namespace {
template <typename F>
hipError_t allow_lds(F* kernel) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(kBoxLdsMax));
}

template <int K, bool SPAN>
hipError_t prepare_ks() {
  hipError_t e = allow_lds(&k_fwd_box<K, SPAN>);
  if (e == hipSuccess) e = allow_lds(&k_adj_box<K, 0, SPAN>);
  if (e == hipSuccess) e = allow_lds(&k_adj_box<K, 1, SPAN>);
  if (e == hipSuccess) e = allow_lds(&k_adj_box<K, 2, SPAN>);
  if (e == hipSuccess) e = allow_lds(&k_adj_box<K, 3, SPAN>);
  if (e == hipSuccess) e = allow_lds(&k_tlm_box<K, SPAN>);
  if (e == hipSuccess) e = allow_lds(&k_adj_strip<K, 0, SPAN>);
  if (e == hipSuccess) e = allow_lds(&k_adj_strip<K, 1, SPAN>);
  if (e == hipSuccess) e = allow_lds(&k_adj_strip<K, 2, SPAN>);
  if (e == hipSuccess) e = allow_lds(&k_adj_strip<K, 3, SPAN>);
  if (e == hipSuccess) e = allow_lds(&k_eval_box<K, SPAN>);
  return e;
}

template <int K, bool SPAN>
hipError_t fwd_box_k(const Dom<float>& D, const double* x, const int32_t* order, int nboxes,
                     size_t lds_bytes, hipStream_t st) {
  auto* kern = &k_fwd_box<K, SPAN>;
  hipLaunchKernelGGL(kern, dim3(nboxes), dim3(kBoxThreads), lds_bytes, st, D, x, order);
  return hipGetLastError();
}

template <int K, bool SPAN>
hipError_t tlm_box_k(const Dom<float>& D, const double* dx, const int32_t* order, int nboxes,
                     size_t lds_bytes, hipStream_t st) {
  auto* kern = &k_tlm_box<K, SPAN>;
  hipLaunchKernelGGL(kern, dim3(nboxes), dim3(kBoxThreads), lds_bytes, st, D, dx, order);
  return hipGetLastError();
}

template <int K, int MODE, bool SPAN>
hipError_t adj_box_k(const Dom<float>& D, const double* x, const double* xb, const double* forcing,
                     double* out, const int32_t* order, int nboxes, size_t lds_bytes,
                     hipStream_t st) {
  auto* kern = &k_adj_box<K, MODE, SPAN>;
  hipLaunchKernelGGL(kern, dim3(nboxes), dim3(kBoxThreads), lds_bytes, st, D, x, xb, forcing, out,
                     order);
  return hipGetLastError();
}

template <int K, bool SPAN>
hipError_t eval_box_k(const Dom<float>& D, const double* x, const double* xb, double* grad,
                      const int32_t* order, int nboxes, size_t lds_bytes, hipStream_t st) {
  auto* kern = &k_eval_box<K, SPAN>;
  hipLaunchKernelGGL(kern, dim3(nboxes), dim3(kBoxThreads), lds_bytes, st, D, x, xb, grad, order);
  return hipGetLastError();
}

template <int K, int MODE, bool SPAN>
hipError_t adj_strip_k(const Dom<float>& D, const double* x, const double* xb, const double* forcing,
                       double* out, const int32_t* order, int nboxes, size_t lds_bytes,
                       hipStream_t st) {
  auto* kern = &k_adj_strip<K, MODE, SPAN>;
  hipLaunchKernelGGL(kern, dim3(nboxes), dim3(kBoxThreads), lds_bytes, st, D, x, xb, forcing, out,
                     order);
  return hipGetLastError();
}

template <int K, bool SPAN>
hipError_t adj_strip_mode(const Dom<float>& D, int mode, const double* x, const double* xb,
                          const double* forcing, double* out, const int32_t* order, int nboxes,
                          size_t lds_bytes, hipStream_t st) {
  if (mode == 0) return adj_strip_k<K, 0, SPAN>(D, x, xb, forcing, out, order, nboxes, lds_bytes, st);
  if (mode == 1) return adj_strip_k<K, 1, SPAN>(D, x, xb, forcing, out, order, nboxes, lds_bytes, st);
  if (mode == 3) return adj_strip_k<K, 3, SPAN>(D, x, xb, forcing, out, order, nboxes, lds_bytes, st);
  return adj_strip_k<K, 2, SPAN>(D, x, xb, forcing, out, order, nboxes, lds_bytes, st);
}

template <int K, bool SPAN>
hipError_t adj_box_mode(const Dom<float>& D, int mode, const double* x, const double* xb,
                        const double* forcing, double* out, const int32_t* order, int nboxes,
                        size_t lds_bytes, hipStream_t st) {
  if (mode == 0) return adj_box_k<K, 0, SPAN>(D, x, xb, forcing, out, order, nboxes, lds_bytes, st);
  if (mode == 1) return adj_box_k<K, 1, SPAN>(D, x, xb, forcing, out, order, nboxes, lds_bytes, st);
  if (mode == 3) return adj_box_k<K, 3, SPAN>(D, x, xb, forcing, out, order, nboxes, lds_bytes, st);
  return adj_box_k<K, 2, SPAN>(D, x, xb, forcing, out, order, nboxes, lds_bytes, st);
}
}  // namespace

int box_passes_max() { return kBoxKMax; }

// rows per column strip of the strip adjoint (0 when it does not apply)
int box_strip_rows(int ny, int nx, int nring, int nlev) {
  if (box_passes(ny, nx, nring, nlev) == 0) return 0;
  const int G = kBoxThreads / nx;
  const int R = (ny + G - 1) / G;
  return R <= kBoxKMax ? R : 0;
}

// raises the dynamic LDS limit of the kernels that run the given pass count
// (once per process and device, before any launch or stream capture)
hipError_t box_prepare(int passes) {
  hipError_t e = passes <= 10 ? prepare_ks<10, false>() : prepare_ks<kBoxKMax, false>();
  if (e == hipSuccess) e = passes <= 10 ? prepare_ks<10, true>() : prepare_ks<kBoxKMax, true>();
  return e;
}

// kernels are instantiated for 10 passes (boxes of up to 10240 cells, e.g.
// 72 x 136) and for the maximum of 11, without and with wrapped frame
// positions (span: some box of the launch spans the circle)
hipError_t launch_fwd_box(const Dom<float>& D, const double* x, const int32_t* order, int nboxes,
                          size_t lds_bytes, int passes, bool span, hipStream_t st) {
  if (passes <= 10)
    return span ? fwd_box_k<10, true>(D, x, order, nboxes, lds_bytes, st)
                : fwd_box_k<10, false>(D, x, order, nboxes, lds_bytes, st);
  return span ? fwd_box_k<kBoxKMax, true>(D, x, order, nboxes, lds_bytes, st)
              : fwd_box_k<kBoxKMax, false>(D, x, order, nboxes, lds_bytes, st);
}

hipError_t launch_tlm_box(const Dom<float>& D, const double* dx, const int32_t* order, int nboxes,
                          size_t lds_bytes, int passes, bool span, hipStream_t st) {
  if (passes <= 10)
    return span ? tlm_box_k<10, true>(D, dx, order, nboxes, lds_bytes, st)
                : tlm_box_k<10, false>(D, dx, order, nboxes, lds_bytes, st);
  return span ? tlm_box_k<kBoxKMax, true>(D, dx, order, nboxes, lds_bytes, st)
              : tlm_box_k<kBoxKMax, false>(D, dx, order, nboxes, lds_bytes, st);
}

hipError_t launch_adj_box(const Dom<float>& D, int mode, const double* x, const double* xb,
                          const double* forcing, double* out, const int32_t* order, int nboxes,
                          size_t lds_bytes, int passes, bool span, bool strip, hipStream_t st) {
  // column strips: passes = rows per strip
  if (strip && passes <= 10)
    return span ? adj_strip_mode<10, true>(D, mode, x, xb, forcing, out, order, nboxes, lds_bytes, st)
                : adj_strip_mode<10, false>(D, mode, x, xb, forcing, out, order, nboxes, lds_bytes, st);
  if (strip)
    return span ? adj_strip_mode<kBoxKMax, true>(D, mode, x, xb, forcing, out, order, nboxes, lds_bytes, st)
                : adj_strip_mode<kBoxKMax, false>(D, mode, x, xb, forcing, out, order, nboxes, lds_bytes, st);
  if (passes <= 10)
    return span ? adj_box_mode<10, true>(D, mode, x, xb, forcing, out, order, nboxes, lds_bytes, st)
                : adj_box_mode<10, false>(D, mode, x, xb, forcing, out, order, nboxes, lds_bytes, st);
  return span ? adj_box_mode<kBoxKMax, true>(D, mode, x, xb, forcing, out, order, nboxes, lds_bytes, st)
              : adj_box_mode<kBoxKMax, false>(D, mode, x, xb, forcing, out, order, nboxes, lds_bytes, st);
}

hipError_t launch_eval_box(const Dom<float>& D, const double* x, const double* xb, double* grad,
                           const int32_t* order, int nboxes, size_t lds_bytes, int passes,
                           bool span, hipStream_t st) {
  if (passes <= 10)
    return span ? eval_box_k<10, true>(D, x, xb, grad, order, nboxes, lds_bytes, st)
                : eval_box_k<10, false>(D, x, xb, grad, order, nboxes, lds_bytes, st);
  return span ? eval_box_k<kBoxKMax, true>(D, x, xb, grad, order, nboxes, lds_bytes, st)
              : eval_box_k<kBoxKMax, false>(D, x, xb, grad, order, nboxes, lds_bytes, st);
}

}  // namespace dd4dvar
