// Persistent per-box sweeps (FP32 state): one workgroup owns one box for its
// whole time interval and keeps the current level in LDS and the level
// before it in registers, so that a forward step touches HBM only to store
// the trajectory and to read the frozen halo ring, and an adjoint step only
// to read the stored state, the overlap targets and the ring.
// Same arithmetic as the step kernels of sweep.hip (restricted model,
// eq. restricted; discrete U, V, H of Sec. 7; leapfrog with a forward-Euler
// half step).
//
// LDS holds each field of the level on a padded (ny+2) x (nx+2) grid whose
// one-cell frame carries the halo: frozen ring values (signs applied), or,
// for a box spanning the circle, copies of the box's own cells across the
// seam or the pole (u, v negated across a pole).  The stencil then needs no
// branches.  Per-row coefficients sit in LDS as well.
//
// Thread t owns column t % nx of the rows k R + t / nx, k = 0, 1, ..., with
// R = floor(1024 / nx) rows per pass, so all of its addresses are a base plus
// multiples of uniform strides.
#include "kernels.h"
#include "launch.h"
#include "stencil.h"

namespace dd4dvar {

using namespace stencil;

namespace {
constexpr int kBoxThreads = 1024;
constexpr int kBoxK = 11;                 // passes: boxes up to 11 R rows
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
__device__ __forceinline__ void fill_wraps(float* Ph, float* Pu, float* Pv, const int32_t* hsrc,
                                           const int32_t* hoff, const int32_t* hsgn, int nring,
                                           int nx, int ny, bool signed_copy) {
  const int nxp = nx + 2;
  for (int k = threadIdx.x; k < nring; k += kBoxThreads) {
    if (hsrc[k] >= 0) continue;
    const int p = frame_index(k, nx, ny);
    const int o = hoff[k], sr = o / nx, sc = o - sr * nx;
    const int q = (sr + 1) * nxp + sc + 1;
    const float sg = signed_copy ? float(hsgn[k]) : 1.0f;
    Ph[p] = Ph[q];
    Pu[p] = sg * Pu[q];
    Pv[p] = sg * Pv[q];
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

// Raw buffer loads: a 32-bit byte offset per lane plus a wave-uniform one,
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
  const float* Z = D.traj + S.traj_off + int64_t(level) * 3 * plane;
  const int o = D.hoff[S.hmap_off + k];
  const float sg = float(D.hsign[S.hmap_off + k]);
  return {Z[o], sg * Z[plane + o], sg * Z[2 * plane + o]};
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

// forward sweep of box s by the whole workgroup
__device__ __forceinline__ void fwd_box_body(const Dom<float>& D, const double* __restrict__ x,
                                             int s, float* lds) {
  const SubDev S = D.subs[s];
  const int nx = S.nx, ny = S.ny, nxp = nx + 2, npad = (ny + 2) * nxp;
  const int ncell = S.ncell, nring = S.nring;
  const int L = S.nlev - 1;
  const int tid = threadIdx.x;
  float* Ph = lds;
  float* Pu = lds + npad;
  float* Pv = lds + 2 * npad;
  float* rowtab = lds + 3 * npad;          // [ny][8]: a1 a2 a3 cf ct c cN cS
  const float h0 = D.h0, st = D.st, stg = D.stg;
  const int64_t plane = ncell;
  float* traj = D.traj + S.traj_off;
  const float* ring = D.ring + S.ring_off;
  const int32_t* hsrc = D.hsrc + S.hmap_off;
  const int32_t* hoff = D.hoff + S.hmap_off;
  const int32_t* hsgn = D.hsign + S.hmap_off;
  const bool wraps = S.span != 0;
  // this thread's column and first row
  const int R = kBoxThreads / nx;
  const int tr = tid / nx, tc = tid - tr * nx;
  const bool lane_on = tr < R;
  const int m0 = tr * nx + tc;                         // cell index, pass 0
  const int p0 = (tr + 1) * nxp + tc + 1;              // padded index, pass 0
  const int dm = R * nx, dp = R * nxp;                 // strides per pass

  for (int r = tid; r < ny; r += kBoxThreads) {
    const int j = S.row0 + r;
    const RowCoef<float> rc = D.rows[j];
    float* q = rowtab + 8 * r;
    q[0] = rc.a1; q[1] = rc.a2; q[2] = rc.a3; q[3] = rc.cf; q[4] = rc.ct; q[5] = rc.c;
    q[6] = D.cosx[j + 2];
    q[7] = D.cosx[j];
  }
  // level 0 from the FP64 control
  const double* xs = x + S.ctrl_off;
#pragma unroll
  for (int k = 0; k < kBoxK; ++k) {
    const int r = tr + k * R;
    if (lane_on && r < ny) {
      const int m = m0 + k * dm, p = p0 + k * dp;
      const float h = float(xs[m] - double(D.h0)), u = float(xs[plane + m]), v = float(xs[2 * plane + m]);
      Ph[p] = h; Pu[p] = u; Pv[p] = v;
      traj[m] = h; traj[plane + m] = u; traj[2 * plane + m] = v;
    }
  }
  for (int k = tid; k < nring; k += kBoxThreads) {
    if (hsrc[k] < 0) continue;
    const int p = frame_index(k, nx, ny);
    Ph[p] = ring[k]; Pu[p] = ring[nring + k]; Pv[p] = ring[2 * nring + k];
  }
  __syncthreads();
  if (wraps) {
    fill_wraps(Ph, Pu, Pv, hsrc, hoff, hsgn, nring, nx, ny, true);
    __syncthreads();
  }

  // zr holds this thread's cells of Z^{n-1} on entry to step n >= 1 (the
  // level before the one in LDS), so the base of the leapfrog update never
  // comes back from memory; the new level replaces it in place and is then
  // swapped with the LDS copy.
  float zr[3][kBoxK];
#pragma unroll
  for (int k = 0; k < kBoxK; ++k) zr[0][k] = zr[1][k] = zr[2][k] = 0.0f;
  for (int n = 0; n < L; ++n) {
    // frozen ring of level n+1, fetched while this step computes
    float rh = 0.f, ru = 0.f, rv = 0.f;
    const bool ring_pos = tid < nring && hsrc[tid] >= 0;
    if (ring_pos) {
      const float* R1 = ring + int64_t(n + 1) * 3 * nring;
      rh = R1[tid]; ru = R1[nring + tid]; rv = R1[2 * nring + tid];
    }
    const bool euler = n == 0;
    // opaque copies of the base offsets: the addresses derived from them are
    // recomputed every step instead of being hoisted out of the time loop
    // (11 passes x 15 neighbours of precomputed addresses spill)
    int pb = p0, mb = m0;
    asm volatile("" : "+v"(pb), "+v"(mb));
    float* out = traj + int64_t(n + 1) * 3 * plane;
#pragma unroll
    for (int k = 0; k < kBoxK; ++k) {
      const int r = tr + k * R;
      if (lane_on && r < ny) {
        const int p = pb + k * dp, m = mb + k * dm;
        const float* q = rowtab + 8 * r;
        const float a1 = q[0], a2 = q[1], a3 = q[2], cf = q[3], ct = q[4], cN = q[6], cS = q[7];
        const float h = Ph[p], u = Pu[p], v = Pv[p];
        const float hE = Ph[p + 1], uE = Pu[p + 1], vE = Pv[p + 1];
        const float hW = Ph[p - 1], uW = Pu[p - 1], vW = Pv[p - 1];
        const float hN = Ph[p + nxp], uN = Pu[p + nxp], vN = Pv[p + nxp];
        const float hS = Ph[p - nxp], uS = Pu[p - nxp], vS = Pv[p - nxp];
        const float cor = cf + ct * u;
        const float U = -a1 * u * (uE - uW) - st * v * (uN - uS) - a2 * (hE - hW) + cor * v;
        const float V = -a1 * u * (vE - vW) - st * v * (vN - vS) - stg * (hN - hS) - cor * u;
        const float H = -a1 * (h0 * (uE - uW) + (hE * uE - hW * uW)) -
                        a3 * (h0 * (vN * cN - vS * cS) + (hN * vN * cN - hS * vS * cS));
        // Z^1 = Z^0 + F(Z^0)/2 (Euler start), else Z^{n+1} = Z^{n-1} + F(Z^n)
        if (euler) {
          zr[0][k] = h + 0.5f * H;
          zr[1][k] = u + 0.5f * U;
          zr[2][k] = v + 0.5f * V;
        } else {
          zr[0][k] += H;
          zr[1][k] += U;
          zr[2][k] += V;
        }
        out[m] = zr[0][k]; out[plane + m] = zr[1][k]; out[2 * plane + m] = zr[2][k];
      }
      // keep each pass's loads within its own iteration: hoisting them all
      // ahead of the unrolled loop exhausts the register file
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();                                    // every read of level n done
    // level n+1 into LDS; level n into the registers (base of the next step)
#pragma unroll
    for (int k = 0; k < kBoxK; ++k) {
      const int r = tr + k * R;
      if (lane_on && r < ny) {
        const int p = pb + k * dp;
        const float th = Ph[p], tu = Pu[p], tv = Pv[p];
        Ph[p] = zr[0][k]; Pu[p] = zr[1][k]; Pv[p] = zr[2][k];
        zr[0][k] = th; zr[1][k] = tu; zr[2][k] = tv;
      }
    }
    if (ring_pos) {
      const int p = frame_index(tid, nx, ny);
      Ph[p] = rh; Pu[p] = ru; Pv[p] = rv;
    }
    __syncthreads();
    if (wraps) {
      fill_wraps(Ph, Pu, Pv, hsrc, hoff, hsgn, nring, nx, ny, true);
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
// or wrapped cells, signs applied) staged in LDS one level ahead.  Gather
// form and forcing as in k_adj (sweep.hip).
// MODE 0: cost forcing, gradient + J out; 1: caller forcing, adjoint out;
// 2: cost forcing, adjoint out.
template <int MODE>
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
  float* Lh = lds;
  float* Lu = lds + npad;
  float* Lv = lds + 2 * npad;
  float* rowtab = lds + 3 * npad;
  float* zring = rowtab + 8 * ny;          // [2 levels][3][nring]: state on the ring
  uint8_t* covl = reinterpret_cast<uint8_t*>(zring + 6 * nring);   // [ny*nx] coverage
  const int64_t plane = ncell;
  const int32_t* hsrc = D.hsrc + S.hmap_off;
  const int32_t* hoff = D.hoff + S.hmap_off;
  const int32_t* hsgn = D.hsign + S.hmap_off;
  const bool wraps = S.span != 0;
  const float st = D.st, stg = D.stg;
  const int fp = ncell * 4, nx4 = nx * 4, lvb = 3 * ncell * 4;   // byte strides
  const __amdgpu_buffer_rsrc_t zrs = make_rsrc(D.traj + S.traj_off, S.nlev * lvb);
  const __amdgpu_buffer_rsrc_t trs = make_rsrc(D.targ + S.traj_off, S.nlev * lvb);
  const float mu_f = float(D.mu);
  const float ib_h = float(D.isb2[0]), ib_u = float(D.isb2[1]), ib_v = float(D.isb2[2]);
  const int R = kBoxThreads / nx;
  const int tr = tid / nx, tc = tid - tr * nx;
  const bool lane_on = tr < R;
  const int m0 = tr * nx + tc;
  const int p0 = (tr + 1) * nxp + tc + 1;
  const int dm = R * nx, dp = R * nxp;

  fill_rowtab(rowtab, D, S);
  for (int i = tid; i < 3 * npad; i += kBoxThreads) lds[i] = 0.0f;   // lambda^{L+1} = 0
  for (int k = tid; k < nring; k += kBoxThreads) {
    const V3<float> g = ring_value(D, S, k, L);
    float* Zr = zring + (L & 1) * 3 * nring;
    Zr[k] = g.h; Zr[nring + k] = g.u; Zr[2 * nring + k] = g.v;
  }
  // coverage counts (the same at every level), kept in LDS so that the
  // target loads wait on an LDS read only
  for (int i = tid; i < ncell; i += kBoxThreads) covl[i] = D.cover[S.cell_off + i];
  __syncthreads();
  double jloc = 0.0;
  // this thread's cells of lambda^{n+2} (zero above the window)
  float ln[3][kBoxK];
#pragma unroll
  for (int k = 0; k < kBoxK; ++k) ln[0][k] = ln[1][k] = ln[2][k] = 0.0f;

  for (int n = L; n >= 0; --n) {
    // opaque per-step copies: neighbour indices and addresses are recomputed
    // each level rather than hoisted (and spilled) out of the level loop
    int pb = p0, mb = m0, trb = tr, tcb = tc;
    asm volatile("" : "+v"(pb), "+v"(mb), "+v"(trb), "+v"(tcb));
    const float* Z = D.traj + S.traj_off + int64_t(n) * 3 * plane;
    const int so = n * lvb;                              // level n, field h
    const float* Zr = zring + (n & 1) * 3 * nring;
    const int tcount = (MODE != 1) ? D.tcount[S.lev0 + n] : 0;
    // ring of level n-1, fetched now and staged after this level's reads
    V3<float> gnext = {0.f, 0.f, 0.f};
    const bool ring_thread = tid < nring && n > 0;
    if (ring_thread) gnext = ring_value(D, S, tid, n - 1);
#pragma unroll
    for (int k = 0; k < kBoxK; ++k) {
      const int r = trb + k * R;
      if (lane_on && r < ny) {
        const int m = mb + k * dm, p = pb + k * dp;
        const int c = tcb;
        const bool e_in = c + 1 < nx, w_in = c > 0, n_in = r + 1 < ny, s_in = r > 0;
        const float* rw = rowtab + 8 * r;
        const float a1 = rw[0], a2 = rw[1], cf = rw[3], ct = rw[4], cc = rw[5];
        const float a3n = rowtab[8 * (r + 1 < ny ? r + 1 : r) + 2];
        const float a3s = rowtab[8 * (r > 0 ? r - 1 : r) + 2];
        const int v0 = m * 4;
        // overlap targets (needed where covered) or the caller's forcing
        int K = 0;
        V3<float> tg = {0.f, 0.f, 0.f};
        float fh = 0.f, fu = 0.f, fv = 0.f;
        if (MODE != 1) {
          K = int(covl[m]) * tcount - 1;
          tg = bload3(trs, K > 0 ? v0 : 0, so, fp);
        } else {
          const double* Fz = forcing + S.traj_off + int64_t(n) * 3 * plane;
          fh = float(Fz[m]);
          fu = float(Fz[plane + m]);
          fv = float(Fz[2 * plane + m]);
        }
        // state of level n: the cell and its neighbours inside the box
        // (offsets clamped to the cell itself at the box edge) ...
        const V3<float> C = bload3(zrs, v0, so, fp);
        V3<float> E = bload3(zrs, e_in ? v0 + 4 : v0, so, fp);
        V3<float> W = bload3(zrs, w_in ? v0 - 4 : v0, so, fp);
        V3<float> N = bload3(zrs, n_in ? v0 + nx4 : v0, so, fp);
        V3<float> Sv = bload3(zrs, s_in ? v0 - nx4 : v0, so, fp);
        // ... and outside it, from the staged ring (every lane reads a valid
        // position and keeps it only at the edge)
        const int iE = e_in ? 0 : 2 * nx + ny + r, iW = w_in ? 0 : 2 * nx + r;
        const int iN = n_in ? 0 : nx + c, iS = s_in ? 0 : c;
        const V3<float> rE = {Zr[iE], Zr[nring + iE], Zr[2 * nring + iE]};
        const V3<float> rW = {Zr[iW], Zr[nring + iW], Zr[2 * nring + iW]};
        const V3<float> rN = {Zr[iN], Zr[nring + iN], Zr[2 * nring + iN]};
        const V3<float> rS = {Zr[iS], Zr[nring + iS], Zr[2 * nring + iS]};
        // every load of the cell is in flight before the first use
        __builtin_amdgcn_sched_barrier(0);
        E = pick3(E, rE, __builtin_amdgcn_ballot_w64(e_in));
        W = pick3(W, rW, __builtin_amdgcn_ballot_w64(w_in));
        N = pick3(N, rN, __builtin_amdgcn_ballot_w64(n_in));
        Sv = pick3(Sv, rS, __builtin_amdgcn_ballot_w64(s_in));
        // across a pole (boxes spanning the circle) the adjoint of a wrapped
        // neighbour carries the sign of u, v
        const int sn = (!n_in && S.pole_n) ? -1 : 1, ss = (!s_in && S.pole_s) ? -1 : 1;
        const V3<float> l2 = {ln[0][k], ln[1][k], ln[2][k]};
        // lambda^{n+1} from LDS (zero in frozen frame entries)
        const V3<float> l0 = {Lh[p], Lu[p], Lv[p]};
        const V3<float> kE = {Lh[p + 1], Lu[p + 1], Lv[p + 1]};
        const V3<float> kW = {Lh[p - 1], Lu[p - 1], Lv[p - 1]};
        const V3<float> kN = {Lh[p + nxp], Lu[p + nxp], Lv[p + nxp]};
        const V3<float> kS = {Lh[p - nxp], Lu[p - nxp], Lv[p - nxp]};
        const float hm = D.h0 + C.h;
        float au = l0.u * (-a1 * (E.u - W.u) + ct * C.v) +
                   l0.v * (-a1 * (E.v - W.v) - cf - 2.0f * ct * C.u);
        float av = l0.u * (-st * (N.u - Sv.u) + cf + ct * C.u) + l0.v * (-st * (N.v - Sv.v));
        float ah = 0.0f;
        au += a1 * (kE.u * E.u + kE.h * hm) - a1 * (kW.u * W.u + kW.h * hm);
        av += a1 * kE.v * E.u - a1 * kW.v * W.u;
        ah += (a2 * kE.u + a1 * kE.h * C.u) - (a2 * kW.u + a1 * kW.h * C.u);
        const float vkn = float(sn) * N.v, vks = float(ss) * Sv.v;
        au += kN.u * st * vkn - kS.u * st * vks;
        av += (kN.v * st * vkn + kN.h * a3n * hm * cc) - (kS.v * st * vks + kS.h * a3s * hm * cc);
        ah += (float(sn) * kN.v * stg + kN.h * a3n * C.v * cc) -
              (float(ss) * kS.v * stg + kS.h * a3s * C.v * cc);
        if (n == 0) {
          au = l0.u + 0.5f * au;
          av = l0.v + 0.5f * av;
          ah = l0.h + 0.5f * ah;
        }
        if (MODE != 1) {
          // overlap residual (the FP32 difference is the correctly rounded
          // exact one), its forcing in FP32 like the adjoint state, and the
          // cell's term of J accumulated in FP64
          const float eh = C.h - tg.h, eu = C.u - tg.u, ev = C.v - tg.v;
          const float mk = mu_f * float(K);
          fh = mk * ib_h * eh;
          fu = mk * ib_u * eu;
          fv = mk * ib_v * ev;
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
            const double wb = D.weight_mode ? 1.0 : 1.0 / double(D.cover[S.cell_off + m]);
            const double dh = x[o] - xb[o];
            const double du = x[o + plane] - xb[o + plane];
            const double dv = x[o + 2 * plane] - xb[o + 2 * plane];
            out[o] = wb * dh * D.isb2[0] + double(bh);
            out[o + plane] = wb * du * D.isb2[1] + double(bu);
            out[o + 2 * plane] = wb * dv * D.isb2[2] + double(bv);
            jloc += 0.5 * wb * (dh * dh * D.isb2[0] + du * du * D.isb2[1] + dv * dv * D.isb2[2]);
          } else {
            out[o] = double(bh);
            out[o + plane] = double(bu);
            out[o + 2 * plane] = double(bv);
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // observations of this box at level n
    int mine = 0;
    if (MODE != 1)
      for (int t = tid; t < S.ntile; t += kBoxThreads) {
        const int64_t key = int64_t(S.tile0 + t) * D.maxlev + n;
        mine += D.obs_ptr[key + 1] - D.obs_ptr[key];
      }
    const bool any_obs = __syncthreads_or(mine > 0);   // also: all reads of lambda^{n+1} done
    if (ring_thread) {
      float* Zq = zring + ((n - 1) & 1) * 3 * nring;
      Zq[tid] = gnext.h; Zq[nring + tid] = gnext.u; Zq[2 * nring + tid] = gnext.v;
    }
    if (n > 0) {
      // lambda^n into LDS; lambda^{n+1} into the registers (the lambda^{n+2}
      // of the next level)
#pragma unroll
      for (int k = 0; k < kBoxK; ++k) {
        const int r = trb + k * R;
        if (lane_on && r < ny) {
          const int p = pb + k * dp;
          const float th = Lh[p], tu = Lu[p], tv = Lv[p];
          Lh[p] = ln[0][k];
          Lu[p] = ln[1][k];
          Lv[p] = ln[2][k];
          ln[0][k] = th;
          ln[1][k] = tu;
          ln[2][k] = tv;
        }
      }
    }
    if (MODE != 1 && any_obs) {
      __syncthreads();                                   // lambda^n (or the gradient) complete
      for (int t = 0; t < S.ntile; ++t) {
        const int64_t key = int64_t(S.tile0 + t) * D.maxlev + n;
        const int o0 = D.obs_ptr[key], o1 = D.obs_ptr[key + 1];
        for (int o = o0 + tid; o < o1; o += kBoxThreads) {
          const int code = D.obs_code[o];
          const int loc = code >> 2, f = code & 3;
          const double rr = double(Z[f * plane + loc]) - D.obs_val[o];
          const double qo = D.obs_q[o];
          jloc += 0.5 * qo * rr * rr;
          if (n > 0) {
            const int lr = loc / nx, lc = loc - lr * nx;
            float* Lf = lds + f * npad;
            Lf[(lr + 1) * nxp + lc + 1] = float(double(Lf[(lr + 1) * nxp + lc + 1]) + qo * rr);
          } else {
            out[S.ctrl_off + f * plane + loc] += qo * rr;
          }
        }
      }
    }
    __syncthreads();
    if (wraps && n > 0) {
      fill_wraps(Lh, Lu, Lv, hsrc, hoff, hsgn, nring, nx, ny, false);
      __syncthreads();
    }
  }
  if (MODE != 1) {
    // the box total goes to its first tile slot, the others are cleared, so
    // the per-subdomain reduction of the step path applies unchanged
    const double tot = block_sum_box(jloc, red);
    for (int t = tid + 1; t < S.ntile; t += kBoxThreads) D.jpart[S.tile0 + t] = 0.0;
    if (tid == 0) D.jpart[S.tile0] = tot;
  }
}

__global__ __launch_bounds__(kBoxThreads) void k_fwd_box(Dom<float> D, const double* __restrict__ x,
                                                         const int32_t* __restrict__ order) {
  extern __shared__ float lds[];
  const int s = order[blockIdx.x];
  if (D.active && !D.active[s]) return;
  fwd_box_body(D, x, s, lds);
}

template <int MODE>
__global__ __launch_bounds__(kBoxThreads) void k_adj_box(Dom<float> D, const double* __restrict__ x,
                                                         const double* __restrict__ xb,
                                                         const double* __restrict__ forcing,
                                                         double* __restrict__ out,
                                                         const int32_t* __restrict__ order) {
  extern __shared__ float lds[];
  __shared__ double red[kBoxThreads / 64];
  const int s = order[blockIdx.x];
  if (D.active && !D.active[s]) return;
  adj_box_body<MODE>(D, x, xb, forcing, out, s, lds, red);
}

// one whole local cost/gradient evaluation of box s in one workgroup: the
// forward sweep, then the adjoint sweep with the cost forcing (the levels the
// adjoint reads first are the ones the forward wrote last, still in the
// last-level cache)
__global__ __launch_bounds__(kBoxThreads) void k_eval_box(Dom<float> D, const double* __restrict__ x,
                                                          const double* __restrict__ xb,
                                                          double* __restrict__ grad,
                                                          const int32_t* __restrict__ order) {
  extern __shared__ float lds[];
  __shared__ double red[kBoxThreads / 64];
  const int s = order[blockIdx.x];
  if (D.active && !D.active[s]) return;
  fwd_box_body(D, x, s, lds);
  __syncthreads();
  // an opaque copy of the box index: the adjoint recomputes its own indices
  // instead of keeping the forward's alive (which would spill)
  int sa = s;
  asm volatile("" : "+s"(sa));
  adj_box_body<0>(D, x, xb, nullptr, grad, sa, lds, red);
}

// dynamic LDS of the persistent kernels: padded level frame, per-row
// coefficients, and (adjoint) the state on the ring for two levels and the
// coverage byte of every cell
size_t box_lds_bytes(int ny, int nx, int nring) {
  return size_t(3 * (ny + 2) * (nx + 2) + 8 * ny + 6 * nring) * sizeof(float) + size_t(ny) * nx;
}

// whether a box fits one workgroup of the persistent kernels
bool box_fits(int ny, int nx, int nring) {
  if (nx > kBoxThreads || nring > kBoxThreads) return false;
  if (box_lds_bytes(ny, nx, nring) > kBoxLdsMax) return false;
  const int R = kBoxThreads / nx;
  return (ny + R - 1) / R <= kBoxK;
}

hipError_t launch_fwd_box(const Dom<float>& D, const double* x, const int32_t* order, int nboxes,
                          size_t lds_bytes, hipStream_t st) {
  static bool configured = false;
  if (!configured) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fwd_box),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(kBoxLdsMax));
    if (e != hipSuccess) return e;
    configured = true;
  }
  hipLaunchKernelGGL(k_fwd_box, dim3(nboxes), dim3(kBoxThreads), lds_bytes, st, D, x, order);
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch_adj_box_mode(const Dom<float>& D, const double* x, const double* xb,
                                      const double* forcing, double* out, const int32_t* order,
                                      int nboxes, size_t lds_bytes, hipStream_t st) {
  static bool configured = false;
  if (!configured) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_adj_box<MODE>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(kBoxLdsMax));
    if (e != hipSuccess) return e;
    configured = true;
  }
  hipLaunchKernelGGL(k_adj_box<MODE>, dim3(nboxes), dim3(kBoxThreads), lds_bytes, st, D, x, xb,
                     forcing, out, order);
  return hipGetLastError();
}

hipError_t launch_eval_box(const Dom<float>& D, const double* x, const double* xb, double* grad,
                           const int32_t* order, int nboxes, size_t lds_bytes, hipStream_t st) {
  static bool configured = false;
  if (!configured) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eval_box),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(kBoxLdsMax));
    if (e != hipSuccess) return e;
    configured = true;
  }
  hipLaunchKernelGGL(k_eval_box, dim3(nboxes), dim3(kBoxThreads), lds_bytes, st, D, x, xb, grad,
                     order);
  return hipGetLastError();
}

hipError_t launch_adj_box(const Dom<float>& D, int mode, const double* x, const double* xb,
                          const double* forcing, double* out, const int32_t* order, int nboxes,
                          size_t lds_bytes, hipStream_t st) {
  if (mode == 0) return launch_adj_box_mode<0>(D, x, xb, forcing, out, order, nboxes, lds_bytes, st);
  if (mode == 1) return launch_adj_box_mode<1>(D, x, xb, forcing, out, order, nboxes, lds_bytes, st);
  return launch_adj_box_mode<2>(D, x, xb, forcing, out, order, nboxes, lds_bytes, st);
}

}  // namespace dd4dvar
