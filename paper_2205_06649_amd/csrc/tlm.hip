// Tangent linear model of the local sweeps (the TLM step of Alg. 6; the
// linearized restricted model, eq. restricted, about the stored trajectory of
// the last forward run), batched over every subdomain like the forward step
// kernels: one workgroup per 256-cell tile of a box.
//
//   dZ^0 = dx,  dZ^1 = dZ^0 + F'(Z^0) dZ^0 / 2,  dZ^{n+1} = dZ^{n-1} + F'(Z^n) dZ^n,
//
// with F' the derivative of the discrete U, V, H of Sec. 7 (p = q = 1,
// alpha = 0) at the stored state Z^n.  The frozen halo ring does not depend
// on the control, so its perturbation is zero; wrapped neighbours of a box
// spanning the circle take the box's own perturbation (u, v negated across a
// pole).  With h stored as h - h_ref, the flux terms linearize as
// (h_ref + h) du + dh u.
#include "kernels.h"
#include "launch.h"
#include "stencil.h"

#ifndef DD4DVAR_TLM_T
#error "compile with -DDD4DVAR_TLM_T=float or double"
#endif

namespace dd4dvar {

using namespace stencil;

namespace {
// perturbation of a neighbour: the box value (signed across a pole), zero on
// a frozen ring position; the load is unconditional (from the cell itself)
template <typename T>
__device__ __forceinline__ V3<T> ld_pert(const T* dZ, int64_t plane, int idx, int m, int sgn) {
  const bool in = idx >= 0;
  const int i = in ? idx : m;
  const T h = dZ[i], u = dZ[plane + i], v = dZ[2 * plane + i];
  const T sg = T(sgn);
  return {in ? h : T(0), in ? sg * u : T(0), in ? sg * v : T(0)};
}

template <typename T>
__device__ __forceinline__ T* dzlevel(const Dom<T>& D, const SubDev& S, int n) {
  return D.dz + S.zoff + int64_t(n) * 3 * S.ncell;
}
}  // namespace

// dZ^0 = dx (packed FP64 control perturbation)
template <typename T>
__global__ __launch_bounds__(kTile) void k_tlm_init(Dom<T> D, const double* __restrict__ dx,
                                                    int tile_base) {
  const int2 wt = D.tiles[tile_base + xcd_tile(blockIdx.x, gridDim.x)];
  if (D.active && !D.active[wt.x]) return;
  const SubDev S = D.subs[wt.x];
  const int m = wt.y * kTile + threadIdx.x;
  if (m >= S.ncell) return;
  const double* d = dx + S.ctrl_off;
  T* dZ = dzlevel(D, S, 0);
  dZ[m] = T(d[m]);
  dZ[S.ncell + m] = T(d[S.ncell + m]);
  dZ[2 * S.ncell + m] = T(d[2 * S.ncell + m]);
}

// dZ^{n+1} from dZ^n, dZ^{n-1} and the stored Z^n
template <typename T>
__global__ __launch_bounds__(kTile) void k_tlm(Dom<T> D, int n, int tile_base) {
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
  const T* dZ = dzlevel(D, S, n);
  const T* dP = n >= 1 ? dzlevel(D, S, n - 1) : dZ;
  const NbrIdx q = nbr_index(S, r, c, D.half);
  const int j = S.row0 + r;
  // every load first, unconditionally
  const V3<T> C = ld_box(Z, plane, m, T(1));
  const V3<T> E = ld_nbr(Z, R, plane, S.nring, q.e, 1);
  const V3<T> W = ld_nbr(Z, R, plane, S.nring, q.w, 1);
  const V3<T> N = ld_nbr(Z, R, plane, S.nring, q.n, q.sn);
  const V3<T> Sv = ld_nbr(Z, R, plane, S.nring, q.s, q.ss);
  const V3<T> dC = ld_box(dZ, plane, m, T(1));
  const V3<T> dE = ld_pert(dZ, plane, q.e, m, 1);
  const V3<T> dW = ld_pert(dZ, plane, q.w, m, 1);
  const V3<T> dN = ld_pert(dZ, plane, q.n, m, q.sn);
  const V3<T> dS = ld_pert(dZ, plane, q.s, m, q.ss);
  const V3<T> B = ld_box(dP, plane, m, T(1));
  const RowCoef<T> rc = D.rows[j];
  const T cN = D.cosx[j + 2], cS = D.cosx[j];
  const T st = D.st, stg = D.stg, h0 = D.h0;
  const T cor = rc.cf + rc.ct * C.u;
  const T dU = -rc.a1 * (dC.u * (E.u - W.u) + C.u * (dE.u - dW.u)) -
               st * (dC.v * (N.u - Sv.u) + C.v * (dN.u - dS.u)) - rc.a2 * (dE.h - dW.h) +
               (cor * dC.v + rc.ct * dC.u * C.v);
  const T dV = -rc.a1 * (dC.u * (E.v - W.v) + C.u * (dE.v - dW.v)) -
               st * (dC.v * (N.v - Sv.v) + C.v * (dN.v - dS.v)) - stg * (dN.h - dS.h) -
               (cor * dC.u + rc.ct * dC.u * C.u);
  const T dH = -rc.a1 * (((h0 + E.h) * dE.u + dE.h * E.u) - ((h0 + W.h) * dW.u + dW.h * W.u)) -
               rc.a3 * (((h0 + N.h) * dN.v + dN.h * N.v) * cN - ((h0 + Sv.h) * dS.v + dS.h * Sv.v) * cS);
  const T wgt = n == 0 ? T(0.5) : T(1);
  T* out = dzlevel(D, S, n + 1);
  out[m] = B.h + wgt * dH;
  out[plane + m] = B.u + wgt * dU;
  out[2 * plane + m] = B.v + wgt * dV;
}

// packed FP64 output of the perturbation trajectory (every level)
template <typename T>
__global__ __launch_bounds__(kTile) void k_dz_out(Dom<T> D, double* __restrict__ out, int tile_base) {
  const int2 wt = D.tiles[tile_base + xcd_tile(blockIdx.x, gridDim.x)];
  const SubDev S = D.subs[wt.x];
  const int m = wt.y * kTile + threadIdx.x;
  if (m >= S.ncell) return;
  const int64_t plane = S.ncell;
  for (int n = 0; n < S.nlev; ++n) {
    const T* dZ = dzlevel(D, S, n);
    double* o = out + S.traj_off + int64_t(n) * 3 * plane;
    o[m] = double(dZ[m]);
    o[plane + m] = double(dZ[plane + m]);
    o[2 * plane + m] = double(dZ[2 * plane + m]);
  }
}

template <typename T>
void launch_tlm_init(const Dom<T>& D, const double* dx, int tile_base, int ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_tlm_init<T>, dim3(ntiles), dim3(kTile), 0, st, D, dx, tile_base);
}
template <typename T>
void launch_tlm(const Dom<T>& D, int n, int tile_base, int ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_tlm<T>, dim3(ntiles), dim3(kTile), 0, st, D, n, tile_base);
}
template <typename T>
void launch_dz_out(const Dom<T>& D, double* out, int tile_base, int ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_dz_out<T>, dim3(ntiles), dim3(kTile), 0, st, D, out, tile_base);
}

#define DD4DVAR_INST(T)                                                                \
  template void launch_tlm_init<T>(const Dom<T>&, const double*, int, int, hipStream_t); \
  template void launch_tlm<T>(const Dom<T>&, int, int, int, hipStream_t);               \
  template void launch_dz_out<T>(const Dom<T>&, double*, int, int, hipStream_t);
// compiled once per state type, with the contraction rules of the sweeps
DD4DVAR_INST(DD4DVAR_TLM_T)
#undef DD4DVAR_INST

}  // namespace dd4dvar
