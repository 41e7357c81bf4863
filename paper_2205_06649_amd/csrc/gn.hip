// Batched Gauss-Newton local solver (Alg. 5; Alg. 6 with the normal
// equations of eq. line5and7 solved by conjugate gradients) over all
// subdomains at once, FP64.  One workgroup owns one subdomain's vectors; dot
// products are block reductions in a fixed order (deterministic).
//
// Variables xi = (x - x^b_s) / sigma_b (the diagonal square root of B as the
// preconditioner, eqs. EqV, Eq_matrixAV).  Each Gauss-Newton update solves
//   (V A V) dxi = -V grad J_s,   A = B_w^{-1} + M'^T W M',  V = diag(sigma_b),
// by CG from dxi = 0; the engine supplies M'^T W M' (V p) (the tangent-linear
// sweep and the adjoint sweep with the Gauss-Newton forcing), the background
// block is w^b per entry.  CG stops after cg_max_iter iterations, at
// |r| <= cg_rtol |r_0|, or when p^T A p is not positive; the update is taken
// in full; a local solve stops after max_iter updates or when
// |V grad J_s| <= grad_rtol |V grad J_s(x^0)|.
#include "gn.h"

namespace dd4dvar {

namespace {
constexpr int kB = 256;

__device__ double bsum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();                       // sh may still be read from a previous call
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < kB / 64; ++i) r += sh[i];
  return r;
}

__device__ double bmax(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = sh[0];
  for (int i = 1; i < kB / 64; ++i) r = fmax(r, sh[i]);
  return r;
}

__device__ __forceinline__ double sigma_of(const double* sb, int i, int ncell) {
  return sb[i / ncell];
}

// background weight w^b of control entry i (restriction weight of the cell)
__device__ __forceinline__ double wb_of(const GnState& G, const SubDev& S, int i) {
  if (G.weight_mode) return 1.0;
  const int cell = i % S.ncell;
  return 1.0 / double(G.cover[S.cell_off + cell]);
}
}  // namespace

__global__ __launch_bounds__(kB) void k_gn_to_x(GnState G) {
  const int s = blockIdx.x;
  const SubDev S = G.subs[s];
  const int n = 3 * S.ncell;
  const double* xi = G.xi + S.ctrl_off;
  const double* xb = G.xb + S.ctrl_off;
  double* x = G.xphys + S.ctrl_off;
  for (int i = threadIdx.x; i < n; i += kB) x[i] = xb[i] + sigma_of(G.sb, i, S.ncell) * xi[i];
}

__global__ __launch_bounds__(kB) void k_gn_from_x(GnState G, const double* __restrict__ x) {
  const int s = blockIdx.x;
  const SubDev S = G.subs[s];
  const int n = 3 * S.ncell;
  const double* xs = x + S.ctrl_off;
  const double* xb = G.xb + S.ctrl_off;
  double* xi = G.xi + S.ctrl_off;
  for (int i = threadIdx.x; i < n; i += kB) xi[i] = (xs[i] - xb[i]) / sigma_of(G.sb, i, S.ncell);
}

// start of a local solve from the evaluated x^0: |V g_0|, status, xi_0
__global__ __launch_bounds__(kB) void k_gn_start(GnState G) {
  __shared__ double sh[kB / 64];
  const int s = blockIdx.x;
  const SubDev S = G.subs[s];
  const int n = 3 * S.ncell;
  const double* gx = G.gradx + S.ctrl_off;
  const double* xi = G.xi + S.ctrl_off;
  double* x0 = G.xi0 + S.ctrl_off;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) {
    const double v = sigma_of(G.sb, i, S.ncell) * gx[i];
    acc += v * v;
    x0[i] = xi[i];
  }
  const double g0 = sqrt(bsum(acc, sh));
  if (threadIdx.x == 0) {
    G.J[s] = G.Jt[s];
    G.g0norm[s] = g0;
    G.gnorm[s] = g0;
    G.iters[s] = 0;
    G.cg_total[s] = 0;
    const int stt = G.max_iter <= 0 ? 3 : (g0 <= G.grad_rtol * g0 ? 1 : 0);
    G.status[s] = stt;
    G.gn_on[s] = stt == 0 ? 1 : 0;
  }
}

__global__ __launch_bounds__(kB) void k_gn_count(GnState G) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= G.nsub) return;
  if (G.gn_on[s]) atomicAdd(G.pending, 1);
}

// r = p = -V g, dxi = 0
__global__ __launch_bounds__(kB) void k_gn_cg_start(GnState G) {
  __shared__ double sh[kB / 64];
  const int s = blockIdx.x;
  if (!G.gn_on[s]) {
    if (threadIdx.x == 0) G.cg_on[s] = 0;
    return;
  }
  const SubDev S = G.subs[s];
  const int n = 3 * S.ncell;
  const double* gx = G.gradx + S.ctrl_off;
  double* r = G.r + S.ctrl_off;
  double* p = G.p + S.ctrl_off;
  double* d = G.dxi + S.ctrl_off;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) {
    const double v = -sigma_of(G.sb, i, S.ncell) * gx[i];
    r[i] = v;
    p[i] = v;
    d[i] = 0.0;
    acc += v * v;
  }
  const double rr = bsum(acc, sh);
  if (threadIdx.x == 0) {
    G.rr[s] = rr;
    G.rr0[s] = rr;
    G.cg_k[s] = 0;
    G.cg_on[s] = (G.cg_max_iter > 0 && sqrt(rr) > G.cg_rtol * sqrt(rr)) ? 1 : 0;
  }
}

__global__ __launch_bounds__(kB) void k_gn_cg_count(GnState G) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= G.nsub) return;
  if (G.cg_on[s]) atomicAdd(G.pending, 1);
}

// physical direction V p for the normal-matrix product
__global__ __launch_bounds__(kB) void k_gn_cg_dir(GnState G) {
  const int s = blockIdx.x;
  if (!G.cg_on[s]) return;
  const SubDev S = G.subs[s];
  const int n = 3 * S.ncell;
  const double* p = G.p + S.ctrl_off;
  double* dx = G.dx + S.ctrl_off;
  for (int i = threadIdx.x; i < n; i += kB) dx[i] = sigma_of(G.sb, i, S.ncell) * p[i];
}

// one CG iteration from hv = M'^T W M' (V p): q = w^b p + V hv
__global__ __launch_bounds__(kB) void k_gn_cg_update(GnState G) {
  __shared__ double sh[kB / 64];
  const int s = blockIdx.x;
  if (!G.cg_on[s]) return;
  const SubDev S = G.subs[s];
  const int n = 3 * S.ncell;
  double* q = G.hv + S.ctrl_off;
  double* p = G.p + S.ctrl_off;
  double* r = G.r + S.ctrl_off;
  double* d = G.dxi + S.ctrl_off;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) {
    const double v = wb_of(G, S, i) * p[i] + sigma_of(G.sb, i, S.ncell) * q[i];
    q[i] = v;
    acc += p[i] * v;
  }
  const double pq = bsum(acc, sh);
  if (!(pq > 0.0)) {
    if (threadIdx.x == 0) G.cg_on[s] = 0;
    return;
  }
  const double rr = G.rr[s];
  const double a = rr / pq;
  acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) {
    d[i] += a * p[i];
    const double v = r[i] - a * q[i];
    r[i] = v;
    acc += v * v;
  }
  const double rn = bsum(acc, sh);
  const double beta = rn / rr;
  for (int i = threadIdx.x; i < n; i += kB) p[i] = r[i] + beta * p[i];
  if (threadIdx.x == 0) {
    G.rr[s] = rn;
    const int k = G.cg_k[s] + 1;
    G.cg_k[s] = k;
    if (k >= G.cg_max_iter || sqrt(rn) <= G.cg_rtol * sqrt(G.rr0[s])) G.cg_on[s] = 0;
  }
}

// xi += dxi (the full Gauss-Newton update)
__global__ __launch_bounds__(kB) void k_gn_update(GnState G) {
  const int s = blockIdx.x;
  if (!G.gn_on[s]) return;
  const SubDev S = G.subs[s];
  const int n = 3 * S.ncell;
  double* xi = G.xi + S.ctrl_off;
  const double* d = G.dxi + S.ctrl_off;
  for (int i = threadIdx.x; i < n; i += kB) xi[i] += d[i];
  if (threadIdx.x == 0) {
    G.iters[s] += 1;
    G.cg_total[s] += G.cg_k[s];
  }
}

// after the evaluation at the updated x: J, |V g|, stop tests
__global__ __launch_bounds__(kB) void k_gn_after(GnState G) {
  __shared__ double sh[kB / 64];
  const int s = blockIdx.x;
  if (!G.gn_on[s]) return;
  const SubDev S = G.subs[s];
  const int n = 3 * S.ncell;
  const double* gx = G.gradx + S.ctrl_off;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) {
    const double v = sigma_of(G.sb, i, S.ncell) * gx[i];
    acc += v * v;
  }
  const double gn = sqrt(bsum(acc, sh));
  if (threadIdx.x == 0) {
    G.J[s] = G.Jt[s];
    G.gnorm[s] = gn;
    int stt = 0;
    if (G.iters[s] >= G.max_iter) stt = 3;
    else if (gn <= G.grad_rtol * G.g0norm[s]) stt = 1;
    G.status[s] = stt;
    G.gn_on[s] = stt == 0 ? 1 : 0;
  }
}

__global__ __launch_bounds__(kB) void k_gn_step(GnState G) {
  __shared__ double sh[kB / 64];
  const int s = blockIdx.x;
  const SubDev S = G.subs[s];
  const int n = 3 * S.ncell;
  const double* xi = G.xi + S.ctrl_off;
  const double* x0 = G.xi0 + S.ctrl_off;
  double mx = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) mx = fmax(mx, fabs(xi[i] - x0[i]));
  mx = bmax(mx, sh);
  if (threadIdx.x == 0) G.step[s] = mx;
}

struct Sb {
  double v[3];
};

__global__ __launch_bounds__(kB) void k_add_bdiag(const SubDev* __restrict__ subs,
                                                  const uint8_t* __restrict__ cover, int weight_mode,
                                                  Sb sb, const double* __restrict__ dx,
                                                  double* __restrict__ out) {
  const int s = blockIdx.x;
  const SubDev S = subs[s];
  const int n = 3 * S.ncell;
  for (int i = threadIdx.x; i < n; i += kB) {
    const int f = i / S.ncell, cell = i - f * S.ncell;
    const double wb = weight_mode ? 1.0 : 1.0 / double(cover[S.cell_off + cell]);
    const int64_t o = S.ctrl_off + i;
    out[o] += wb / (sb.v[f] * sb.v[f]) * dx[o];
  }
}

void gn_to_x(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_to_x, dim3(G.nsub), dim3(kB), 0, st, G);
}
void gn_from_x(const GnState& G, const double* x, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_from_x, dim3(G.nsub), dim3(kB), 0, st, G, x);
}
void gn_start(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_start, dim3(G.nsub), dim3(kB), 0, st, G);
}
void gn_count(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_count, dim3((G.nsub + kB - 1) / kB), dim3(kB), 0, st, G);
}
void gn_cg_start(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_cg_start, dim3(G.nsub), dim3(kB), 0, st, G);
}
void gn_cg_count(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_cg_count, dim3((G.nsub + kB - 1) / kB), dim3(kB), 0, st, G);
}
void gn_cg_dir(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_cg_dir, dim3(G.nsub), dim3(kB), 0, st, G);
}
void gn_cg_update(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_cg_update, dim3(G.nsub), dim3(kB), 0, st, G);
}
void gn_update(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_update, dim3(G.nsub), dim3(kB), 0, st, G);
}
void gn_after(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_after, dim3(G.nsub), dim3(kB), 0, st, G);
}
void gn_step(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_step, dim3(G.nsub), dim3(kB), 0, st, G);
}
void launch_add_bdiag(const SubDev* subs, int nsub, const uint8_t* cover, int weight_mode,
                      const double sb[3], const double* dx, double* out, hipStream_t st) {
  const Sb v{{sb[0], sb[1], sb[2]}};
  hipLaunchKernelGGL(k_add_bdiag, dim3(nsub), dim3(kB), 0, st, subs, cover, weight_mode, v, dx, out);
}

}  // namespace dd4dvar
