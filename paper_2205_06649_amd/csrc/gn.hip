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
//
// Or by the Lanczos method (Alg. 7) on the same system: V_1 = r_0 / |r_0|,
// w = A V_j - beta_j V_{j-1}, alpha_j = w . V_j, beta_{j+1} = |w - alpha_j V_j|,
// x_j = V_j y_j with T_j y_j = |r_0| e_1 (T_j the tridiagonal of the alphas
// and betas, factorized as L D L^T by one thread per subdomain after every
// product), residual norm beta_{j+1} |e_j^T y_j|: the same caps and stop tests
// as CG (a pivot of T_j that is not positive ends the run at x_{j-1}).  The
// basis is kept (cg_max_iter vectors) and x formed once at the end, with the
// extreme eigenvalues of T_j (Ritz values) by Sturm-sequence bisection.
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

// ---- Lanczos ----------------------------------------------------------------

// V_0 = p = -V g / |V g|, dxi = 0
__global__ __launch_bounds__(kB) void k_gn_lz_start(GnState G) {
  __shared__ double sh[kB / 64];
  const int s = blockIdx.x;
  if (!G.gn_on[s]) {
    if (threadIdx.x == 0) G.cg_on[s] = 0;
    return;
  }
  const SubDev S = G.subs[s];
  const int n = 3 * S.ncell;
  const double* gx = G.gradx + S.ctrl_off;
  double* d = G.dxi + S.ctrl_off;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) {
    const double v = sigma_of(G.sb, i, S.ncell) * gx[i];
    d[i] = 0.0;
    acc += v * v;
  }
  const double beta1 = sqrt(bsum(acc, sh));
  const bool on = G.cg_max_iter > 0 && beta1 > G.cg_rtol * beta1;
  if (on) {
    double* p = G.p + S.ctrl_off;
    double* v0 = G.lv + S.ctrl_off;
    for (int i = threadIdx.x; i < n; i += kB) {
      const double v = -sigma_of(G.sb, i, S.ncell) * gx[i] / beta1;
      p[i] = v;
      v0[i] = v;
    }
  }
  if (threadIdx.x == 0) {
    G.lb[int64_t(s) * (G.cg_max_iter + 1)] = beta1;
    G.cg_k[s] = 0;
    G.cg_on[s] = on ? 1 : 0;
  }
}

// one Lanczos step from hv = M'^T W M' (V p), p = V[j]
__global__ __launch_bounds__(kB) void k_gn_lz_update(GnState G) {
  __shared__ double sh[kB / 64];
  __shared__ int go;
  __shared__ double bnext;
  const int s = blockIdx.x;
  if (!G.cg_on[s]) return;
  const SubDev S = G.subs[s];
  const int n = 3 * S.ncell;
  const int K = G.cg_max_iter, j = G.cg_k[s];
  const int64_t sk = int64_t(s) * (K + 1);
  const double* q = G.hv + S.ctrl_off;
  const double* vj = G.lv + int64_t(j) * G.N + S.ctrl_off;
  const double* vm = G.lv + int64_t(j > 0 ? j - 1 : 0) * G.N + S.ctrl_off;
  const double bj = j > 0 ? G.lb[sk + j] : 0.0;
  double* w = G.r + S.ctrl_off;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) {
    double v = wb_of(G, S, i) * vj[i] + sigma_of(G.sb, i, S.ncell) * q[i];
    if (j > 0) v -= bj * vm[i];
    w[i] = v;
    acc += v * vj[i];
  }
  const double a = bsum(acc, sh);
  acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) {
    const double v = w[i] - a * vj[i];
    w[i] = v;
    acc += v * v;
  }
  const double b = sqrt(bsum(acc, sh));
  if (threadIdx.x == 0) {
    // T_{j+1} y = |r_0| e_1 by L D L^T (pivots d_i = a_i - lb_i^2 / d_{i-1}),
    // in scratch; a pivot that is not positive ends the run at the previous
    // iterate, whose coefficients stay in ly
    const double* la = G.la + sk;
    const double* lb = G.lb + sk;
    double* dv = G.ld + sk;
    double* z = G.lz + sk;
    bool pd = true;
    for (int i = 0; i <= j; ++i) {
      const double ai = i < j ? la[i] : a;
      const double l = i > 0 ? lb[i] / dv[i - 1] : 0.0;
      const double di = ai - l * (i > 0 ? lb[i] : 0.0);
      if (!(di > 0.0)) {
        pd = false;
        break;
      }
      dv[i] = di;
      z[i] = i == 0 ? lb[0] : -l * z[i - 1];
    }
    int cont = 0;
    if (pd) {
      double* y = G.ly + sk;
      y[j] = z[j] / dv[j];
      for (int i = j - 1; i >= 0; --i) y[i] = z[i] / dv[i] - (lb[i + 1] / dv[i]) * y[i + 1];
      G.la[sk + j] = a;
      G.lb[sk + j + 1] = b;
      const int k = j + 1;
      G.cg_k[s] = k;
      const bool stop = k >= K || !(b > 0.0) || b * fabs(y[j]) <= G.cg_rtol * lb[0];
      cont = stop ? 0 : 1;
    }
    go = cont;
    bnext = b;
    if (!cont) G.cg_on[s] = 0;
  }
  __syncthreads();
  if (!go) return;
  double* vn = G.lv + int64_t(j + 1) * G.N + S.ctrl_off;
  double* p = G.p + S.ctrl_off;
  const double ib = 1.0 / bnext;
  for (int i = threadIdx.x; i < n; i += kB) {
    const double v = w[i] * ib;
    vn[i] = v;
    p[i] = v;
  }
}

// number of eigenvalues of T (diagonal la, off-diagonal lb[1..]) below x
__device__ int sturm_count(const double* la, const double* lb, int k, double x) {
  int c = 0;
  double d = 1.0;
  for (int i = 0; i < k; ++i) {
    const double off = i > 0 ? lb[i] * lb[i] / d : 0.0;
    d = la[i] - x - off;
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++c;
  }
  return c;
}

// dxi = sum_j y_j V[j]; extreme Ritz values of T
__global__ __launch_bounds__(kB) void k_gn_lz_finish(GnState G) {
  const int s = blockIdx.x;
  if (!G.gn_on[s]) return;
  const SubDev S = G.subs[s];
  const int n = 3 * S.ncell;
  const int K = G.cg_max_iter, k = G.cg_k[s];
  const int64_t sk = int64_t(s) * (K + 1);
  double* d = G.dxi + S.ctrl_off;
  for (int i = threadIdx.x; i < n; i += kB) {
    double acc = 0.0;
    for (int t = 0; t < k; ++t) acc += G.ly[sk + t] * G.lv[int64_t(t) * G.N + S.ctrl_off + i];
    d[i] = acc;
  }
  if (threadIdx.x == 0 && k > 0) {
    const double* la = G.la + sk;
    const double* lb = G.lb + sk;
    double lo = la[0], hi = la[0];
    for (int i = 0; i < k; ++i) {
      const double r = (i > 0 ? fabs(lb[i]) : 0.0) + (i + 1 < k ? fabs(lb[i + 1]) : 0.0);
      lo = fmin(lo, la[i] - r);
      hi = fmax(hi, la[i] + r);
    }
    double a = lo, b = hi;
    for (int it = 0; it < 200 && a < b; ++it) {      // smallest: first x with count >= 1
      const double m = 0.5 * (a + b);
      if (m <= a || m >= b) break;
      if (sturm_count(la, lb, k, m) >= 1) b = m; else a = m;
    }
    G.ritz_lo[s] = 0.5 * (a + b);
    a = lo;
    b = hi;
    for (int it = 0; it < 200 && a < b; ++it) {      // largest: first x with count >= k
      const double m = 0.5 * (a + b);
      if (m <= a || m >= b) break;
      if (sturm_count(la, lb, k, m) >= k) b = m; else a = m;
    }
    G.ritz_hi[s] = 0.5 * (a + b);
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
void gn_lz_start(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_lz_start, dim3(G.nsub), dim3(kB), 0, st, G);
}
void gn_lz_update(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_lz_update, dim3(G.nsub), dim3(kB), 0, st, G);
}
void gn_lz_finish(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_lz_finish, dim3(G.nsub), dim3(kB), 0, st, G);
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
