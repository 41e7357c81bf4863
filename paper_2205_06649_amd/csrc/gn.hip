// Batched Gauss-Newton local solver (Alg. 5; Alg. 6 with the normal
// equations of eq. line5and7 solved by conjugate gradients) over all
// subdomains at once, FP64.  The vector work runs over parts of the boxes'
// controls (one workgroup per part); per-box dot products are sums of the
// parts' partial sums in a fixed order (deterministic), and the per-box
// scalar logic runs in kernels of one wave (or thread) per box between the
// vector passes.
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
constexpr int kBoxB = 64 * kBoxWaves;

__device__ __forceinline__ double sigma_of(const GnState& G, const Part& pt, int i) {
  return G.sb[i / pt.ncell];
}

// background weight w^b of control entry i (restriction weight of the cell)
__device__ __forceinline__ double wb_of(const uint8_t* cover, int weight_mode, const Part& pt, int i) {
  if (weight_mode) return 1.0;
  return 1.0 / double(cover[pt.cell_off + i % pt.ncell]);
}

dim3 parts_grid(const GnState& G) { return dim3(unsigned(G.P.nparts)); }
dim3 box_grid(const GnState& G) { return dim3(box_wave_blocks(G.nsub)); }
dim3 thread_grid(const GnState& G) { return dim3(unsigned((G.nsub + kPartB - 1) / kPartB)); }
}  // namespace

#define PART_LOOP(i) for (int i = pt.lo + int(threadIdx.x); i < pt.hi; i += kPartB)

__global__ __launch_bounds__(kPartB) void k_gn_to_x(GnState G) {
  const Part pt = G.P.part[blockIdx.x];
  const double* xi = G.xi + pt.off;
  const double* xb = G.xb + pt.off;
  double* x = G.xphys + pt.off;
  PART_LOOP(i) x[i] = xb[i] + sigma_of(G, pt, i) * xi[i];
}

__global__ __launch_bounds__(kPartB) void k_gn_from_x(GnState G, const double* __restrict__ x) {
  const Part pt = G.P.part[blockIdx.x];
  const double* xs = x + pt.off;
  const double* xb = G.xb + pt.off;
  double* xi = G.xi + pt.off;
  PART_LOOP(i) xi[i] = (xs[i] - xb[i]) / sigma_of(G, pt, i);
}

// |V g|^2 by parts (slot 0); at the start of a local solve also xi_0 = xi
template <bool kStart>
__global__ __launch_bounds__(kPartB) void k_gn_gnorm_v(GnState G) {
  __shared__ double sh[kPartB / 64];
  const Part pt = G.P.part[blockIdx.x];
  if (!kStart && !G.gn_on[pt.box]) return;
  const double* gx = G.gradx + pt.off;
  const double* xi = G.xi + pt.off;
  double* x0 = G.xi0 + pt.off;
  double acc = 0.0;
  PART_LOOP(i) {
    const double v = sigma_of(G, pt, i) * gx[i];
    acc += v * v;
    if (kStart) x0[i] = xi[i];
  }
  part_put(G.P, 0, blockIdx.x, acc, sh);
}

// start of a local solve from the evaluated x^0: |V g_0|, status
__global__ __launch_bounds__(kBoxB) void k_gn_start_s(GnState G) {
  const int s = wave_box();
  if (s >= G.nsub) return;
  const double g0 = sqrt(box_total(G.P, 0, s));
  if ((threadIdx.x & 63) != 0) return;
  G.J[s] = G.Jt[s];
  G.g0norm[s] = g0;
  G.gnorm[s] = g0;
  G.iters[s] = 0;
  G.cg_total[s] = 0;
  const int stt = G.max_iter <= 0 ? 3 : (g0 <= G.grad_rtol * g0 ? 1 : 0);
  G.status[s] = stt;
  G.gn_on[s] = stt == 0 ? 1 : 0;
}

__global__ __launch_bounds__(kPartB) void k_gn_count(GnState G) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= G.nsub) return;
  if (G.gn_on[s]) atomicAdd(G.pending, 1);
}

// r = p = -V g, dxi = 0; |r|^2 by parts
__global__ __launch_bounds__(kPartB) void k_gn_cg_start_v(GnState G) {
  __shared__ double sh[kPartB / 64];
  const Part pt = G.P.part[blockIdx.x];
  if (!G.gn_on[pt.box]) return;
  const double* gx = G.gradx + pt.off;
  double* r = G.r + pt.off;
  double* p = G.p + pt.off;
  double* d = G.dxi + pt.off;
  double acc = 0.0;
  PART_LOOP(i) {
    const double v = -sigma_of(G, pt, i) * gx[i];
    r[i] = v;
    p[i] = v;
    d[i] = 0.0;
    acc += v * v;
  }
  part_put(G.P, 0, blockIdx.x, acc, sh);
}

__global__ __launch_bounds__(kBoxB) void k_gn_cg_start_s(GnState G) {
  const int s = wave_box();
  if (s >= G.nsub) return;
  if (!G.gn_on[s]) {
    if ((threadIdx.x & 63) == 0) G.cg_on[s] = 0;
    return;
  }
  const double rr = box_total(G.P, 0, s);
  if ((threadIdx.x & 63) != 0) return;
  G.rr[s] = rr;
  G.rr0[s] = rr;
  G.cg_k[s] = 0;
  G.cg_on[s] = (G.cg_max_iter > 0 && sqrt(rr) > G.cg_rtol * sqrt(rr)) ? 1 : 0;
}

__global__ __launch_bounds__(kPartB) void k_gn_cg_count(GnState G) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= G.nsub) return;
  if (G.cg_on[s]) atomicAdd(G.pending, 1);
}

// physical direction V p for the normal-matrix product
__global__ __launch_bounds__(kPartB) void k_gn_cg_dir(GnState G) {
  const Part pt = G.P.part[blockIdx.x];
  if (!G.cg_on[pt.box]) return;
  const double* p = G.p + pt.off;
  double* dx = G.dx + pt.off;
  PART_LOOP(i) dx[i] = sigma_of(G, pt, i) * p[i];
}

// one CG iteration from hv = M'^T W M' (V p), in three vector passes with a
// per-box step between them:
//   q = w^b p + V hv, partial p . q      -> a = r.r / p.q (stop if p.q <= 0)
//   dxi += a p, r -= a q, partial r . r  -> beta, stop tests
//   p = r + beta p
__global__ __launch_bounds__(kPartB) void k_gn_cg_q(GnState G) {
  __shared__ double sh[kPartB / 64];
  const Part pt = G.P.part[blockIdx.x];
  if (!G.cg_on[pt.box]) return;
  double* q = G.hv + pt.off;
  const double* p = G.p + pt.off;
  double acc = 0.0;
  PART_LOOP(i) {
    const double v = wb_of(G.cover, G.weight_mode, pt, i) * p[i] + sigma_of(G, pt, i) * q[i];
    q[i] = v;
    acc += p[i] * v;
  }
  part_put(G.P, 0, blockIdx.x, acc, sh);
}

__global__ __launch_bounds__(kBoxB) void k_gn_cg_a(GnState G) {
  const int s = wave_box();
  if (s >= G.nsub || !G.cg_on[s]) return;
  const double pq = box_total(G.P, 0, s);
  if ((threadIdx.x & 63) != 0) return;
  if (!(pq > 0.0)) G.cg_on[s] = 0;
  else G.ca[s] = G.rr[s] / pq;
}

__global__ __launch_bounds__(kPartB) void k_gn_cg_r(GnState G) {
  __shared__ double sh[kPartB / 64];
  const Part pt = G.P.part[blockIdx.x];
  if (!G.cg_on[pt.box]) return;
  const double a = G.ca[pt.box];
  const double* q = G.hv + pt.off;
  const double* p = G.p + pt.off;
  double* r = G.r + pt.off;
  double* d = G.dxi + pt.off;
  double acc = 0.0;
  PART_LOOP(i) {
    d[i] += a * p[i];
    const double v = r[i] - a * q[i];
    r[i] = v;
    acc += v * v;
  }
  part_put(G.P, 1, blockIdx.x, acc, sh);
}

__global__ __launch_bounds__(kBoxB) void k_gn_cg_beta(GnState G) {
  const int s = wave_box();
  if (s >= G.nsub || !G.cg_on[s]) return;
  const double rn = box_total(G.P, 1, s);
  if ((threadIdx.x & 63) != 0) return;
  G.cb[s] = rn / G.rr[s];
  G.rr[s] = rn;
  const int k = G.cg_k[s] + 1;
  G.cg_k[s] = k;
  if (k >= G.cg_max_iter || sqrt(rn) <= G.cg_rtol * sqrt(G.rr0[s])) G.cg_on[s] = 0;
}

// (a run that stopped no longer needs p)
__global__ __launch_bounds__(kPartB) void k_gn_cg_p(GnState G) {
  const Part pt = G.P.part[blockIdx.x];
  if (!G.cg_on[pt.box]) return;
  const double beta = G.cb[pt.box];
  const double* r = G.r + pt.off;
  double* p = G.p + pt.off;
  PART_LOOP(i) p[i] = r[i] + beta * p[i];
}

// ---- Lanczos ----------------------------------------------------------------

// dxi = 0, |V g|^2 by parts
__global__ __launch_bounds__(kPartB) void k_gn_lz_start_v(GnState G) {
  __shared__ double sh[kPartB / 64];
  const Part pt = G.P.part[blockIdx.x];
  if (!G.gn_on[pt.box]) return;
  const double* gx = G.gradx + pt.off;
  double* d = G.dxi + pt.off;
  double acc = 0.0;
  PART_LOOP(i) {
    const double v = sigma_of(G, pt, i) * gx[i];
    d[i] = 0.0;
    acc += v * v;
  }
  part_put(G.P, 0, blockIdx.x, acc, sh);
}

__global__ __launch_bounds__(kBoxB) void k_gn_lz_start_s(GnState G) {
  const int s = wave_box();
  if (s >= G.nsub) return;
  if (!G.gn_on[s]) {
    if ((threadIdx.x & 63) == 0) G.cg_on[s] = 0;
    return;
  }
  const double beta1 = sqrt(box_total(G.P, 0, s));
  if ((threadIdx.x & 63) != 0) return;
  const bool on = G.cg_max_iter > 0 && beta1 > G.cg_rtol * beta1;
  G.lb[int64_t(s) * (G.cg_max_iter + 1)] = beta1;
  G.cg_k[s] = 0;
  G.cg_on[s] = on ? 1 : 0;
}

// V_0 = p = -V g / |V g|
__global__ __launch_bounds__(kPartB) void k_gn_lz_v0(GnState G) {
  const Part pt = G.P.part[blockIdx.x];
  if (!G.cg_on[pt.box]) return;
  const double beta1 = G.lb[int64_t(pt.box) * (G.cg_max_iter + 1)];
  const double* gx = G.gradx + pt.off;
  double* p = G.p + pt.off;
  double* v0 = G.lv + pt.off;
  PART_LOOP(i) {
    const double v = -sigma_of(G, pt, i) * gx[i] / beta1;
    p[i] = v;
    v0[i] = v;
  }
}

// one Lanczos step from hv = M'^T W M' (V p), p = V[j]:
//   w = A V_j - beta_j V_{j-1}, partial w . V_j     -> alpha_j
//   w -= alpha_j V_j, partial w . w                 -> beta_{j+1}, T y = |r_0| e_1
//   V_{j+1} = p = w / beta_{j+1}
__global__ __launch_bounds__(kPartB) void k_gn_lz_w(GnState G) {
  __shared__ double sh[kPartB / 64];
  const Part pt = G.P.part[blockIdx.x];
  const int s = pt.box;
  if (!G.cg_on[s]) return;
  const int j = G.cg_k[s];
  const double* q = G.hv + pt.off;
  const double* vj = G.lv + int64_t(j) * G.N + pt.off;
  const double* vm = G.lv + int64_t(j > 0 ? j - 1 : 0) * G.N + pt.off;
  const double bj = j > 0 ? G.lb[int64_t(s) * (G.cg_max_iter + 1) + j] : 0.0;
  double* w = G.r + pt.off;
  double acc = 0.0;
  PART_LOOP(i) {
    double v = wb_of(G.cover, G.weight_mode, pt, i) * vj[i] + sigma_of(G, pt, i) * q[i];
    if (j > 0) v -= bj * vm[i];
    w[i] = v;
    acc += v * vj[i];
  }
  part_put(G.P, 0, blockIdx.x, acc, sh);
}

__global__ __launch_bounds__(kBoxB) void k_gn_lz_a(GnState G) {
  const int s = wave_box();
  if (s >= G.nsub || !G.cg_on[s]) return;
  const double a = box_total(G.P, 0, s);
  if ((threadIdx.x & 63) == 0) G.ca[s] = a;
}

__global__ __launch_bounds__(kPartB) void k_gn_lz_orth(GnState G) {
  __shared__ double sh[kPartB / 64];
  const Part pt = G.P.part[blockIdx.x];
  const int s = pt.box;
  if (!G.cg_on[s]) return;
  const double a = G.ca[s];
  const double* vj = G.lv + int64_t(G.cg_k[s]) * G.N + pt.off;
  double* w = G.r + pt.off;
  double acc = 0.0;
  PART_LOOP(i) {
    const double v = w[i] - a * vj[i];
    w[i] = v;
    acc += v * v;
  }
  part_put(G.P, 1, blockIdx.x, acc, sh);
}

// T_{j+1} y = |r_0| e_1 by L D L^T (pivots d_i = a_i - lb_i^2 / d_{i-1}), in
// scratch; a pivot that is not positive ends the run at the previous
// iterate, whose coefficients stay in ly
__global__ __launch_bounds__(kBoxB) void k_gn_lz_tri(GnState G) {
  const int s = wave_box();
  if (s >= G.nsub || !G.cg_on[s]) return;
  const double b = sqrt(box_total(G.P, 1, s));
  if ((threadIdx.x & 63) != 0) return;
  const int K = G.cg_max_iter, j = G.cg_k[s];
  const int64_t sk = int64_t(s) * (K + 1);
  const double a = G.ca[s];
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
  G.cb[s] = b;
  if (!cont) G.cg_on[s] = 0;
}

// a run that goes on: V_{j+1} = p = w / beta_{j+1} (cg_k already j + 1)
__global__ __launch_bounds__(kPartB) void k_gn_lz_next(GnState G) {
  const Part pt = G.P.part[blockIdx.x];
  const int s = pt.box;
  if (!G.cg_on[s]) return;
  const double ib = 1.0 / G.cb[s];
  const double* w = G.r + pt.off;
  double* vn = G.lv + int64_t(G.cg_k[s]) * G.N + pt.off;
  double* p = G.p + pt.off;
  PART_LOOP(i) {
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

// dxi = sum_j y_j V[j]
__global__ __launch_bounds__(kPartB) void k_gn_lz_x(GnState G) {
  const Part pt = G.P.part[blockIdx.x];
  const int s = pt.box;
  if (!G.gn_on[s]) return;
  const int K = G.cg_max_iter, k = G.cg_k[s];
  const int64_t sk = int64_t(s) * (K + 1);
  double* d = G.dxi + pt.off;
  PART_LOOP(i) {
    double acc = 0.0;
    for (int t = 0; t < k; ++t) acc += G.ly[sk + t] * G.lv[int64_t(t) * G.N + pt.off + i];
    d[i] = acc;
  }
}

// extreme Ritz values of T (one thread per box)
__global__ __launch_bounds__(kPartB) void k_gn_lz_ritz(GnState G) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= G.nsub || !G.gn_on[s]) return;
  const int K = G.cg_max_iter, k = G.cg_k[s];
  if (k == 0) return;
  const int64_t sk = int64_t(s) * (K + 1);
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

// xi += dxi (the full Gauss-Newton update); the box's first part counts it
__global__ __launch_bounds__(kPartB) void k_gn_update(GnState G) {
  const Part pt = G.P.part[blockIdx.x];
  const int s = pt.box;
  if (!G.gn_on[s]) return;
  double* xi = G.xi + pt.off;
  const double* d = G.dxi + pt.off;
  PART_LOOP(i) xi[i] += d[i];
  if (pt.lo == 0 && threadIdx.x == 0) {
    G.iters[s] += 1;
    G.cg_total[s] += G.cg_k[s];
  }
}

// after the evaluation at the updated x: J, |V g|, stop tests
__global__ __launch_bounds__(kBoxB) void k_gn_after_s(GnState G) {
  const int s = wave_box();
  if (s >= G.nsub || !G.gn_on[s]) return;
  const double gn = sqrt(box_total(G.P, 0, s));
  if ((threadIdx.x & 63) != 0) return;
  G.J[s] = G.Jt[s];
  G.gnorm[s] = gn;
  int stt = 0;
  if (G.iters[s] >= G.max_iter) stt = 3;
  else if (gn <= G.grad_rtol * G.g0norm[s]) stt = 1;
  G.status[s] = stt;
  G.gn_on[s] = stt == 0 ? 1 : 0;
}

// out += B_w^{-1} dx (w^b / sigma_b^2 per entry)
struct Sb {
  double v[3];
};

__global__ __launch_bounds__(kPartB) void k_add_bdiag(PartMap P, const uint8_t* __restrict__ cover,
                                                      int weight_mode, Sb sb,
                                                      const double* __restrict__ dx,
                                                      double* __restrict__ out) {
  const Part pt = P.part[blockIdx.x];
  PART_LOOP(i) {
    const int f = i / pt.ncell;
    const double wb = wb_of(cover, weight_mode, pt, i);
    const int64_t o = pt.off + i;
    out[o] += wb / (sb.v[f] * sb.v[f]) * dx[o];
  }
}

#undef PART_LOOP

void gn_to_x(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_to_x, parts_grid(G), dim3(kPartB), 0, st, G);
}
void gn_from_x(const GnState& G, const double* x, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_from_x, parts_grid(G), dim3(kPartB), 0, st, G, x);
}
void gn_start(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_gnorm_v<true>, parts_grid(G), dim3(kPartB), 0, st, G);
  hipLaunchKernelGGL(k_gn_start_s, box_grid(G), dim3(kBoxB), 0, st, G);
}
void gn_count(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_count, thread_grid(G), dim3(kPartB), 0, st, G);
}
void gn_cg_start(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_cg_start_v, parts_grid(G), dim3(kPartB), 0, st, G);
  hipLaunchKernelGGL(k_gn_cg_start_s, box_grid(G), dim3(kBoxB), 0, st, G);
}
void gn_cg_count(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_cg_count, thread_grid(G), dim3(kPartB), 0, st, G);
}
void gn_cg_dir(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_cg_dir, parts_grid(G), dim3(kPartB), 0, st, G);
}
void gn_cg_update(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_cg_q, parts_grid(G), dim3(kPartB), 0, st, G);
  hipLaunchKernelGGL(k_gn_cg_a, box_grid(G), dim3(kBoxB), 0, st, G);
  hipLaunchKernelGGL(k_gn_cg_r, parts_grid(G), dim3(kPartB), 0, st, G);
  hipLaunchKernelGGL(k_gn_cg_beta, box_grid(G), dim3(kBoxB), 0, st, G);
  hipLaunchKernelGGL(k_gn_cg_p, parts_grid(G), dim3(kPartB), 0, st, G);
}
void gn_lz_start(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_lz_start_v, parts_grid(G), dim3(kPartB), 0, st, G);
  hipLaunchKernelGGL(k_gn_lz_start_s, box_grid(G), dim3(kBoxB), 0, st, G);
  hipLaunchKernelGGL(k_gn_lz_v0, parts_grid(G), dim3(kPartB), 0, st, G);
}
void gn_lz_update(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_lz_w, parts_grid(G), dim3(kPartB), 0, st, G);
  hipLaunchKernelGGL(k_gn_lz_a, box_grid(G), dim3(kBoxB), 0, st, G);
  hipLaunchKernelGGL(k_gn_lz_orth, parts_grid(G), dim3(kPartB), 0, st, G);
  hipLaunchKernelGGL(k_gn_lz_tri, box_grid(G), dim3(kBoxB), 0, st, G);
  hipLaunchKernelGGL(k_gn_lz_next, parts_grid(G), dim3(kPartB), 0, st, G);
}
void gn_lz_finish(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_lz_x, parts_grid(G), dim3(kPartB), 0, st, G);
  hipLaunchKernelGGL(k_gn_lz_ritz, thread_grid(G), dim3(kPartB), 0, st, G);
}
void gn_update(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_update, parts_grid(G), dim3(kPartB), 0, st, G);
}
void gn_after(const GnState& G, hipStream_t st) {
  hipLaunchKernelGGL(k_gn_gnorm_v<false>, parts_grid(G), dim3(kPartB), 0, st, G);
  hipLaunchKernelGGL(k_gn_after_s, box_grid(G), dim3(kBoxB), 0, st, G);
}
void launch_add_bdiag(const PartMap& P, const uint8_t* cover, int weight_mode, const double sb[3],
                      const double* dx, double* out, hipStream_t st) {
  const Sb v{{sb[0], sb[1], sb[2]}};
  hipLaunchKernelGGL(k_add_bdiag, dim3(unsigned(P.nparts)), dim3(kPartB), 0, st, P, cover,
                     weight_mode, v, dx, out);
}

}  // namespace dd4dvar
