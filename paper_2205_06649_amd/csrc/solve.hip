// Batched L-BFGS over all subdomains (FP64), for the local minimizations of
// Alg. 1.  The paper names L-BFGS as the quasi-Newton variant of the local
// Newton step (remark after Alg. 5); variables are xi = (x - x^b_s)/sigma_b,
// the diagonal special case of the B = V V^T preconditioning (eqs. EqV,
// Eq_matrixAV).  One workgroup owns one subdomain's vectors; dot products are
// block reductions in a fixed order (deterministic).
//
// Per subdomain: two-loop recursion with the m newest pairs and initial
// scaling gamma = s^T y / y^T y of the newest pair (1 without pairs);
// descent safeguard (steepest descent when g^T d >= 0); Armijo backtracking
// from step 1, halving; a pair is kept when s^T y > 1e-12 |s| |y|.  With a
// noise floor eps > 0, a local solve also stops when alpha |g^T d| <= eps |J|:
// decreases that small are below the rounding noise of J and cannot be
// resolved by the Armijo test.
#include "kernels.h"
#include "solve.h"

namespace dd4dvar {

namespace {
constexpr int kB = 256;

// sum over the block, returned to every thread
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

__device__ double dot(const double* a, const double* b, int n, double* sh) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) acc += a[i] * b[i];
  return bsum(acc, sh);
}

__device__ __forceinline__ double sigma_of(const LbState& L, int i, int ncell) {
  const int f = i / ncell;
  return L.sb[f];
}
}  // namespace

// x = x^b + sigma_b * v  for the selected subdomains (sel: 0 all, 1 = in line search)
__global__ __launch_bounds__(kB) void k_lb_to_x(LbState L, int use_trial, int sel) {
  const int s = blockIdx.x;
  if (sel == 1 && !L.ls[s]) return;
  const SubDev S = L.subs[s];
  const int n = 3 * S.ncell;
  const double* v = (use_trial ? L.xt : L.xi) + S.ctrl_off;
  const double* xb = L.xb + S.ctrl_off;
  double* x = L.xphys + S.ctrl_off;
  for (int i = threadIdx.x; i < n; i += kB) x[i] = xb[i] + sigma_of(L, i, S.ncell) * v[i];
}

// xi = (x - x^b) / sigma_b
__global__ __launch_bounds__(kB) void k_lb_from_x(LbState L, const double* __restrict__ x) {
  const int s = blockIdx.x;
  const SubDev S = L.subs[s];
  const int n = 3 * S.ncell;
  const double* xs = x + S.ctrl_off;
  const double* xb = L.xb + S.ctrl_off;
  double* xi = L.xi + S.ctrl_off;
  for (int i = threadIdx.x; i < n; i += kB) xi[i] = (xs[i] - xb[i]) / sigma_of(L, i, S.ncell);
}

// start of a local solve: g = sigma_b * grad_x at xi, J, |g0|, reset memory
__global__ __launch_bounds__(kB) void k_lb_start(LbState L) {
  __shared__ double sh[kB / 64];
  const int s = blockIdx.x;
  const SubDev S = L.subs[s];
  const int n = 3 * S.ncell;
  const double* gx = L.gradx + S.ctrl_off;
  double* g = L.g + S.ctrl_off;
  double* x0 = L.xi0 + S.ctrl_off;
  const double* xi = L.xi + S.ctrl_off;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) {
    const double v = sigma_of(L, i, S.ncell) * gx[i];
    g[i] = v;
    acc += v * v;
    x0[i] = xi[i];
  }
  const double gg = bsum(acc, sh);
  if (threadIdx.x == 0) {
    L.J[s] = L.Jt[s];
    L.g0norm[s] = sqrt(gg);
    L.gnorm[s] = sqrt(gg);
    L.npairs[s] = 0;
    L.head[s] = 0;
    L.iters[s] = 0;
    L.status[s] = (L.max_iter <= 0) ? 3 : ((sqrt(gg) <= L.grad_rtol * sqrt(gg)) ? 1 : 0);
    L.ls[s] = 0;
  }
}

// two-loop recursion: d = -H g for every subdomain still iterating
__global__ __launch_bounds__(kB) void k_lb_direction(LbState L) {
  __shared__ double sh[kB / 64];
  __shared__ double alph[kMaxPairs];
  const int s = blockIdx.x;
  if (L.status[s] != 0) return;
  const SubDev S = L.subs[s];
  const int n = 3 * S.ncell;
  const double* g = L.g + S.ctrl_off;
  double* d = L.d + S.ctrl_off;
  const int np = L.npairs[s], head = L.head[s];
  for (int i = threadIdx.x; i < n; i += kB) d[i] = g[i];    // q = g
  __syncthreads();
  for (int k = 0; k < np; ++k) {                             // newest to oldest
    const int slot = (head - 1 - k + L.m) % L.m;
    const double* sv = L.S + int64_t(slot) * L.N + S.ctrl_off;
    const double* yv = L.Y + int64_t(slot) * L.N + S.ctrl_off;
    const double rho = L.rho[int64_t(slot) * L.nsub + s];
    const double a = rho * dot(sv, d, n, sh);
    if (threadIdx.x == 0) alph[k] = a;
    for (int i = threadIdx.x; i < n; i += kB) d[i] -= a * yv[i];
    __syncthreads();
  }
  double gamma = 1.0;
  if (np > 0) gamma = L.gamma[s];
  for (int i = threadIdx.x; i < n; i += kB) d[i] *= gamma;
  __syncthreads();
  for (int k = np - 1; k >= 0; --k) {                        // oldest to newest
    const int slot = (head - 1 - k + L.m) % L.m;
    const double* sv = L.S + int64_t(slot) * L.N + S.ctrl_off;
    const double* yv = L.Y + int64_t(slot) * L.N + S.ctrl_off;
    const double rho = L.rho[int64_t(slot) * L.nsub + s];
    const double b = rho * dot(yv, d, n, sh);
    const double a = alph[k];
    for (int i = threadIdx.x; i < n; i += kB) d[i] += sv[i] * (a - b);
    __syncthreads();
  }
  // d = -r, descent safeguard
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) {
    d[i] = -d[i];
    acc += g[i] * d[i];
  }
  double gd = bsum(acc, sh);
  if (!(gd < 0.0)) {
    double gg = 0.0;
    for (int i = threadIdx.x; i < n; i += kB) {
      d[i] = -g[i];
      gg += g[i] * g[i];
    }
    gd = -bsum(gg, sh);
  }
  if (threadIdx.x == 0) {
    L.gd[s] = gd;
    L.alpha[s] = 1.0;
    L.trials[s] = 0;
    // a full step could not show a decrease above the noise floor of J
    const bool flat = -gd <= L.jnoise * fabs(L.J[s]);
    L.ls[s] = flat ? 0 : 1;
    if (flat) L.status[s] = 1;
  }
}

// trial point xt = xi + alpha d and its physical control
__global__ __launch_bounds__(kB) void k_lb_trial(LbState L) {
  const int s = blockIdx.x;
  if (!L.ls[s]) return;
  const SubDev S = L.subs[s];
  const int n = 3 * S.ncell;
  const double a = L.alpha[s];
  const double* xi = L.xi + S.ctrl_off;
  const double* d = L.d + S.ctrl_off;
  const double* xb = L.xb + S.ctrl_off;
  double* xt = L.xt + S.ctrl_off;
  double* x = L.xphys + S.ctrl_off;
  for (int i = threadIdx.x; i < n; i += kB) {
    const double v = xi[i] + a * d[i];
    xt[i] = v;
    x[i] = xb[i] + sigma_of(L, i, S.ncell) * v;
  }
}

// Armijo test of the evaluated trial; on acceptance the pair update and the
// move; counts the subdomains still searching in *pending
__global__ __launch_bounds__(kB) void k_lb_armijo(LbState L) {
  __shared__ double sh[kB / 64];
  __shared__ int accept;
  const int s = blockIdx.x;
  if (!L.ls[s]) return;
  const SubDev S = L.subs[s];
  const int n = 3 * S.ncell;
  if (threadIdx.x == 0) {
    const double Jt = L.Jt[s];
    accept = (Jt <= L.J[s] + L.c1 * L.alpha[s] * L.gd[s]) ? 1 : 0;
  }
  __syncthreads();
  if (!accept) {
    if (threadIdx.x == 0) {
      const int t = L.trials[s] + 1;
      L.trials[s] = t;
      const double a = 0.5 * L.alpha[s];
      L.alpha[s] = a;
      if (t >= L.max_ls || a * fabs(L.gd[s]) <= L.jnoise * fabs(L.J[s])) {
        L.ls[s] = 0;
        L.status[s] = 2;              // line search failed: keep the iterate
      } else {
        atomicAdd(L.pending, 1);
      }
    }
    return;
  }
  const int slot = L.head[s];
  double* sv = L.S + int64_t(slot) * L.N + S.ctrl_off;
  double* yv = L.Y + int64_t(slot) * L.N + S.ctrl_off;
  double* xi = L.xi + S.ctrl_off;
  double* g = L.g + S.ctrl_off;
  const double* xt = L.xt + S.ctrl_off;
  const double* gx = L.gradx + S.ctrl_off;
  double sy = 0, yy = 0, ss = 0, gg = 0;
  for (int i = threadIdx.x; i < n; i += kB) {
    const double gn = sigma_of(L, i, S.ncell) * gx[i];
    const double a = xt[i] - xi[i];
    const double b = gn - g[i];
    sy += a * b;
    yy += b * b;
    ss += a * a;
    gg += gn * gn;
  }
  sy = bsum(sy, sh);
  yy = bsum(yy, sh);
  ss = bsum(ss, sh);
  gg = bsum(gg, sh);
  const bool keep = sy > 1e-12 * sqrt(ss) * sqrt(yy);
  for (int i = threadIdx.x; i < n; i += kB) {
    const double gn = sigma_of(L, i, S.ncell) * gx[i];
    if (keep) {
      sv[i] = xt[i] - xi[i];
      yv[i] = gn - g[i];
    }
    xi[i] = xt[i];
    g[i] = gn;
  }
  if (threadIdx.x == 0) {
    if (keep) {
      L.rho[int64_t(slot) * L.nsub + s] = 1.0 / sy;
      L.gamma[s] = sy / yy;
      L.head[s] = (slot + 1) % L.m;
      L.npairs[s] = min(L.npairs[s] + 1, L.m);
    }
    L.J[s] = L.Jt[s];
    const double gn = sqrt(gg);
    L.gnorm[s] = gn;
    const int it = L.iters[s] + 1;
    L.iters[s] = it;
    L.ls[s] = 0;
    if (gn <= L.grad_rtol * L.g0norm[s]) L.status[s] = 1;
    else if (it >= L.max_iter) L.status[s] = 3;
  }
}

// number of subdomains still iterating, and the largest |xi - xi0| (per box,
// for the outer stop test of Alg. 1)
__global__ __launch_bounds__(kB) void k_lb_count(LbState L) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= L.nsub) return;
  if (L.status[s] == 0) atomicAdd(L.pending, 1);
}

__global__ __launch_bounds__(kB) void k_lb_step(LbState L) {
  __shared__ double sh[kB / 64];
  const int s = blockIdx.x;
  const SubDev S = L.subs[s];
  const int n = 3 * S.ncell;
  const double* xi = L.xi + S.ctrl_off;
  const double* x0 = L.xi0 + S.ctrl_off;
  double mx = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) mx = fmax(mx, fabs(xi[i] - x0[i]));
  mx = bmax(mx, sh);
  if (threadIdx.x == 0) L.step[s] = mx;
}

void lb_to_x(const LbState& L, int use_trial, int sel, hipStream_t st) {
  hipLaunchKernelGGL(k_lb_to_x, dim3(L.nsub), dim3(kB), 0, st, L, use_trial, sel);
}
void lb_from_x(const LbState& L, const double* x, hipStream_t st) {
  hipLaunchKernelGGL(k_lb_from_x, dim3(L.nsub), dim3(kB), 0, st, L, x);
}
void lb_start(const LbState& L, hipStream_t st) {
  hipLaunchKernelGGL(k_lb_start, dim3(L.nsub), dim3(kB), 0, st, L);
}
void lb_direction(const LbState& L, hipStream_t st) {
  hipLaunchKernelGGL(k_lb_direction, dim3(L.nsub), dim3(kB), 0, st, L);
}
void lb_trial(const LbState& L, hipStream_t st) {
  hipLaunchKernelGGL(k_lb_trial, dim3(L.nsub), dim3(kB), 0, st, L);
}
void lb_armijo(const LbState& L, hipStream_t st) {
  hipLaunchKernelGGL(k_lb_armijo, dim3(L.nsub), dim3(kB), 0, st, L);
}
void lb_count(const LbState& L, hipStream_t st) {
  hipLaunchKernelGGL(k_lb_count, dim3((L.nsub + kB - 1) / kB), dim3(kB), 0, st, L);
}
void lb_step(const LbState& L, hipStream_t st) {
  hipLaunchKernelGGL(k_lb_step, dim3(L.nsub), dim3(kB), 0, st, L);
}

}  // namespace dd4dvar
