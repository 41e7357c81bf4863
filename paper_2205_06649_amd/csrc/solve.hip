// Batched L-BFGS over all subdomains (FP64), for the local minimizations of
// Alg. 1.  The paper names L-BFGS as the quasi-Newton variant of the local
// Newton step (remark after Alg. 5); variables are xi = (x - x^b_s)/sigma_b,
// the diagonal special case of the B = V V^T preconditioning (eqs. EqV,
// Eq_matrixAV).  The vector work runs over parts of the boxes' controls (one
// workgroup per part); per-box dot products are sums of the parts' partial
// sums in a fixed order (deterministic), and the per-box scalar logic runs in
// kernels of one wave (or thread) per box between the vector passes.
//
// Per subdomain: two-loop recursion with the m newest pairs and initial
// scaling gamma = s^T y / y^T y of the newest pair (1 without pairs);
// descent safeguard (steepest descent when g^T d >= 0); Armijo backtracking
// from step 1, halving; a pair is kept when s^T y > 1e-12 |s| |y|.  With a
// noise floor eps > 0, a local solve also stops when alpha |g^T d| <= eps |J|:
// decreases that small are below the rounding noise of J and cannot be
// resolved by the Armijo test.
#include "kernels.h"
#include "parts.h"
#include "solve.h"

namespace dd4dvar {

namespace {
__device__ __forceinline__ double sigma_of(const LbState& L, const Part& pt, int i) {
  return L.sb[i / pt.ncell];
}
// newest-first pair k of box s -> its ring slot
__device__ __forceinline__ int pair_slot(const LbState& L, int s, int k) {
  return (L.head[s] - 1 - k + L.m) % L.m;
}
}  // namespace

// x = x^b + sigma_b * v  for the selected subdomains (sel: 0 all, 1 = in line search)
__global__ __launch_bounds__(kPartB) void k_lb_to_x(LbState L, int use_trial, int sel) {
  const Part pt = L.P.part[blockIdx.x];
  if (sel == 1 && !L.ls[pt.box]) return;
  const double* v = (use_trial ? L.xt : L.xi) + pt.off;
  const double* xb = L.xb + pt.off;
  double* x = L.xphys + pt.off;
  for (int i = pt.lo + threadIdx.x; i < pt.hi; i += kPartB) x[i] = xb[i] + sigma_of(L, pt, i) * v[i];
}

// xi = (x - x^b) / sigma_b
__global__ __launch_bounds__(kPartB) void k_lb_from_x(LbState L, const double* __restrict__ x) {
  const Part pt = L.P.part[blockIdx.x];
  const double* xs = x + pt.off;
  const double* xb = L.xb + pt.off;
  double* xi = L.xi + pt.off;
  for (int i = pt.lo + threadIdx.x; i < pt.hi; i += kPartB) xi[i] = (xs[i] - xb[i]) / sigma_of(L, pt, i);
}

// start of a local solve: g = sigma_b * grad_x at xi, xi0 = xi, |g|^2 by parts
__global__ __launch_bounds__(kPartB) void k_lb_start_v(LbState L) {
  __shared__ double sh[kPartB / 64];
  const Part pt = L.P.part[blockIdx.x];
  const double* gx = L.gradx + pt.off;
  double* g = L.g + pt.off;
  double* x0 = L.xi0 + pt.off;
  const double* xi = L.xi + pt.off;
  double acc = 0.0;
  for (int i = pt.lo + threadIdx.x; i < pt.hi; i += kPartB) {
    const double v = sigma_of(L, pt, i) * gx[i];
    g[i] = v;
    acc += v * v;
    x0[i] = xi[i];
  }
  part_put(L.P, 0, blockIdx.x, acc, sh);
}

// J, |g0|, empty memory, status
__global__ __launch_bounds__(64 * kBoxWaves) void k_lb_start_s(LbState L) {
  const int s = wave_box();
  if (s >= L.nsub) return;
  const double gg = box_total(L.P, 0, s);
  if ((threadIdx.x & 63) != 0) return;
  L.J[s] = L.Jt[s];
  L.g0norm[s] = sqrt(gg);
  L.gnorm[s] = sqrt(gg);
  L.npairs[s] = 0;
  L.head[s] = 0;
  L.iters[s] = 0;
  L.status[s] = (L.max_iter <= 0) ? 3 : ((sqrt(gg) <= L.grad_rtol * sqrt(gg)) ? 1 : 0);
  L.ls[s] = 0;
}

// step t of the two-loop recursion d = -H g for a box with np pairs (slots
// (t - 1) & 1 in, t & 1 out of the partial sums):
//   t = 0:            q = g, partial s_0 . q (np = 0: d = -g, partial g . d)
//   t = 1 .. np:      a_k = rho_k s_k . q (k = t - 1), q -= a_k y_k, then
//                     q *= gamma after the oldest pair; partial of the next
//                     pair's s . q, or of y_{np-1} . r after the last
//   t = np+1 .. 2np:  b_k = rho_k y_k . r (k = 2np - t), r += s_k (a_k - b_k);
//                     partial y_{k-1} . r, or after k = 0 d = -r, partial g . d
//   t = 2np + 1:      descent safeguard: g . d >= 0 -> d = -g, partial g . g
__global__ __launch_bounds__(kPartB) void k_lb_dir_step(LbState L, int t) {
  __shared__ double sh[kPartB / 64];
  const Part pt = L.P.part[blockIdx.x];
  const int s = pt.box;
  if (L.status[s] != 0) return;
  const int np = L.npairs[s];
  if (t > 2 * np + 1) return;
  const int in = (t - 1) & 1, out = t & 1;
  const int64_t N = L.N;
  double* d = L.d + pt.off;
  const double* g = L.g + pt.off;
  double acc = 0.0;
  if (t == 0) {
    if (np == 0) {
      for (int i = pt.lo + threadIdx.x; i < pt.hi; i += kPartB) {
        const double v = -g[i];
        d[i] = v;
        acc += g[i] * v;
      }
    } else {
      const double* sv = L.S + int64_t(pair_slot(L, s, 0)) * N + pt.off;
      for (int i = pt.lo + threadIdx.x; i < pt.hi; i += kPartB) {
        d[i] = g[i];
        acc += sv[i] * g[i];
      }
    }
  } else if (t <= np) {
    const int k = t - 1, slot = pair_slot(L, s, k);
    const double a = L.rho[int64_t(slot) * L.nsub + s] * box_total(L.P, in, s);
    if (pt.lo == 0 && threadIdx.x == 0) L.alph[int64_t(k) * L.nsub + s] = a;
    const double* yv = L.Y + int64_t(slot) * N + pt.off;
    if (t < np) {
      const double* sn = L.S + int64_t(pair_slot(L, s, t)) * N + pt.off;
      for (int i = pt.lo + threadIdx.x; i < pt.hi; i += kPartB) {
        const double v = d[i] - a * yv[i];
        d[i] = v;
        acc += sn[i] * v;
      }
    } else {
      const double gamma = L.gamma[s];
      for (int i = pt.lo + threadIdx.x; i < pt.hi; i += kPartB) {
        double v = d[i] - a * yv[i];
        v *= gamma;
        d[i] = v;
        acc += yv[i] * v;
      }
    }
  } else if (t <= 2 * np) {
    const int k = 2 * np - t, slot = pair_slot(L, s, k);
    const double b = L.rho[int64_t(slot) * L.nsub + s] * box_total(L.P, in, s);
    const double ab = L.alph[int64_t(k) * L.nsub + s] - b;
    const double* sv = L.S + int64_t(slot) * N + pt.off;
    if (k > 0) {
      const double* yn = L.Y + int64_t(pair_slot(L, s, k - 1)) * N + pt.off;
      for (int i = pt.lo + threadIdx.x; i < pt.hi; i += kPartB) {
        const double v = d[i] + sv[i] * ab;
        d[i] = v;
        acc += yn[i] * v;
      }
    } else {
      for (int i = pt.lo + threadIdx.x; i < pt.hi; i += kPartB) {
        const double v = -(d[i] + sv[i] * ab);
        d[i] = v;
        acc += g[i] * v;
      }
    }
  } else {
    if (box_total(L.P, in, s) < 0.0) return;
    for (int i = pt.lo + threadIdx.x; i < pt.hi; i += kPartB) {
      d[i] = -g[i];
      acc += g[i] * g[i];
    }
  }
  part_put(L.P, out, blockIdx.x, acc, sh);
}

// end of the recursion: g . d (or -|g|^2 after the safeguard), line-search start
__global__ __launch_bounds__(64 * kBoxWaves) void k_lb_dir_end(LbState L) {
  const int s = wave_box();
  if (s >= L.nsub || L.status[s] != 0) return;
  const int np = L.npairs[s];
  double gd = box_total(L.P, (2 * np) & 1, s);
  if (!(gd < 0.0)) gd = -box_total(L.P, (2 * np + 1) & 1, s);
  if ((threadIdx.x & 63) != 0) return;
  L.gd[s] = gd;
  L.alpha[s] = 1.0;
  L.trials[s] = 0;
  // a full step could not show a decrease above the noise floor of J
  const bool flat = -gd <= L.jnoise * fabs(L.J[s]);
  L.ls[s] = flat ? 0 : 1;
  if (flat) L.status[s] = 1;
}

// trial point xt = xi + alpha d and its physical control
__global__ __launch_bounds__(kPartB) void k_lb_trial(LbState L) {
  const Part pt = L.P.part[blockIdx.x];
  if (!L.ls[pt.box]) return;
  const double a = L.alpha[pt.box];
  const double* xi = L.xi + pt.off;
  const double* d = L.d + pt.off;
  const double* xb = L.xb + pt.off;
  double* xt = L.xt + pt.off;
  double* x = L.xphys + pt.off;
  for (int i = pt.lo + threadIdx.x; i < pt.hi; i += kPartB) {
    const double v = xi[i] + a * d[i];
    xt[i] = v;
    x[i] = xb[i] + sigma_of(L, pt, i) * v;
  }
}

// Armijo test of the evaluated trial (one thread per box): a rejected step
// is halved (or the search given up), counted in *pending; acc marks the
// accepted ones
__global__ __launch_bounds__(kPartB) void k_lb_accept(LbState L) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= L.nsub) return;
  if (!L.ls[s]) {
    L.acc[s] = 0;
    return;
  }
  const bool accept = L.Jt[s] <= L.J[s] + L.c1 * L.alpha[s] * L.gd[s];
  L.acc[s] = accept ? 1 : 0;
  if (accept) return;
  const int t = L.trials[s] + 1;
  L.trials[s] = t;
  const double a = 0.5 * L.alpha[s];
  L.alpha[s] = a;
  if (t >= L.max_ls || a * fabs(L.gd[s]) <= L.jnoise * fabs(L.J[s])) {
    L.ls[s] = 0;
    L.status[s] = 2;                  // line search failed: keep the iterate
  } else {
    atomicAdd(L.pending, 1);
  }
}

// accepted boxes: s . y, y . y, s . s and |g_new|^2 by parts
__global__ __launch_bounds__(kPartB) void k_lb_pair_v(LbState L) {
  __shared__ double sh[kPartB / 64];
  const Part pt = L.P.part[blockIdx.x];
  if (!L.acc[pt.box]) return;
  const double* xi = L.xi + pt.off;
  const double* g = L.g + pt.off;
  const double* xt = L.xt + pt.off;
  const double* gx = L.gradx + pt.off;
  double sy = 0, yy = 0, ss = 0, gg = 0;
  for (int i = pt.lo + threadIdx.x; i < pt.hi; i += kPartB) {
    const double gn = sigma_of(L, pt, i) * gx[i];
    const double a = xt[i] - xi[i];
    const double b = gn - g[i];
    sy += a * b;
    yy += b * b;
    ss += a * a;
    gg += gn * gn;
  }
  part_put(L.P, 0, blockIdx.x, sy, sh);
  part_put(L.P, 1, blockIdx.x, yy, sh);
  part_put(L.P, 2, blockIdx.x, ss, sh);
  part_put(L.P, 3, blockIdx.x, gg, sh);
}

// accepted boxes: keep the pair when s . y > 1e-12 |s| |y| (its ring slot
// in wslot, -1 if not kept), J, |g|, stop tests
__global__ __launch_bounds__(64 * kBoxWaves) void k_lb_pair_s(LbState L) {
  const int s = wave_box();
  if (s >= L.nsub || !L.acc[s]) return;
  const double sy = box_total(L.P, 0, s), yy = box_total(L.P, 1, s);
  const double ss = box_total(L.P, 2, s), gg = box_total(L.P, 3, s);
  if ((threadIdx.x & 63) != 0) return;
  const bool keep = sy > 1e-12 * sqrt(ss) * sqrt(yy);
  const int slot = L.head[s];
  L.wslot[s] = keep ? slot : -1;
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

// accepted boxes: the pair into its slot, the move xi = xt, g = g_new
__global__ __launch_bounds__(kPartB) void k_lb_move(LbState L) {
  const Part pt = L.P.part[blockIdx.x];
  const int s = pt.box;
  if (!L.acc[s]) return;
  const int slot = L.wslot[s];
  double* xi = L.xi + pt.off;
  double* g = L.g + pt.off;
  const double* xt = L.xt + pt.off;
  const double* gx = L.gradx + pt.off;
  if (slot >= 0) {
    double* sv = L.S + int64_t(slot) * L.N + pt.off;
    double* yv = L.Y + int64_t(slot) * L.N + pt.off;
    for (int i = pt.lo + threadIdx.x; i < pt.hi; i += kPartB) {
      const double gn = sigma_of(L, pt, i) * gx[i];
      sv[i] = xt[i] - xi[i];
      yv[i] = gn - g[i];
      xi[i] = xt[i];
      g[i] = gn;
    }
  } else {
    for (int i = pt.lo + threadIdx.x; i < pt.hi; i += kPartB) {
      xi[i] = xt[i];
      g[i] = sigma_of(L, pt, i) * gx[i];
    }
  }
}

// number of subdomains still iterating
__global__ __launch_bounds__(kPartB) void k_lb_count(LbState L) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= L.nsub) return;
  if (L.status[s] == 0) atomicAdd(L.pending, 1);
}

// the largest |xi - xi0| per box (the outer stop test of Alg. 1); a NaN
// counts as infinite so that the caller sees a non-finite step
__global__ __launch_bounds__(kPartB) void k_lb_step_v(LbState L) {
  __shared__ double sh[kPartB / 64];
  const Part pt = L.P.part[blockIdx.x];
  const double* xi = L.xi + pt.off;
  const double* x0 = L.xi0 + pt.off;
  double mx = 0.0;
  for (int i = pt.lo + threadIdx.x; i < pt.hi; i += kPartB) {
    const double v = fabs(xi[i] - x0[i]);
    mx = fmax(mx, v != v ? HUGE_VAL : v);
  }
  mx = part_bmax(mx, sh);
  if (threadIdx.x == 0) L.P.acc[blockIdx.x] = mx;
}

__global__ __launch_bounds__(64 * kBoxWaves) void k_lb_step_s(LbState L) {
  const int s = wave_box();
  if (s >= L.nsub) return;
  const double mx = box_max(L.P, 0, s);
  if ((threadIdx.x & 63) == 0) L.step[s] = mx;
}

namespace {
dim3 parts_grid(const LbState& L) { return dim3(unsigned(L.P.nparts)); }
}  // namespace

void lb_to_x(const LbState& L, int use_trial, int sel, hipStream_t st) {
  hipLaunchKernelGGL(k_lb_to_x, parts_grid(L), dim3(kPartB), 0, st, L, use_trial, sel);
}
void lb_from_x(const LbState& L, const double* x, hipStream_t st) {
  hipLaunchKernelGGL(k_lb_from_x, parts_grid(L), dim3(kPartB), 0, st, L, x);
}
void lb_start(const LbState& L, hipStream_t st) {
  hipLaunchKernelGGL(k_lb_start_v, parts_grid(L), dim3(kPartB), 0, st, L);
  hipLaunchKernelGGL(k_lb_start_s, dim3(box_wave_blocks(L.nsub)), dim3(64 * kBoxWaves), 0, st, L);
}
void lb_direction(const LbState& L, hipStream_t st) {
  // 2 m + 2 steps cover every box (np <= m); a box idles after its own
  for (int t = 0; t <= 2 * L.m + 1; ++t)
    hipLaunchKernelGGL(k_lb_dir_step, parts_grid(L), dim3(kPartB), 0, st, L, t);
  hipLaunchKernelGGL(k_lb_dir_end, dim3(box_wave_blocks(L.nsub)), dim3(64 * kBoxWaves), 0, st, L);
}
void lb_trial(const LbState& L, hipStream_t st) {
  hipLaunchKernelGGL(k_lb_trial, parts_grid(L), dim3(kPartB), 0, st, L);
}
void lb_armijo(const LbState& L, hipStream_t st) {
  hipLaunchKernelGGL(k_lb_accept, dim3((L.nsub + kPartB - 1) / kPartB), dim3(kPartB), 0, st, L);
  hipLaunchKernelGGL(k_lb_pair_v, parts_grid(L), dim3(kPartB), 0, st, L);
  hipLaunchKernelGGL(k_lb_pair_s, dim3(box_wave_blocks(L.nsub)), dim3(64 * kBoxWaves), 0, st, L);
  hipLaunchKernelGGL(k_lb_move, parts_grid(L), dim3(kPartB), 0, st, L);
}
void lb_count(const LbState& L, hipStream_t st) {
  hipLaunchKernelGGL(k_lb_count, dim3((L.nsub + kPartB - 1) / kPartB), dim3(kPartB), 0, st, L);
}
void lb_step(const LbState& L, hipStream_t st) {
  hipLaunchKernelGGL(k_lb_step_v, parts_grid(L), dim3(kPartB), 0, st, L);
  hipLaunchKernelGGL(k_lb_step_s, dim3(box_wave_blocks(L.nsub)), dim3(64 * kBoxWaves), 0, st, L);
}

}  // namespace dd4dvar
