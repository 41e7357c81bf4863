// Batched L-BFGS state (device pointers, passed by value to the kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.h"
#include "parts.h"

namespace dd4dvar {

constexpr int kMaxPairs = 32;

struct LbState {
  const SubDev* subs;
  int nsub, m, max_iter, max_ls;
  int64_t N;                // packed control length
  double sb[3];             // sigma_b per field
  double c1, grad_rtol, jnoise;
  const double* xb;         // packed background controls
  // vectors (packed layout, FP64); S and Y hold m vectors each
  double *xi, *xi0, *g, *d, *xt, *xphys, *gradx, *S, *Y;
  // per subdomain
  double *J, *Jt, *gd, *alpha, *rho /* [m][nsub] */, *gamma, *g0norm, *gnorm, *step;
  int32_t *npairs, *head, *status, *iters, *trials;
  uint8_t* ls;              // in the line search (also the evaluation mask)
  int32_t* pending;         // device counter
  // vector work by parts; per box the recursion's a_k ([m][nsub]), the
  // accepted trial of the current line-search round and the ring slot its
  // pair went to (-1: not kept)
  PartMap P;
  double* alph;
  uint8_t* acc;
  int32_t* wslot;
};

void lb_to_x(const LbState& L, int use_trial, int sel, hipStream_t st);
void lb_from_x(const LbState& L, const double* x, hipStream_t st);
void lb_start(const LbState& L, hipStream_t st);
void lb_direction(const LbState& L, hipStream_t st);
void lb_trial(const LbState& L, hipStream_t st);
void lb_armijo(const LbState& L, hipStream_t st);
void lb_count(const LbState& L, hipStream_t st);
void lb_step(const LbState& L, hipStream_t st);

}  // namespace dd4dvar
