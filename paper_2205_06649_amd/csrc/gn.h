// Batched Gauss-Newton local solver state (device pointers, passed by value).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.h"
#include "parts.h"

namespace dd4dvar {

struct GnState {
  const SubDev* subs;
  int nsub, max_iter, cg_max_iter;
  int weight_mode;
  int64_t N;                // packed control length
  double sb[3];             // sigma_b per field
  double grad_rtol, cg_rtol;
  const double* xb;         // packed background controls
  const uint8_t* cover;     // spatial coverage per box cell (background weights)
  // vectors (packed layout, FP64)
  double *xi, *xi0, *dxi, *r, *p, *dx, *hv, *xphys, *gradx;
  // per subdomain
  double *J, *Jt, *g0norm, *gnorm, *rr, *rr0, *step;
  int32_t *status, *iters, *cg_k, *cg_total;
  uint8_t *gn_on, *cg_on;   // evaluation masks: in the GN loop, in CG
  int32_t* pending;         // device counter
  // Lanczos (krylov = 1): basis vectors V[j] at lv + j N (j < cg_max_iter),
  // per subdomain the recurrence coefficients la[j] (diagonal of T) and
  // lb[j] (lb[0] = |r_0|, lb[j] couples V[j-1] and V[j]), the coefficients
  // y of x = sum_j y_j V[j] (stride cg_max_iter + 1) and the extreme Ritz
  // values of the last run with at least one product
  int krylov;
  double *lv, *la, *lb, *ly, *ritz_lo, *ritz_hi;
  double *ld, *lz;          // per-subdomain scratch of the L D L^T solve
  // vector work by parts; per box the step's scalars between the passes
  // (CG: a and beta; Lanczos: alpha_j and beta_{j+1})
  PartMap P;
  double *ca, *cb;
};

void gn_to_x(const GnState& G, hipStream_t st);
void gn_from_x(const GnState& G, const double* x, hipStream_t st);
void gn_start(const GnState& G, hipStream_t st);
void gn_count(const GnState& G, hipStream_t st);
void gn_cg_start(const GnState& G, hipStream_t st);
void gn_cg_count(const GnState& G, hipStream_t st);
void gn_cg_dir(const GnState& G, hipStream_t st);
void gn_cg_update(const GnState& G, hipStream_t st);
void gn_lz_start(const GnState& G, hipStream_t st);
void gn_lz_update(const GnState& G, hipStream_t st);
void gn_lz_finish(const GnState& G, hipStream_t st);
void gn_update(const GnState& G, hipStream_t st);
void gn_after(const GnState& G, hipStream_t st);
// out += B_w^{-1} dx over every subdomain (w^b / sigma_b^2 per control entry)
void launch_add_bdiag(const PartMap& P, const uint8_t* cover, int weight_mode, const double sb[3],
                      const double* dx, double* out, hipStream_t st);

}  // namespace dd4dvar
