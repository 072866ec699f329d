// The scalar steps of LSQR (Paige & Saunders 1982, damp 0; the method's solver, Sec. 4.1) on a
// device SolveState, given the reduced sum of their norm partials, and the last-workgroup
// reduction that lets the kernel producing those partials run them itself: every workgroup
// writes its partial, then counts itself in; the workgroup that arrives last sums all partials
// in the fixed order of a separate reduction kernel and applies the scalar step, so the result
// is bit-identical to launching that kernel, one launch fewer per step.
#pragma once

#include "device.h"

namespace elmfb {

// beta = sqrt(s) = ||A v - alpha u||; su = 1/beta; anorm = sqrt(anorm^2 + alpha^2 + beta^2).
// hist (may be NULL) receives beta_{i+1} of step i = itn + 1.
__device__ inline void lsqr_beta_scalar(SolveState* st, double s, double* hist) {
  const double beta = sqrt(s);
  st->beta = beta;
  const int i = st->itn + 1;
  if (hist && i < kHistCap) hist[2 * i + 1] = beta;
  if (beta > 0.0) {
    st->su = 1.0 / beta;
    const double a = st->alpha;
    st->anorm = sqrt(st->anorm * st->anorm + a * a + beta * beta);
  }
}

// alpha = sqrt(s) = ||A^T u - beta v||, sv = 1/alpha, then the plane rotation of this step.
// hist (may be NULL) receives alpha_{i+1} of step i = itn + 1.
__device__ inline void lsqr_alpha_scalar(SolveState* st, double s, double* hist) {
  const double beta = st->beta;
  double alpha = st->alpha;
  if (beta > 0.0) {
    alpha = sqrt(s);
    st->alpha = alpha;
    if (alpha > 0.0) st->sv = 1.0 / alpha;
  }
  const int i = st->itn + 1;
  if (hist && i < kHistCap) hist[2 * i] = alpha;
  const double rhobar = st->rhobar;
  const double rho = sqrt(rhobar * rhobar + beta * beta);
  const double c = rhobar / rho, sn = beta / rho;
  const double theta = sn * alpha;
  st->rhobar = -c * alpha;
  const double phi = c * st->phibar;
  const double phibar = sn * st->phibar;
  st->phibar = phibar;
  st->t1 = phi / rho;
  st->t2 = -theta / rho;
  st->rnorm = phibar;
  st->arnorm = alpha * fabs(c) * phibar;
}

// xnorm = sqrt(s); the Paige-Saunders stopping tests (conlim off).
__device__ inline void lsqr_stop_scalar(SolveState* st, double s) {
  const double eps = 2.220446049250313e-16;
  const double xnorm = sqrt(s);
  st->xnorm = xnorm;
  st->itn += 1;
  const double anorm = st->anorm, rnorm = st->rnorm, bnorm = st->bnorm;
  const double test1 = rnorm / bnorm;
  const double test2 = st->arnorm / (anorm * rnorm + eps);
  const double t1 = test1 / (1.0 + anorm * xnorm / bnorm);
  const double rtol = st->btol + st->atol * anorm * xnorm / bnorm;
  int istop = 0;
  if (1.0 + test2 <= 1.0) istop = 5;
  if (1.0 + t1 <= 1.0) istop = 4;
  if (test2 <= st->atol) istop = 2;
  if (test1 <= rtol) istop = 1;
  if (istop == 0 && st->itn >= st->iter_lim) istop = 7;
  if (istop != 0) { st->istop = istop; st->done = 1; }
}

// Called by every thread of every workgroup after thread 0 has written the workgroup's partial:
// true in the workgroup that arrives last (which also resets the counter for the next launch).
__device__ inline bool last_workgroup(unsigned int* counter) {
  __shared__ int last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();                                     // this workgroup's partial is visible
    const unsigned int t = atomicAdd(counter, 1u);
    last = t == gridDim.x - 1;
    if (last) atomicExch(counter, 0u);
  }
  __syncthreads();
  if (last) __threadfence();
  return last;
}

// The same sum as reduce_partials (valid in thread 0), reading the partials at device scope so
// that values written by other workgroups of this launch are seen.
__device__ inline double sum_partials_device(const double* red, int n, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256)
    v += __hip_atomic_load(red + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return block_sum256(v, sh);
}

}  // namespace elmfb
