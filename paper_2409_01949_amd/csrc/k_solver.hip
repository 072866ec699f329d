// Krylov recurrences on the device: LSQR (Paige & Saunders 1982, damp = 0, no condition limit;
// the method's solver, Sec. 4.1) and CGLS.  All scalars live in a device SolveState and every
// scalar update runs in one workgroup, so the iteration loop needs no host round trip and can
// be captured in a hipGraph.  Norms are reduced in a fixed order (deterministic).  The stored
// u and v are kept unnormalised with their scales su = 1/beta and sv = 1/alpha; consumers apply
// the scale as they read.
#include "device.h"
#include "kernels.h"

namespace elmfb {

// Sum of n partials in a fixed order by one workgroup of 256 threads (valid in thread 0).
__device__ double reduce_partials(const double* __restrict__ red, int n, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += red[i];
  return block_sum256(v, sh);
}

__global__ void __launch_bounds__(256) k_sumsq(const double* __restrict__ x, int64_t n,
                                               double* __restrict__ red) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = x[i];
    acc += v * v;
  }
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = s;
}

template <int PREC>
__global__ void __launch_bounds__(256) k_sumsq_entries(const void* __restrict__ A, int64_t n,
                                                       double* __restrict__ red) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = load_entry<PREC>(A, i);
    acc += v * v;
  }
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_reduce_to(const double* __restrict__ red, int n,
                                                   double* __restrict__ out) {
  __shared__ double sh[4];
  const double s = reduce_partials(red, n, sh);
  if (threadIdx.x == 0) *out = s;
}

// bnorm = ||h||, beta = ||u||, su = 1/beta.
__global__ void __launch_bounds__(256) k_lsqr_init(SolveState* st, const double* red_b, int nb,
                                                   const double* red_u, int nu) {
  __shared__ double sh[4];
  const double sb = reduce_partials(red_b, nb, sh);
  const double su = reduce_partials(red_u, nu, sh);
  if (threadIdx.x == 0) {
    const double beta = sqrt(su);
    st->bnorm = sqrt(sb);
    st->beta = beta;
    st->su = beta > 0.0 ? 1.0 / beta : 0.0;
    st->alpha = 0.0;
    st->sv = 0.0;
    st->anorm = 0.0;
    st->itn = 0;
    st->istop = 0;
    st->done = 0;
    st->rel_l2 = -1.0;
  }
}

// alpha = ||A^T u||, phibar = beta, rhobar = alpha; stop at once if x0 is exact (istop 0).
// hist (may be NULL) receives (alpha_1, beta_1).
__global__ void __launch_bounds__(256) k_lsqr_init_alpha(SolveState* st, const double* red,
                                                         int n, double* hist) {
  __shared__ double sh[4];
  const double s = reduce_partials(red, n, sh);
  if (threadIdx.x == 0) {
    const double beta = st->beta;
    const double alpha = beta > 0.0 ? sqrt(s) : 0.0;
    if (hist) {
      hist[0] = alpha;
      hist[1] = beta;
    }
    st->alpha = alpha;
    st->sv = alpha > 0.0 ? 1.0 / alpha : 0.0;
    st->phibar = beta;
    st->rhobar = alpha;
    st->rnorm = beta;
    st->arnorm = alpha * beta;
    if (st->bnorm == 0.0) st->bnorm = beta;
    if (alpha * beta == 0.0) { st->istop = 0; st->done = 1; }
    if (st->iter_lim <= 0 && !st->done) { st->istop = 7; st->done = 1; }
  }
}

// x = x0 (or 0), w = v / alpha.
__global__ void k_init_xw(Geo g, const double* __restrict__ x0, double* __restrict__ x,
                          double* __restrict__ w, const double* __restrict__ v,
                          const SolveState* __restrict__ st) {
  const double sv = st->sv;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < g.n_phi;
       q += (int64_t)gridDim.x * blockDim.x) {
    x[q] = x0 ? x0[q] : 0.0;
    w[q] = v[q] * sv;
  }
}

// beta = ||A v - alpha u||; su = 1/beta; anorm = sqrt(anorm^2 + alpha^2 + beta^2).
// hist (may be NULL) receives beta_{i+1} of step i = itn + 1.
__global__ void __launch_bounds__(256) k_lsqr_beta(SolveState* st, const double* red, int n,
                                                   double* hist) {
  __shared__ double sh[4];
  if (st->done) return;
  const double s = reduce_partials(red, n, sh);
  if (threadIdx.x == 0) {
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
}

// alpha = ||A^T u - beta v||, sv = 1/alpha, then the plane rotation of this step.
// hist (may be NULL) receives alpha_{i+1} of step i = itn + 1.
__global__ void __launch_bounds__(256) k_lsqr_alpha(SolveState* st, const double* red, int n,
                                                    double* hist) {
  __shared__ double sh[4];
  if (st->done) return;
  const double s = reduce_partials(red, n, sh);
  if (threadIdx.x == 0) {
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
}

// x += t1 w ; w = v/alpha + t2 w ; partial ||x||^2.
__global__ void __launch_bounds__(256) k_lsqr_update(Geo g, double* __restrict__ x,
                                                     double* __restrict__ w,
                                                     const double* __restrict__ v,
                                                     const SolveState* __restrict__ st,
                                                     double* __restrict__ red) {
  __shared__ double sh[4];
  if (st->done) return;
  const double t1 = st->t1, t2 = st->t2, sv = st->sv;
  double acc = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < g.n_phi;
       q += (int64_t)gridDim.x * blockDim.x) {
    const double wq = w[q];
    const double xq = x[q] + t1 * wq;
    x[q] = xq;
    w[q] = v[q] * sv + t2 * wq;
    acc += xq * xq;
  }
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = s;
}

// Paige-Saunders stopping tests (conlim off).
__global__ void __launch_bounds__(256) k_lsqr_stop(SolveState* st, const double* red, int n) {
  __shared__ double sh[4];
  if (st->done) return;
  const double s = reduce_partials(red, n, sh);
  if (threadIdx.x == 0) {
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
}

// ---- CGLS
__global__ void __launch_bounds__(256) k_cgls_init(SolveState* st, const double* red_b, int nb,
                                                   const double* red_r, int nr,
                                                   const double* red_s, int ns, double anorm_f) {
  __shared__ double sh[4];
  const double sb = reduce_partials(red_b, nb, sh);
  const double sr = reduce_partials(red_r, nr, sh);
  const double ss = reduce_partials(red_s, ns, sh);
  if (threadIdx.x == 0) {
    st->bnorm = sqrt(sb);
    st->rnorm = sqrt(sr);
    st->gamma = ss;
    st->arnorm = sqrt(ss);
    st->anorm = anorm_f;
    st->itn = 0;
    st->istop = 0;
    st->done = 0;
    st->rel_l2 = -1.0;
    if (ss == 0.0) { st->istop = 0; st->done = 1; }
    if (st->iter_lim <= 0 && !st->done) { st->istop = 7; st->done = 1; }
  }
}

__global__ void __launch_bounds__(256) k_cgls_step_a(SolveState* st, const double* red, int n) {
  __shared__ double sh[4];
  if (st->done) return;
  const double s = reduce_partials(red, n, sh);
  if (threadIdx.x == 0) st->cg_a = st->gamma / s;
}

__global__ void k_cgls_update_x(Geo g, double* __restrict__ x, const double* __restrict__ p,
                                const SolveState* __restrict__ st) {
  if (st->done) return;
  const double a = st->cg_a;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < g.n_phi;
       q += (int64_t)gridDim.x * blockDim.x)
    x[q] = x[q] + a * p[q];
}

__global__ void __launch_bounds__(256) k_cgls_update_r(Geo g, double* __restrict__ r,
                                                       const double* __restrict__ t,
                                                       const SolveState* __restrict__ st,
                                                       double* __restrict__ red) {
  __shared__ double sh[4];
  if (st->done) return;
  const double a = st->cg_a;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n_rows + g.n_bc;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = r[i] - a * t[i];
    r[i] = v;
    acc += v * v;
  }
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_cgls_step_b(SolveState* st, const double* red_r, int nr,
                                                     const double* red_s, int ns) {
  __shared__ double sh[4];
  if (st->done) return;
  const double sr = reduce_partials(red_r, nr, sh);
  const double ss = reduce_partials(red_s, ns, sh);
  if (threadIdx.x == 0) {
    st->cg_b = ss / st->gamma;
    st->gamma = ss;
    const double rnorm = sqrt(sr);
    st->rnorm = rnorm;
    st->arnorm = sqrt(ss);
    st->itn += 1;
    int istop = 0;
    if (sqrt(ss) <= st->atol * st->anorm * rnorm) istop = 2;
    if (rnorm <= st->btol * st->bnorm) istop = 1;
    if (istop == 0 && st->itn >= st->iter_lim) istop = 7;
    if (istop != 0) { st->istop = istop; st->done = 1; }
  }
}

// p = s + b p   (runs even on the step that stopped: p is not used afterwards)
__global__ void k_cgls_update_p(Geo g, double* __restrict__ p, const double* __restrict__ s,
                                const SolveState* __restrict__ st) {
  const double b = st->cg_b;
  if (st->done) return;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < g.n_phi;
       q += (int64_t)gridDim.x * blockDim.x)
    p[q] = s[q] + b * p[q];
}

__global__ void k_axpy(double a, const double* __restrict__ x, double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = y[i] + a * x[i];
}

__global__ void k_copy(const double* __restrict__ src, double* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// ---- launchers
static dim3 grid_for(int64_t n) {
  int64_t nb = (n + 255) / 256;
  if (nb > 2048) nb = 2048;
  if (nb < 1) nb = 1;
  return dim3((unsigned)nb);
}

hipError_t launch_sumsq(const double* x, int64_t n, double* red, int n_wg, hipStream_t s) {
  hipLaunchKernelGGL(k_sumsq, dim3(n_wg), dim3(256), 0, s, x, n, red);
  return hipGetLastError();
}
hipError_t launch_sumsq_entries(int prec, const void* A, int64_t n, double* red, int n_wg,
                                hipStream_t s) {
  if (prec == ELMFB_FP32)
    hipLaunchKernelGGL(k_sumsq_entries<ELMFB_FP32>, dim3(n_wg), dim3(256), 0, s, A, n, red);
  else if (prec == ELMFB_BF16)
    hipLaunchKernelGGL(k_sumsq_entries<ELMFB_BF16>, dim3(n_wg), dim3(256), 0, s, A, n, red);
  else if (prec == ELMFB_FP16)
    hipLaunchKernelGGL(k_sumsq_entries<ELMFB_FP16>, dim3(n_wg), dim3(256), 0, s, A, n, red);
  else
    hipLaunchKernelGGL(k_sumsq_entries<ELMFB_FP64>, dim3(n_wg), dim3(256), 0, s, A, n, red);
  return hipGetLastError();
}
hipError_t launch_reduce_to(const double* red, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_to, dim3(1), dim3(256), 0, s, red, n, out);
  return hipGetLastError();
}
hipError_t launch_lsqr_init(SolveState* st, const double* red_b, int nb, const double* red_u,
                            int nu, hipStream_t s) {
  hipLaunchKernelGGL(k_lsqr_init, dim3(1), dim3(256), 0, s, st, red_b, nb, red_u, nu);
  return hipGetLastError();
}
hipError_t launch_lsqr_init_alpha(SolveState* st, const double* red, int n, double* hist,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_lsqr_init_alpha, dim3(1), dim3(256), 0, s, st, red, n, hist);
  return hipGetLastError();
}
hipError_t launch_init_xw(const Geo& g, const double* x0, double* x, double* w, const double* v,
                          const SolveState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_init_xw, grid_for(g.n_phi), dim3(256), 0, s, g, x0, x, w, v, st);
  return hipGetLastError();
}
hipError_t launch_lsqr_beta(SolveState* st, const double* red, int n, double* hist,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_lsqr_beta, dim3(1), dim3(256), 0, s, st, red, n, hist);
  return hipGetLastError();
}
hipError_t launch_lsqr_alpha(SolveState* st, const double* red, int n, double* hist,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_lsqr_alpha, dim3(1), dim3(256), 0, s, st, red, n, hist);
  return hipGetLastError();
}
hipError_t launch_lsqr_update(const Geo& g, double* x, double* w, const double* v,
                              const SolveState* st, double* red, int n_wg, hipStream_t s) {
  hipLaunchKernelGGL(k_lsqr_update, dim3(n_wg), dim3(256), 0, s, g, x, w, v, st, red);
  return hipGetLastError();
}
hipError_t launch_lsqr_stop(SolveState* st, const double* red, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_lsqr_stop, dim3(1), dim3(256), 0, s, st, red, n);
  return hipGetLastError();
}
hipError_t launch_cgls_init(SolveState* st, const double* red_b, int nb, const double* red_r,
                            int nr, const double* red_s, int ns, double anorm_f, hipStream_t s) {
  hipLaunchKernelGGL(k_cgls_init, dim3(1), dim3(256), 0, s, st, red_b, nb, red_r, nr, red_s, ns,
                     anorm_f);
  return hipGetLastError();
}
hipError_t launch_axpy(double a, const double* x, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, grid_for(n), dim3(256), 0, s, a, x, y, n);
  return hipGetLastError();
}
hipError_t launch_copy(const double* src, double* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, grid_for(n), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}
hipError_t launch_cgls_step_a(SolveState* st, const double* red, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_cgls_step_a, dim3(1), dim3(256), 0, s, st, red, n);
  return hipGetLastError();
}
hipError_t launch_cgls_update_x(const Geo& g, double* x, const double* p, const SolveState* st,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_cgls_update_x, grid_for(g.n_phi), dim3(256), 0, s, g, x, p, st);
  return hipGetLastError();
}
hipError_t launch_cgls_update_r(const Geo& g, double* r, const double* t, const SolveState* st,
                                double* red, int n_wg, hipStream_t s) {
  hipLaunchKernelGGL(k_cgls_update_r, dim3(n_wg), dim3(256), 0, s, g, r, t, st, red);
  return hipGetLastError();
}
hipError_t launch_cgls_step_b(SolveState* st, const double* red_r, int nr, const double* red_s,
                              int ns, hipStream_t s) {
  hipLaunchKernelGGL(k_cgls_step_b, dim3(1), dim3(256), 0, s, st, red_r, nr, red_s, ns);
  return hipGetLastError();
}
hipError_t launch_cgls_update_p(const Geo& g, double* p, const double* sv, const SolveState* st,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_cgls_update_p, grid_for(g.n_phi), dim3(256), 0, s, g, p, sv, st);
  return hipGetLastError();
}

// ---- CG on the assembled Gram blocks, G a = g (g = M^T h), optionally preconditioned by the
// block-Jacobi factors (z = R^{-1} R^{-T} r, R^T R = G_jj + lambda I): Hestenes-Stiefel CG with
// FP64 vectors and scalars.  gamma holds r.z (r.r without preconditioning), cg_a / cg_b the
// step sizes, bnorm ||g||, rnorm ||r||.

// Start: bnorm = ||g||, rnorm = ||r0||, gamma = r0.z0; done at once when r0 = 0 or iter_lim = 0.
__global__ void __launch_bounds__(256) k_gcg_init(SolveState* st, const double* red_b, int nb,
                                                  const double* red_r, int nr,
                                                  const double* red_z, int nz) {
  __shared__ double sh[4];
  const double bb = reduce_partials(red_b, nb, sh);
  const double rr = reduce_partials(red_r, nr, sh);
  const double rz = red_z ? reduce_partials(red_z, nz, sh) : rr;
  if (threadIdx.x == 0) {
    st->bnorm = sqrt(bb);
    st->rnorm = sqrt(rr);
    st->gamma = rz;
    st->cg_a = st->cg_b = 0.0;
    st->itn = 0;
    st->istop = 0;
    st->done = 0;
    st->rel_l2 = -1.0;
    if (rr == 0.0) st->done = 1;                                   // exact at the start
    else if (st->iter_lim <= 0) { st->istop = 7; st->done = 1; }
  }
}

// cg_a = gamma / (p . q); a breakdown (p . q <= 0: G not positive definite in this precision)
// stops with istop 3.
__global__ void __launch_bounds__(256) k_gcg_alpha(SolveState* st, const double* red, int n) {
  __shared__ double sh[4];
  if (st->done) return;
  const double pq = reduce_partials(red, n, sh);
  if (threadIdx.x == 0) {
    if (pq > 0.0) {
      st->cg_a = st->gamma / pq;
    } else {
      st->cg_a = 0.0;
      st->istop = 3;
      st->done = 1;
    }
  }
}

// a += cg_a p ; r -= cg_a q ; partial r . r.
__global__ void __launch_bounds__(256) k_gcg_update(Geo g, double* __restrict__ a,
                                                    double* __restrict__ r,
                                                    const double* __restrict__ p,
                                                    const double* __restrict__ q,
                                                    const SolveState* __restrict__ st,
                                                    double* __restrict__ red) {
  __shared__ double sh[4];
  if (st->done) return;
  const double al = st->cg_a;
  double acc = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < g.n_phi;
       t += (int64_t)gridDim.x * blockDim.x) {
    a[t] += al * p[t];
    const double rt = r[t] - al * q[t];
    r[t] = rt;
    acc += rt * rt;
  }
  const double sum = block_sum256(acc, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = sum;
}

// partial x . y (skipped once the solve is done; st may be NULL).
__global__ void __launch_bounds__(256) k_dot(const double* __restrict__ x,
                                             const double* __restrict__ y, int64_t n,
                                             const SolveState* __restrict__ st,
                                             double* __restrict__ red) {
  __shared__ double sh[4];
  if (st && st->done) return;
  double acc = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    acc += x[t] * y[t];
  const double sum = block_sum256(acc, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = sum;
}

// rnorm = ||r||, gamma' = r.z, cg_b = gamma'/gamma; stop on ||r|| <= btol ||g|| (istop 1) or
// the iteration limit (istop 7).
__global__ void __launch_bounds__(256) k_gcg_beta(SolveState* st, const double* red_r, int nr,
                                                  const double* red_z, int nz) {
  __shared__ double sh[4];
  if (st->done) return;
  const double rr = reduce_partials(red_r, nr, sh);
  const double rz = red_z ? reduce_partials(red_z, nz, sh) : rr;
  if (threadIdx.x == 0) {
    st->itn += 1;
    st->rnorm = sqrt(rr);
    st->cg_b = st->gamma > 0.0 ? rz / st->gamma : 0.0;
    st->gamma = rz;
    int istop = 0;
    if (st->rnorm <= st->btol * st->bnorm) istop = 1;
    else if (st->itn >= st->iter_lim) istop = 7;
    if (istop) { st->istop = istop; st->done = 1; }
  }
}

// p = z + cg_b p (p = z at the start: cg_b = 0 with init = 1).
__global__ void k_gcg_pupdate(Geo g, double* __restrict__ p, const double* __restrict__ z,
                              const SolveState* __restrict__ st, int init) {
  if (!init && st->done) return;
  const double b = init ? 0.0 : st->cg_b;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < g.n_phi;
       t += (int64_t)gridDim.x * blockDim.x)
    p[t] = z[t] + (init ? 0.0 : b * p[t]);
}

hipError_t launch_gcg_init(SolveState* st, const double* red_b, int nb, const double* red_r,
                           int nr, const double* red_z, int nz, hipStream_t s) {
  hipLaunchKernelGGL(k_gcg_init, dim3(1), dim3(256), 0, s, st, red_b, nb, red_r, nr, red_z, nz);
  return hipGetLastError();
}
hipError_t launch_gcg_alpha(SolveState* st, const double* red, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_gcg_alpha, dim3(1), dim3(256), 0, s, st, red, n);
  return hipGetLastError();
}
hipError_t launch_gcg_update(const Geo& g, double* a, double* r, const double* p, const double* q,
                             const SolveState* st, double* red, int n_wg, hipStream_t s) {
  hipLaunchKernelGGL(k_gcg_update, dim3(n_wg), dim3(256), 0, s, g, a, r, p, q, st, red);
  return hipGetLastError();
}
hipError_t launch_dot(const double* x, const double* y, int64_t n, const SolveState* st,
                      double* red, int n_wg, hipStream_t s) {
  hipLaunchKernelGGL(k_dot, dim3(n_wg), dim3(256), 0, s, x, y, n, st, red);
  return hipGetLastError();
}
hipError_t launch_gcg_beta(SolveState* st, const double* red_r, int nr, const double* red_z,
                           int nz, hipStream_t s) {
  hipLaunchKernelGGL(k_gcg_beta, dim3(1), dim3(256), 0, s, st, red_r, nr, red_z, nz);
  return hipGetLastError();
}
hipError_t launch_gcg_pupdate(const Geo& g, double* p, const double* z, const SolveState* st,
                              int init, hipStream_t s) {
  hipLaunchKernelGGL(k_gcg_pupdate, grid_for(g.n_phi), dim3(256), 0, s, g, p, z, st, init);
  return hipGetLastError();
}

}  // namespace elmfb
