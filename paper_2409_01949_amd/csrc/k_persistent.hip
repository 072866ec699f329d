// LSQR (Sec. 3: the method's least-squares solver, Paige-Saunders recurrences) for systems that
// fit in one compute unit: one workgroup of 1024 threads runs whole iterations, with u, v, w,
// x and the per-block-point partials t_j held in LDS and the FP64 matrix read from global memory
// (it stays in the CU's caches between iterations).  A step here costs its arithmetic and a few
// workgroup barriers instead of the ~9 kernel launches per step of the multi-workgroup path,
// which dominate when the system holds only thousands of entries (the damped oscillator of
// Sec. 5.1).
//
// The step is the same one the multi-workgroup path takes, on the same stored (unnormalised)
// u and v with their scales su = 1/beta and sv = 1/alpha:
//   t_j[p] = sum_k M_j[k][p] v[q0_j + k] sv                    (per block point)
//   u_r    = sum over covering blocks of t_j[p_j(r)] - alpha su u_r      (collocation rows)
//   u_b    = sum_q B[b][q] v[q] sv - alpha su u_b              (soft-constraint rows)
//   beta   = ||u||, x_q = sum_p M_j[k][p] u[r(p)] su + sum_b B[b][q] u_b su,
//   v      = x - beta sv v, alpha = ||v||, the plane rotation, x += t1 w, w = v sv + t2 w,
// then the stopping tests.  Each reduction is a fixed-order wavefront butterfly and a
// fixed-order sum of the 16 wavefront partials that every thread reads, so every thread holds
// the same scalar state and the result is deterministic.
#include "device.h"
#include "kernels.h"

namespace elmfb {

namespace {

constexpr int kPThreads = 1024;
constexpr int kPWaves = kPThreads / 64;

// Fixed-order sum over the workgroup; every thread returns the same value.  slot holds
// kPWaves doubles and must not be rewritten before every thread has passed a later barrier.
__device__ __forceinline__ double wg_sum(double v, double* slot) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) slot[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kPWaves; ++i) s += slot[i];
  return s;
}

// Global row of point p of block B (box row-major, y fastest).
__device__ __forceinline__ int64_t block_row(const Geo& g, const DevBlock& B, int p) {
  const int px = p / B.ny, py = p - px * B.ny;
  return (int64_t)(B.ix0 + px) * g.ny + (B.iy0 + py);
}

}  // namespace

size_t persistent_lds_bytes(const Geo& g, int64_t n_pts) {
  const int64_t nrt = g.n_rows + g.n_bc;
  return (size_t)(8 * (nrt + 3 * g.n_phi + n_pts + 3 * kPWaves) + 4 * n_pts);
}

__global__ void __launch_bounds__(kPThreads) k_lsqr_persistent(
    Geo g, const DevBlock* __restrict__ blocks, const int32_t* __restrict__ cov,
    const double* __restrict__ A, const double* __restrict__ bc, double* __restrict__ u_g,
    double* __restrict__ v_g, double* __restrict__ w_g, double* __restrict__ x_g,
    SolveState* st, double* __restrict__ hist, int n_iter, int64_t n_pts) {
  if (st->done) return;
  extern __shared__ double lds[];
  const int64_t nrt = g.n_rows + g.n_bc;
  const int64_t n_phi = g.n_phi;
  double* u = lds;
  double* v = u + nrt;
  double* w = v + n_phi;
  double* x = w + n_phi;
  double* tp = x + n_phi;
  double* slot = tp + n_pts;    // 3 x kPWaves reduction slots
  int32_t* pblk = reinterpret_cast<int32_t*>(slot + 3 * kPWaves);
  const int tid = threadIdx.x;
  const int K = g.K;

  for (int64_t i = tid; i < nrt; i += kPThreads) u[i] = u_g[i];
  for (int64_t i = tid; i < n_phi; i += kPThreads) {
    v[i] = v_g[i];
    w[i] = w_g[i];
    x[i] = x_g[i];
  }
  for (int j = tid; j < g.n_blocks; j += kPThreads) {
    const DevBlock& B = blocks[j];
    for (int p = 0; p < B.n; ++p) pblk[B.p_off + p] = j;
  }

  // scalar state: the same copy in every thread
  double alpha = st->alpha, beta = st->beta, su = st->su, sv = st->sv;
  double rhobar = st->rhobar, phibar = st->phibar, anorm = st->anorm;
  double xnorm = st->xnorm, rnorm = st->rnorm, arnorm = st->arnorm, t1 = st->t1, t2 = st->t2;
  const double bnorm = st->bnorm, atol = st->atol, btol = st->btol;
  const int iter_lim = st->iter_lim;
  int itn = st->itn, istop = st->istop, done = 0;

  // threads per column of M^T u: the largest power of two with n_phi * T <= 1024, at most 64
  int T = 1;
  while (T < 64 && (int64_t)(2 * T) * n_phi <= kPThreads) T *= 2;
  const int sub = tid & (T - 1);
  __syncthreads();

  for (int it = 0; it < n_iter && !done; ++it) {
    // t_j[p] = sum_k M_j[k][p] v[q0_j + k] sv
    for (int64_t f = tid; f < n_pts; f += kPThreads) {
      const DevBlock& B = blocks[pblk[f]];
      const int p = (int)(f - B.p_off);
      const double* a = A + B.a_off + p;
      const double* vb = v + B.q0;
      const int ld = B.ld;
      double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
      int k = 0;
      for (; k + 4 <= K; k += 4) {
        const double a0 = a[(int64_t)k * ld], a1 = a[(int64_t)(k + 1) * ld];
        const double a2 = a[(int64_t)(k + 2) * ld], a3 = a[(int64_t)(k + 3) * ld];
        c0 += a0 * vb[k];
        c1 += a1 * vb[k + 1];
        c2 += a2 * vb[k + 2];
        c3 += a3 * vb[k + 3];
      }
      for (; k < K; ++k) c0 += a[(int64_t)k * ld] * vb[k];
      tp[f] = ((c0 + c1) + (c2 + c3)) * sv;
    }
    __syncthreads();

    // u = M v sv - alpha su u over the collocation rows, then the soft-constraint rows
    const double coef_u = alpha * su;
    double acc = 0.0;
    for (int64_t r = tid; r < g.n_rows; r += kPThreads) {
      const int ix = (int)(r / g.ny), iy = (int)(r - (int64_t)ix * g.ny);
      double y = 0.0;
      for (int l = 0; l < g.n_levels; ++l) {
        const int jx0 = cov[g.cov_off[l][0] + 2 * ix], jx1 = cov[g.cov_off[l][0] + 2 * ix + 1];
        const int jy0 = cov[g.cov_off[l][1] + 2 * iy], jy1 = cov[g.cov_off[l][1] + 2 * iy + 1];
        const int Jy = g.J[l][1];
        for (int jx = jx0; jx <= jx1; ++jx)
          for (int jy = jy0; jy <= jy1; ++jy) {
            const DevBlock& B = blocks[g.bbase[l] + jx * Jy + jy];
            y += tp[B.p_off + (ix - B.ix0) * B.ny + (iy - B.iy0)];
          }
      }
      const double un = y - coef_u * u[r];
      u[r] = un;
      acc += un * un;
    }
    const int wave = tid >> 6, lane = tid & 63;
    if (wave < g.n_bc) {
      double d = 0.0;
      for (int64_t q = lane; q < n_phi; q += 64) d += bc[(int64_t)wave * n_phi + q] * v[q];
      d = wave_sum(d) * sv;
      if (lane == 0) {
        const double un = d - coef_u * u[g.n_rows + wave];
        u[g.n_rows + wave] = un;
        acc += un * un;
      }
    }
    beta = sqrt(wg_sum(acc, slot));
    if (tid == 0 && hist && itn + 1 < kHistCap) hist[2 * (itn + 1) + 1] = beta;
    if (beta > 0.0) {
      su = 1.0 / beta;
      anorm = sqrt(anorm * anorm + alpha * alpha + beta * beta);
    }

    // v = M^T u su - beta sv v (v and alpha stay when beta == 0)
    const double coef_v = beta * sv;
    const bool keep = !(beta > 0.0);
    acc = 0.0;
    const int64_t qspan = (n_phi + (kPThreads / T) - 1) / (kPThreads / T) * (kPThreads / T);
    for (int64_t q = tid / T; q < qspan; q += kPThreads / T) {
      // all T threads of a column take this branch together, so the butterfly below reads
      // only active lanes
      if (q < n_phi) {
        const int b = (int)(q / K), k = (int)(q - (int64_t)b * K);
        const DevBlock& B = blocks[b];
        const double* a = A + B.a_off + (int64_t)k * B.ld;
        double s0 = 0.0, s1 = 0.0;
        int p = sub;
        for (; p + T < B.n; p += 2 * T) {
          s0 += a[p] * u[block_row(g, B, p)];
          s1 += a[p + T] * u[block_row(g, B, p + T)];
        }
        if (p < B.n) s0 += a[p] * u[block_row(g, B, p)];
        double s = s0 + s1;
        for (int o = T >> 1; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
        double xq = s * su;
        for (int r = 0; r < g.n_bc; ++r) xq += bc[(int64_t)r * n_phi + q] * (u[g.n_rows + r] * su);
        if (sub == 0) {
          double vq = v[q];
          if (!keep) {
            vq = xq - coef_v * vq;
            v[q] = vq;
          }
          acc += vq * vq;
        }
      }
    }
    const double sa = wg_sum(acc, slot + kPWaves);
    if (beta > 0.0) {
      alpha = sqrt(sa);
      if (alpha > 0.0) sv = 1.0 / alpha;
    }
    if (tid == 0 && hist && itn + 1 < kHistCap) hist[2 * (itn + 1)] = alpha;
    const double rho = sqrt(rhobar * rhobar + beta * beta);
    const double c = rhobar / rho, sn = beta / rho;
    const double theta = sn * alpha;
    rhobar = -c * alpha;
    const double phi = c * phibar;
    phibar = sn * phibar;
    t1 = phi / rho;
    t2 = -theta / rho;
    rnorm = phibar;
    arnorm = alpha * fabs(c) * phibar;

    // x += t1 w, w = v sv + t2 w
    acc = 0.0;
    for (int64_t q = tid; q < n_phi; q += kPThreads) {
      const double wq = w[q];
      const double xq = x[q] + t1 * wq;
      x[q] = xq;
      w[q] = v[q] * sv + t2 * wq;
      acc += xq * xq;
    }
    xnorm = sqrt(wg_sum(acc, slot + 2 * kPWaves));
    itn += 1;

    // stopping tests (conlim off)
    const double eps = 2.220446049250313e-16;
    const double test1 = rnorm / bnorm;
    const double test2 = arnorm / (anorm * rnorm + eps);
    const double tt = test1 / (1.0 + anorm * xnorm / bnorm);
    const double rtol = btol + atol * anorm * xnorm / bnorm;
    int is = 0;
    if (1.0 + test2 <= 1.0) is = 5;
    if (1.0 + tt <= 1.0) is = 4;
    if (test2 <= atol) is = 2;
    if (test1 <= rtol) is = 1;
    if (is == 0 && itn >= iter_lim) is = 7;
    if (is != 0) {
      istop = is;
      done = 1;
    }
  }
  __syncthreads();

  for (int64_t i = tid; i < nrt; i += kPThreads) u_g[i] = u[i];
  for (int64_t i = tid; i < n_phi; i += kPThreads) {
    v_g[i] = v[i];
    w_g[i] = w[i];
    x_g[i] = x[i];
  }
  if (tid == 0) {
    st->alpha = alpha;
    st->beta = beta;
    st->su = su;
    st->sv = sv;
    st->rhobar = rhobar;
    st->phibar = phibar;
    st->anorm = anorm;
    st->xnorm = xnorm;
    st->rnorm = rnorm;
    st->arnorm = arnorm;
    st->t1 = t1;
    st->t2 = t2;
    st->itn = itn;
    st->istop = istop;
    st->done = done;
  }
}

hipError_t launch_lsqr_persistent(const Geo& g, const DevBlock* blocks, const int32_t* cov,
                                  const double* A, const double* bc, double* u, double* v,
                                  double* w, double* x, SolveState* st, double* hist, int n_iter,
                                  int64_t n_pts, hipStream_t s) {
  const size_t lds = persistent_lds_bytes(g, n_pts);
  if (lds > kPersistMaxLds || n_iter <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lsqr_persistent, dim3(1), dim3(kPThreads), lds, s, g, blocks, cov, A, bc,
                     u, v, w, x, st, hist, n_iter, n_pts);
  return hipGetLastError();
}

}  // namespace elmfb
