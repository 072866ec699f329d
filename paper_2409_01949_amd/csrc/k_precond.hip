// Block-Jacobi preconditioning of the least-squares system from the diagonal Gram blocks.
//
// The random features of one subdomain are strongly redundant, which is the main source of
// the huge condition numbers of M (Sec. 5 "Conditioning and redundancy").  Right
// preconditioning with the block-diagonal R, R_j^T R_j = G_jj + lambda_j I (a Cholesky factor of
// each subdomain's Gram block, shifted by lambda_j = shift * trace(G_jj)/K), orthonormalises
// every subdomain's columns over its own support; LSQR then runs on M R^{-1} and the solution
// is x = R^{-1} y.  Factors are computed once in FP64 (one workgroup per block) and R^{-1} is
// stored explicitly together with its transpose, so both applications read memory
// contiguously.
#include "device.h"
#include "kernels.h"

namespace elmfb {

// One workgroup per block: Cholesky of G_jj + lambda I (upper factor, in work[j]), then the
// explicit inverse (rinv[j], rinvT[j]).  A failed factorisation is retried with a 100x larger
// shift; an empty block gets the identity.
__global__ void __launch_bounds__(256) k_bj_factor(Geo g, const double* __restrict__ G,
                                                   const int64_t* __restrict__ diag_off,
                                                   double shift, double* __restrict__ work,
                                                   double* __restrict__ rinv,
                                                   double* __restrict__ rinvT,
                                                   int32_t* __restrict__ nfail) {
  __shared__ int bad;
  __shared__ double lam_s;
  const int K = g.K;
  const int b = blockIdx.x;
  const double* Gj = G + diag_off[b];
  double* R = work + (int64_t)b * K * K;
  double* Ri = rinv + (int64_t)b * K * K;
  double* RiT = rinvT + (int64_t)b * K * K;
  if (threadIdx.x == 0) {
    double tr = 0.0;
    for (int i = 0; i < K; ++i) tr += Gj[i * K + i];
    lam_s = shift * tr / K;
  }
  __syncthreads();
  double lam = lam_s;
  bool ok = lam > 0.0;
  for (int attempt = 0; attempt < 8 && ok; ++attempt) {
    for (int e = threadIdx.x; e < K * K; e += 256) {
      const int i = e / K, j = e - i * K;
      R[e] = (j >= i) ? Gj[e] + (i == j ? lam : 0.0) : 0.0;
    }
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int k = 0; k < K; ++k) {
      if (threadIdx.x == 0) {
        const double d = R[k * K + k];
        if (!(d > 0.0)) bad = 1;
        R[k * K + k] = d > 0.0 ? sqrt(d) : 1.0;
      }
      __syncthreads();
      if (bad) break;
      const double dk = R[k * K + k];
      for (int j = k + 1 + threadIdx.x; j < K; j += 256) R[k * K + j] /= dk;
      __syncthreads();
      const int m = K - k - 1;            // trailing (m x m) upper triangle
      for (int e = threadIdx.x; e < m * m; e += 256) {
        const int i = k + 1 + e / m, j = k + 1 + (e - (e / m) * m);
        if (j >= i) R[i * K + j] -= R[k * K + i] * R[k * K + j];
      }
      __syncthreads();
    }
    if (!bad) break;
    lam *= 100.0;
    __syncthreads();
    if (threadIdx.x == 0 && attempt == 7) atomicAdd(nfail, 1);
    ok = attempt < 7;
  }
  __syncthreads();
  if (!ok || bad) {
    for (int e = threadIdx.x; e < K * K; e += 256) {
      const int i = e / K, j = e - i * K;
      const double v = (i == j) ? 1.0 : 0.0;
      R[e] = v; Ri[e] = v; RiT[e] = v;
    }
    return;
  }
  // inverse of the upper factor, one column per thread: R Ri = I
  for (int j = threadIdx.x; j < K; j += 256) {
    for (int i = j + 1; i < K; ++i) Ri[i * K + j] = 0.0;
    Ri[j * K + j] = 1.0 / R[j * K + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int m = i + 1; m <= j; ++m) s += R[i * K + m] * Ri[m * K + j];
      Ri[i * K + j] = -s / R[i * K + i];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < K * K; e += 256) {
    const int i = e / K, j = e - i * K;
    RiT[j * K + i] = Ri[e];
  }
}

// The three applications below are batched upper-triangular matrix-vector products, one K x K
// factor per subdomain.  Work is split into tasks of 32 output coefficients of one block; a
// workgroup of 256 threads takes a task at a time (grid-stride), thread t owns output
// coefficient t % 32 and sums every 8th term of its dot product (split t / 32), and the 8
// partial sums are added in a fixed order through LDS.  Consecutive threads read consecutive
// factor entries.
constexpr int kBjRows = 32;
constexpr int kBjSplit = 8;

__device__ __forceinline__ int bj_tasks(const Geo& g) {
  return g.n_blocks * ((g.K + kBjRows - 1) / kBjRows);
}

// y = R^{-1} (v * scale):  y_i = sum_{k >= i} Ri[i][k] v_k = sum_k T[k][i] v_k
__global__ void __launch_bounds__(256) k_bj_apply(Geo g, const double* __restrict__ rinvT,
                                                  const double* __restrict__ v,
                                                  const double* __restrict__ scale,
                                                  double* __restrict__ y,
                                                  const SolveState* __restrict__ st) {
  __shared__ double part[kBjSplit][kBjRows];
  if (st && st->done) return;
  const int K = g.K;
  const int per = (K + kBjRows - 1) / kBjRows;
  const double sc = scale ? *scale : 1.0;
  const int ro = threadIdx.x % kBjRows, sp = threadIdx.x / kBjRows;
  for (int task = blockIdx.x; task < bj_tasks(g); task += gridDim.x) {
    const int b = task / per, i = (task - b * per) * kBjRows + ro;
    const int64_t q0 = (int64_t)b * K;
    const double* T = rinvT + (int64_t)b * K * K;
    double s = 0.0;
    if (i < K)
      for (int k = i + sp; k < K; k += kBjSplit) s += T[(int64_t)k * K + i] * v[q0 + k];
    part[sp][ro] = s;
    __syncthreads();
    if (sp == 0 && i < K) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < kBjSplit; ++q) t += part[q][ro];
      y[q0 + i] = t * sc;
    }
    __syncthreads();
  }
}

// z = R^{-T} x:  z_k = sum_{i <= k} Ri[i][k] x_i, then the LSQR epilogue on v
// (v = z - beta sv v, partial ||v||^2) or a plain store (COL_STORE / COL_STORE_SQ).
__global__ void __launch_bounds__(256) k_bj_apply_t(Geo g, const double* __restrict__ rinv,
                                                    const double* __restrict__ x, int mode,
                                                    double* __restrict__ out,
                                                    const SolveState* __restrict__ st,
                                                    double* __restrict__ red) {
  __shared__ double part[kBjSplit][kBjRows];
  __shared__ double sh[4];
  if (st && st->done) return;
  const int K = g.K;
  const int per = (K + kBjRows - 1) / kBjRows;
  double coef_v = 0.0;
  bool keep = false;
  if (mode == COL_LSQR_V) {
    coef_v = st->beta * st->sv;
    keep = !(st->beta > 0.0);
  }
  const int ro = threadIdx.x % kBjRows, sp = threadIdx.x / kBjRows;
  double acc = 0.0;
  for (int task = blockIdx.x; task < bj_tasks(g); task += gridDim.x) {
    const int b = task / per, k = (task - b * per) * kBjRows + ro;
    const int64_t q0 = (int64_t)b * K;
    const double* Ri = rinv + (int64_t)b * K * K;
    double s = 0.0;
    if (k < K)
      for (int i = sp; i <= k; i += kBjSplit) s += Ri[(int64_t)i * K + k] * x[q0 + i];
    part[sp][ro] = s;
    __syncthreads();
    if (sp == 0 && k < K) {
      double z = 0.0;
#pragma unroll
      for (int q = 0; q < kBjSplit; ++q) z += part[q][ro];
      if (mode == COL_STORE) {
        out[q0 + k] = z;
      } else if (mode == COL_LSQR_V) {
        double vv = out[q0 + k];
        if (!keep) { vv = z - coef_v * vv; out[q0 + k] = vv; }
        acc += vv * vv;
      } else {
        out[q0 + k] = z;
        acc += z * z;
      }
    }
    __syncthreads();
  }
  if (mode != COL_STORE) {
    const double t = block_sum256(acc, sh);
    if (threadIdx.x == 0) red[blockIdx.x] = t;
  }
}

// x = x0 + R^{-1} y  (x0 may be NULL).  x0 and x may be the same vector: each element is read
// and then written by one thread, after every read of y.
__global__ void __launch_bounds__(256) k_bj_recover(Geo g, const double* __restrict__ rinvT,
                                                    const double* __restrict__ yv,
                                                    const double* x0, double* x) {
  __shared__ double part[kBjSplit][kBjRows];
  const int K = g.K;
  const int per = (K + kBjRows - 1) / kBjRows;
  const int ro = threadIdx.x % kBjRows, sp = threadIdx.x / kBjRows;
  for (int task = blockIdx.x; task < bj_tasks(g); task += gridDim.x) {
    const int b = task / per, i = (task - b * per) * kBjRows + ro;
    const int64_t q0 = (int64_t)b * K;
    const double* T = rinvT + (int64_t)b * K * K;
    double s = 0.0;
    if (i < K)
      for (int k = i + sp; k < K; k += kBjSplit) s += T[(int64_t)k * K + i] * yv[q0 + k];
    part[sp][ro] = s;
    __syncthreads();
    if (sp == 0 && i < K) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < kBjSplit; ++q) t += part[q][ro];
      x[q0 + i] = (x0 ? x0[q0 + i] : 0.0) + t;
    }
    __syncthreads();
  }
}

int bj_wg(const Geo& g) {
  const int tasks = g.n_blocks * ((g.K + kBjRows - 1) / kBjRows);
  return tasks < kRedBlocks ? tasks : kRedBlocks;
}

hipError_t launch_bj_factor(const Geo& g, const double* G, const int64_t* diag_off, double shift,
                            double* work, double* rinv, double* rinvT, int32_t* nfail,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_bj_factor, dim3(g.n_blocks), dim3(256), 0, s, g, G, diag_off, shift, work,
                     rinv, rinvT, nfail);
  return hipGetLastError();
}
hipError_t launch_bj_apply(const Geo& g, const double* rinvT, const double* v,
                           const double* scale, double* y, const SolveState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_bj_apply, dim3(bj_wg(g)), dim3(256), 0, s, g, rinvT, v, scale, y, st);
  return hipGetLastError();
}
hipError_t launch_bj_apply_t(const Geo& g, const double* rinv, const double* x, int mode,
                             double* out, const SolveState* st, double* red, hipStream_t s) {
  hipLaunchKernelGGL(k_bj_apply_t, dim3(bj_wg(g)), dim3(256), 0, s, g, rinv, x, mode, out, st,
                     red);
  return hipGetLastError();
}
hipError_t launch_bj_recover(const Geo& g, const double* rinvT, const double* y, const double* x0,
                             double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_bj_recover, dim3(bj_wg(g)), dim3(256), 0, s, g, rinvT, y, x0, x);
  return hipGetLastError();
}

}  // namespace elmfb
