// Block-Jacobi preconditioning for batches: per subdomain block b (K_b <= 128 features) the
// diagonal Gram block G_b = M_b^T M_b on the matrix cores, the upper Cholesky factor R_b of
// G_b + lambda_b I (lambda_b = shift trace(G_b)/K_b) and its inverse (column-packed), then the
// preconditioned matrix M_b R_b^{-1} formed once on the matrix cores, so that preconditioned
// Krylov steps cost the same as plain ones.  Same preconditioner as for single problems (the
// random features of one subdomain are the main source of the condition numbers of M, Sec. 5),
// with the ragged K of the instances.
#include "device.h"
#include "kernels.h"

namespace elmfb {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kGdStage = 32;   // points per LDS stage

// G_b[i][j] for 16 x 16 tiles with I <= J (the factorisation reads the upper triangle only),
// FP64 inputs and accumulation on v_mfma_f64_16x16x4_f64.  One workgroup per block, the
// block's points staged 32 at a time ([K][32], feature-major).
__global__ void __launch_bounds__(256) k_bt_gram_diag(const Geo* __restrict__ geos,
                                                      const DevBlock* __restrict__ blocks,
                                                      const double* __restrict__ A,
                                                      const int64_t* __restrict__ goff,
                                                      double* __restrict__ G) {
  constexpr int STR = kGdStage + 1;
  __shared__ double X[kBatchMaxK * STR];
  const DevBlock B = blocks[blockIdx.x];
  const int K = geos[B.inst].K;
  const int Kp = (K + 15) & ~15;
  const int nT = Kp / 16;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const double* Ab = A + B.a_off;
  const int n = B.n;
  d4_t acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = d4_t{0, 0, 0, 0};
  for (int p0 = 0; p0 < n; p0 += kGdStage) {
    for (int e = threadIdx.x; e < Kp * kGdStage; e += 256) {
      const int k = e / kGdStage, c = e - (e / kGdStage) * kGdStage;
      X[k * STR + c] = (k < K && p0 + c < n) ? Ab[(int64_t)k * B.ld + p0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int t = wid + 4 * i;
      if (t < nT * nT) {
        const int I = t / nT, J = t - (t / nT) * nT;
        if (I <= J) {
          const double* xr = X + (I * 16 + li) * STR;
          const double* yr = X + (J * 16 + li) * STR;
#pragma unroll
          for (int q = 0; q < kGdStage; q += 4)
            acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[q + lq], yr[q + lq], acc[i], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // v_mfma_f64_16x16x4_f64 accumulator: lane holds column li, rows lq + 4 v
  double* Gb = G + goff[blockIdx.x];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int t = wid + 4 * i;
    if (t < nT * nT) {
      const int I = t / nT, J = t - (t / nT) * nT;
      if (I <= J) {
        const int col = J * 16 + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = I * 16 + lq + 4 * v;
          if (row < K && col < K) Gb[(int64_t)row * K + col] = acc[i][v];
        }
      }
    }
  }
}

// One workgroup per block: Cholesky of G_b + lambda I (upper factor, in work), the inverse
// Ri = R^{-1} (one column per thread, into G_b's storage once the factor exists), then the
// column-packed copy (Ri[i][k], i <= k, at k(k+1)/2 + i).  A failed factorisation is retried with a 100x larger shift up to 8 times; after
// that, or for an all-zero block, the block gets the identity and nfail counts it.
__global__ void __launch_bounds__(256) k_bt_bj_factor(const Geo* __restrict__ geos,
                                                      const DevBlock* __restrict__ blocks,
                                                      double* __restrict__ G,
                                                      const int64_t* __restrict__ goff,
                                                      double* __restrict__ work,
                                                      const int64_t* __restrict__ foff,
                                                      double shift, double* __restrict__ rc,
                                                      int32_t* __restrict__ nfail) {
  __shared__ int bad;
  __shared__ double lam_s;
  const DevBlock B = blocks[blockIdx.x];
  const int K = geos[B.inst].K;
  double* Gj = G + goff[blockIdx.x];
  double* R = work + goff[blockIdx.x];
  double* Pc = rc + foff[blockIdx.x];
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
      const int m = K - k - 1;
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
  const bool ident = !ok || bad;
  if (!ident) {
    // Ri (upper) into Gj's storage: R Ri = I, one column per thread
    for (int j = threadIdx.x; j < K; j += 256) {
      Gj[j * K + j] = 1.0 / R[j * K + j];
      for (int i = j - 1; i >= 0; --i) {
        double s = 0.0;
        for (int m = i + 1; m <= j; ++m) s += R[i * K + m] * Gj[m * K + j];
        Gj[i * K + j] = -s / R[i * K + i];
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < K * K; e += 256) {
    const int i = e / K, k = e - i * K;
    if (i <= k) {
      const double v = ident ? (i == k ? 1.0 : 0.0) : Gj[i * K + k];
      Pc[(int64_t)k * (k + 1) / 2 + i] = v;
    }
  }
}

// Fold the preconditioner into the matrix: Mhat_b = M_b R_b^{-1}, i.e. in the feature-major
// block layout Mhat_b[k'][p] = sum_{k <= k'} Ri[k][k'] M_b[k][p] (R^{-T} times the block), on
// v_mfma_f64_16x16x4_f64 (K <= 256).  One workgroup per 64-point run of a block: the four waves own output
// row tiles (16 features each) w, w + 4, ... and the four 16-point column tiles; the contraction
// over k runs in LDS stages of 16 (R^{-T} columns from the column-packed factor, M_b rows), and
// tiles entirely above the diagonal are skipped.  The FP64 result goes to Mhat (if not NULL) and,
// rounded to nearest even, to the low-precision copy.
constexpr int kFoldK = 16;
constexpr int kFoldP = 64;

template <int LO, bool FULL, int TPW>
__global__ void __launch_bounds__(256) k_bt_fold(const Geo* __restrict__ geos,
                                                 const DevBlock* __restrict__ blocks,
                                                 const Tile* __restrict__ ftiles,
                                                 const double* __restrict__ A,
                                                 const double* __restrict__ rc,
                                                 const int64_t* __restrict__ foff,
                                                 double* __restrict__ Ahat,
                                                 void* __restrict__ Ahat_lo) {
  constexpr int KMAX = 64 * TPW;                  // TPW row tiles of 16 features per wave
  __shared__ double Rt[KMAX][kFoldK + 1];         // Rt[k'][kk] = Ri[k0 + kk][k']
  __shared__ double At[kFoldK][kFoldP + 1];       // At[kk][c] = M_b[k0 + kk][p0 + c]
  const Tile t = ftiles[blockIdx.x];
  const DevBlock B = blocks[t.blk];
  const int K = geos[B.inst].K;
  const int n = B.n, p0 = t.p0;
  const double* Ab = A + B.a_off;
  // FULL: R^{-1} stored K x K row-major per block (single problems); else column-packed
  const double* Rb = FULL ? rc + (int64_t)t.blk * K * K : rc + foff[t.blk];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int nT = (K + 15) >> 4;
  d4_t acc[TPW][4];
#pragma unroll
  for (int a = 0; a < TPW; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4_t{0, 0, 0, 0};
  for (int k0 = 0; k0 < K; k0 += kFoldK) {
    for (int e = threadIdx.x; e < KMAX * kFoldK; e += 256) {
      const int kp = e / kFoldK, kk = e - (e / kFoldK) * kFoldK;
      const int k = k0 + kk;
      const int64_t ri = FULL ? (int64_t)k * K + kp : (int64_t)kp * (kp + 1) / 2 + k;
      Rt[kp][kk] = (kp < K && k <= kp) ? Rb[ri] : 0.0;
    }
    for (int e = threadIdx.x; e < kFoldK * kFoldP; e += 256) {
      const int kk = e / kFoldP, c = e - (e / kFoldP) * kFoldP;
      const int k = k0 + kk, p = p0 + c;
      At[kk][c] = (k < K && p < n) ? Ab[(int64_t)k * B.ld + p] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < TPW; ++a) {
      const int I = wid + 4 * a;
      if (I < nT && 16 * I + 15 >= k0) {     // rows k' < k0 of R^{-T} vanish on this stage
#pragma unroll
        for (int b = 0; b < 4; ++b) {
#pragma unroll
          for (int q = 0; q < kFoldK; q += 4)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(Rt[16 * I + li][q + lq],
                                                             At[q + lq][16 * b + li], acc[a][b],
                                                             0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // accumulator of v_mfma_f64_16x16x4_f64: lane holds column li, rows lq + 4 v
#pragma unroll
  for (int a = 0; a < TPW; ++a) {
    const int I = wid + 4 * a;
    if (I >= nT) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int p = p0 + 16 * b + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int kp = 16 * I + lq + 4 * v;
        if (kp < K && p < n) {
          const int64_t o = B.a_off + (int64_t)kp * B.ld + p;
          const double val = acc[a][b][v];
          if (Ahat) Ahat[o] = val;
          if constexpr (LO == ELMFB_FP32) static_cast<float*>(Ahat_lo)[o] = (float)val;
          if constexpr (LO == ELMFB_BF16) static_cast<uint16_t*>(Ahat_lo)[o] = f64_to_bf16_rne(val);
          if constexpr (LO == ELMFB_FP16) static_cast<uint16_t*>(Ahat_lo)[o] = f64_to_fp16_rne(val);
        }
      }
    }
  }
}

hipError_t launch_bt_fold(int lo_prec, bool full, int kmax, const Geo* geos,
                          const DevBlock* blocks, const Tile* ftiles, int64_t n_ftiles,
                          const double* A, const double* rc, const int64_t* foff, double* Ahat,
                          void* Ahat_lo, hipStream_t s) {
  if (n_ftiles == 0) return hipSuccess;
  if (kmax > 256) return hipErrorInvalidValue;
  const dim3 grid((unsigned)n_ftiles), blk(256);
#define FOLD(L, F, T)                                                                            \
  hipLaunchKernelGGL((k_bt_fold<L, F, T>), grid, blk, 0, s, geos, blocks, ftiles, A, rc, foff,    \
                     Ahat, Ahat_lo)
#define FOLD_T(L, F) do { if (kmax > 128) FOLD(L, F, 4); else FOLD(L, F, 2); } while (0)
  if (lo_prec == ELMFB_FP32) { if (full) FOLD_T(ELMFB_FP32, true); else FOLD_T(ELMFB_FP32, false); }
  else if (lo_prec == ELMFB_BF16) { if (full) FOLD_T(ELMFB_BF16, true); else FOLD_T(ELMFB_BF16, false); }
  else if (lo_prec == ELMFB_FP16) { if (full) FOLD_T(ELMFB_FP16, true); else FOLD_T(ELMFB_FP16, false); }
  else { if (full) FOLD_T(-1, true); else FOLD_T(-1, false); }
#undef FOLD_T
#undef FOLD
  return hipGetLastError();
}

hipError_t launch_bt_gram_diag(const Geo* geos, const DevBlock* blocks, int64_t n_blocks,
                               const double* A, const int64_t* goff, double* G, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bt_gram_diag, dim3((unsigned)n_blocks), dim3(256), 0, s, geos, blocks, A,
                     goff, G);
  return hipGetLastError();
}

hipError_t launch_bt_bj_factor(const Geo* geos, const DevBlock* blocks, int64_t n_blocks,
                               double* G, const int64_t* goff, double* work, const int64_t* foff,
                               double shift, double* rc, int32_t* nfail, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bt_bj_factor, dim3((unsigned)n_blocks), dim3(256), 0, s, geos, blocks, G,
                     goff, work, foff, shift, rc, nfail);
  return hipGetLastError();
}

}  // namespace elmfb
