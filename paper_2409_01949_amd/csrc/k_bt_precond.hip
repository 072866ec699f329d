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

// One workgroup of 1,024 threads per block, everything in LDS (two packed upper triangles of
// K(K+1)/2 doubles, (i, j) at j(j+1)/2 + i, and one row vector): the upper Cholesky factor R of
// G_b + lambda I by right-looking elimination (step k: the pivot row R[k][j] = G'[k][j] / sqrt of
// the pivot, kept in the row vector, then the trailing update R[i][j] -= R[k][i] R[k][j] for
// k < i <= j), then X = R^{-1} by the same elimination from the bottom row (row i of X is row i of
// the running right-hand side over R[i][i]; rows r < i then lose R[r][i] X[i][j]), written out in
// the same column-packed layout.  Each update is spread as 8 threads per column j over its rows,
// which are contiguous in the packed layout, so a thread's updates are independent of each
// other.  A failed factorisation is retried with a 100x larger shift up to 8 times; after that,
// or for an all-zero block, the block gets the identity and nfail counts it.
constexpr int kFacThreads = 1024;

__global__ void __launch_bounds__(kFacThreads) k_bt_bj_factor(const Geo* __restrict__ geos,
                                                              const DevBlock* __restrict__ blocks,
                                                              const double* __restrict__ G,
                                                              const int64_t* __restrict__ goff,
                                                              const int64_t* __restrict__ foff,
                                                              double shift,
                                                              double* __restrict__ rc,
                                                              int32_t* __restrict__ nfail) {
  extern __shared__ double lds[];
  __shared__ double part[kFacThreads / 64];
  __shared__ double row[kBatchMaxK];
  const DevBlock B = blocks[blockIdx.x];
  const int K = geos[B.inst].K;
  const int np = K * (K + 1) / 2;
  double* Rp = lds;
  double* Xp = lds + np;
  const double* Gj = G + goff[blockIdx.x];
  double* Pc = rc + foff[blockIdx.x];
  const int t = threadIdx.x, tc = t >> 3, ts = t & 7;   // column offset, row phase
  // trace of G_b
  double tr = 0.0;
  for (int i = t; i < K; i += kFacThreads) tr += Gj[(int64_t)i * K + i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o);
  if ((t & 63) == 0) part[t >> 6] = tr;
  __syncthreads();
  tr = 0.0;
  for (int w = 0; w < kFacThreads / 64; ++w) tr += part[w];
  double lam = shift * tr / K;
  bool ok = lam > 0.0;
  bool bad = true;
  for (int attempt = 0; attempt < 8 && ok; ++attempt) {
    for (int e = t; e < K * K; e += kFacThreads) {
      const int i = e / K, j = e - (e / K) * K;
      if (i <= j) Rp[j * (j + 1) / 2 + i] = Gj[e] + (i == j ? lam : 0.0);
    }
    __syncthreads();
    bad = false;
    for (int k = 0; k < K; ++k) {
      const double d = Rp[k * (k + 1) / 2 + k];
      if (!(d > 0.0)) { bad = true; break; }    // every thread reads the same value
      const double rk = sqrt(d);
      for (int j = k + 1 + t; j < K; j += kFacThreads) {
        const double v = Rp[j * (j + 1) / 2 + k] / rk;
        Rp[j * (j + 1) / 2 + k] = v;
        row[j] = v;
      }
      __syncthreads();
      if (t == 0) Rp[k * (k + 1) / 2 + k] = rk;
      const int j = k + 1 + tc;
      if (j < K) {
        double* cj = Rp + j * (j + 1) / 2;
        const double rkj = row[j];
        for (int i = k + 1 + ts; i <= j; i += 8) cj[i] -= row[i] * rkj;
      }
      __syncthreads();
    }
    if (!bad) break;
    __syncthreads();
    lam *= 100.0;
    ok = attempt < 7;
  }
  if (bad) {
    if (t == 0) atomicAdd(nfail, 1);
    for (int e = t; e < np; e += kFacThreads) Pc[e] = 0.0;
    for (int i = t; i < K; i += kFacThreads) Pc[i * (i + 1) / 2 + i] = 1.0;
    return;
  }
  for (int e = t; e < np; e += kFacThreads) Xp[e] = 0.0;
  __syncthreads();
  for (int i = t; i < K; i += kFacThreads) Xp[i * (i + 1) / 2 + i] = 1.0;
  __syncthreads();
  for (int i = K - 1; i >= 0; --i) {
    const int ci = i * (i + 1) / 2;
    const double rii = Rp[ci + i];
    for (int j = i + t; j < K; j += kFacThreads) {
      const double v = Xp[j * (j + 1) / 2 + i] / rii;
      Xp[j * (j + 1) / 2 + i] = v;
      row[j] = v;
    }
    __syncthreads();
    const int j = i + tc;
    if (j < K) {
      double* xj = Xp + j * (j + 1) / 2;
      const double xij = row[j];
      for (int r = ts; r < i; r += 8) xj[r] -= Rp[ci + r] * xij;
    }
    __syncthreads();
  }
  for (int e = t; e < np; e += kFacThreads) Pc[e] = Xp[e];
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
  if (t.blk < 0) return;                          // an empty run (launch order padding)
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
                               const double* G, const int64_t* goff, const int64_t* foff, int kmax,
                               double shift, double* rc, int32_t* nfail, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  if (kmax < 1 || kmax > kBatchMaxK) return hipErrorInvalidValue;
  const size_t lds = (size_t)kmax * (kmax + 1) * sizeof(double);    // two packed triangles
  hipError_t e = hipFuncSetAttribute((const void*)k_bt_bj_factor,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bt_bj_factor, dim3((unsigned)n_blocks), dim3(kFacThreads), lds, s, geos,
                     blocks, G, goff, foff, shift, rc, nfail);
  return hipGetLastError();
}

}  // namespace elmfb
