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
constexpr int kGdStr = kGdStage + 1;

// One tile of G_b (a GramTask: rows i0.., columns j0.., at most 128 each) in 16 x 16 MFMA tiles,
// FP64 inputs and accumulation on v_mfma_f64_16x16x4_f64; on the diagonal tile only the tiles
// I <= J.  One workgroup per task, the block's points staged 32 at a time (feature-major rows
// i0.. in X and, off the diagonal, rows j0.. in Y: dynamic LDS of one or two panels).
__global__ void __launch_bounds__(256) k_bt_gram_diag(const DevBlock* __restrict__ blocks,
                                                      const GramTask* __restrict__ tasks,
                                                      const double* __restrict__ A,
                                                      const int64_t* __restrict__ goff,
                                                      double* __restrict__ G) {
  extern __shared__ double gd_lds[];
  const GramTask T = tasks[blockIdx.x];
  const DevBlock B = blocks[T.blk];
  const int K = B.nk;
  const bool diag = T.i0 == T.j0;
  double* X = gd_lds;
  double* Y = diag ? gd_lds : gd_lds + kBatchMaxK * kGdStr;
  const int ni = min(kBatchMaxK, K - T.i0), nj = min(kBatchMaxK, K - T.j0);
  const int nTi = (ni + 15) >> 4, nTj = (nj + 15) >> 4;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const double* Ab = A + B.a_off;
  const int n = B.n;
  d4_t acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = d4_t{0, 0, 0, 0};
  for (int p0 = 0; p0 < n; p0 += kGdStage) {
    for (int e = threadIdx.x; e < nTi * 16 * kGdStage; e += 256) {
      const int k = e / kGdStage, c = e - (e / kGdStage) * kGdStage;
      X[k * kGdStr + c] = (k < ni && p0 + c < n) ? Ab[(int64_t)(T.i0 + k) * B.ld + p0 + c] : 0.0;
    }
    if (!diag) {
      for (int e = threadIdx.x; e < nTj * 16 * kGdStage; e += 256) {
        const int k = e / kGdStage, c = e - (e / kGdStage) * kGdStage;
        Y[k * kGdStr + c] = (k < nj && p0 + c < n) ? Ab[(int64_t)(T.j0 + k) * B.ld + p0 + c] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int t = wid + 4 * i;
      if (t < nTi * nTj) {
        const int I = t / nTj, J = t - (t / nTj) * nTj;
        if (!diag || I <= J) {
          const double* xr = X + (I * 16 + li) * kGdStr;
          const double* yr = Y + (J * 16 + li) * kGdStr;
#pragma unroll
          for (int q = 0; q < kGdStage; q += 4)
            acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[q + lq], yr[q + lq], acc[i], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // v_mfma_f64_16x16x4_f64 accumulator: lane holds column li, rows lq + 4 v
  double* Gb = G + goff[T.blk];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int t = wid + 4 * i;
    if (t < nTi * nTj) {
      const int I = t / nTj, J = t - (t / nTj) * nTj;
      if (!diag || I <= J) {
        const int col = J * 16 + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = I * 16 + lq + 4 * v;
          if (row < ni && col < nj) Gb[(int64_t)(T.i0 + row) * K + T.j0 + col] = acc[i][v];
        }
      }
    }
  }
}

// Blocks of at most 128 columns: one workgroup of 1,024 threads per block (blocks blk0 + workgroup
// index), everything in LDS (two packed upper triangles of
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

__global__ void __launch_bounds__(kFacThreads) k_bt_bj_factor(const DevBlock* __restrict__ blocks,
                                                              int blk0,
                                                              const double* __restrict__ G,
                                                              const int64_t* __restrict__ goff,
                                                              const int64_t* __restrict__ foff,
                                                              double shift,
                                                              double* __restrict__ rc,
                                                              int32_t* __restrict__ nfail) {
  extern __shared__ double lds[];
  __shared__ double part[kFacThreads / 64];
  __shared__ double row[kBatchMaxK];
  const int b = blk0 + (int)blockIdx.x;
  const DevBlock B = blocks[b];
  const int K = B.nk;
  const int np = K * (K + 1) / 2;
  double* Rp = lds;
  double* Xp = lds + np;
  const double* Gj = G + goff[b];
  double* Pc = rc + foff[b];
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
// v_mfma_f64_16x16x4_f64 (K <= 512).  One workgroup per run of 16 NB points of a block: the four
// waves own output row tiles (16 features each) w, w + 4, ... and the NB 16-point column tiles;
// the contraction over k runs in LDS stages of 16 (R^{-T} columns from the factor, M_b rows), and
// tiles entirely above the diagonal are skipped.  The FP64 result goes to Mhat (if not NULL) and,
// rounded to nearest even, to the low-precision copy.  Each workgroup reads all K rows of its
// points before it writes any, so Mhat may be A itself (the patch blocks fold in place).
constexpr int kFoldK = 16;

template <int LO, bool FULL, int TPW, int NB>
__global__ void __launch_bounds__(256) k_bt_fold(const DevBlock* __restrict__ blocks,
                                                 const Tile* __restrict__ ftiles,
                                                 const double* A,
                                                 const double* __restrict__ rc,
                                                 const int64_t* __restrict__ foff,
                                                 double* Ahat,
                                                 void* __restrict__ Ahat_lo) {
  constexpr int KMAX = 64 * TPW;                  // TPW row tiles of 16 features per wave
  constexpr int NP = 16 * NB;                     // points per run
  __shared__ double Rt[KMAX][kFoldK + 1];         // Rt[k'][kk] = Ri[k0 + kk][k']
  __shared__ double At[kFoldK][NP + 1];           // At[kk][c] = M_b[k0 + kk][p0 + c]
  const Tile t = ftiles[blockIdx.x];
  if (t.blk < 0) return;                          // an empty run (launch order padding)
  const DevBlock B = blocks[t.blk];
  const int K = B.nk;
  const int n = B.n, p0 = t.p0;
  const double* Ab = A + B.a_off;
  // FULL: R^{-1} stored K x K row-major per block (single problems); else column-packed
  const double* Rb = FULL ? rc + (int64_t)t.blk * K * K : rc + foff[t.blk];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int nT = (K + 15) >> 4;
  d4_t acc[TPW][NB];
#pragma unroll
  for (int a = 0; a < TPW; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = d4_t{0, 0, 0, 0};
  for (int k0 = 0; k0 < K; k0 += kFoldK) {
    for (int e = threadIdx.x; e < KMAX * kFoldK; e += 256) {
      const int kp = e / kFoldK, kk = e - (e / kFoldK) * kFoldK;
      const int k = k0 + kk;
      const int64_t ri = FULL ? (int64_t)k * K + kp : (int64_t)kp * (kp + 1) / 2 + k;
      Rt[kp][kk] = (kp < K && k <= kp) ? Rb[ri] : 0.0;
    }
    for (int e = threadIdx.x; e < kFoldK * NP; e += 256) {
      const int kk = e / NP, c = e - (e / NP) * NP;
      const int k = k0 + kk, p = p0 + c;
      At[kk][c] = (k < K && p < n) ? Ab[(int64_t)k * B.ld + p] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < TPW; ++a) {
      const int I = wid + 4 * a;
      if (I < nT && 16 * I + 15 >= k0) {     // rows k' < k0 of R^{-T} vanish on this stage
#pragma unroll
        for (int b = 0; b < NB; ++b) {
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
    for (int b = 0; b < NB; ++b) {
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

// Points per run of the fold for blocks of up to kmax columns: 64, or 32 above 256 columns.
int fold_run_points(int kmax) { return kmax > 256 ? 32 : 64; }

hipError_t launch_bt_fold(int lo_prec, bool full, int kmax, const DevBlock* blocks,
                          const Tile* ftiles, int64_t n_ftiles, const double* A, const double* rc,
                          const int64_t* foff, double* Ahat, void* Ahat_lo, hipStream_t s) {
  if (n_ftiles == 0) return hipSuccess;
  if (kmax > kPatchMaxK || (full && kmax > 256)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)n_ftiles), blk(256);
#define FOLD(L, F, T, N)                                                                         \
  hipLaunchKernelGGL((k_bt_fold<L, F, T, N>), grid, blk, 0, s, blocks, ftiles, A, rc, foff, Ahat, \
                     Ahat_lo)
#define FOLD_T(L, F)                                                                             \
  do {                                                                                           \
    if (kmax > 256) FOLD(L, F, 8, 2);                                                            \
    else if (kmax > 128) FOLD(L, F, 4, 4);                                                       \
    else FOLD(L, F, 2, 4);                                                                       \
  } while (0)
  if (lo_prec == ELMFB_FP32) { if (full) FOLD_T(ELMFB_FP32, true); else FOLD_T(ELMFB_FP32, false); }
  else if (lo_prec == ELMFB_BF16) { if (full) FOLD_T(ELMFB_BF16, true); else FOLD_T(ELMFB_BF16, false); }
  else if (lo_prec == ELMFB_FP16) { if (full) FOLD_T(ELMFB_FP16, true); else FOLD_T(ELMFB_FP16, false); }
  else { if (full) FOLD_T(-1, true); else FOLD_T(-1, false); }
#undef FOLD_T
#undef FOLD
  return hipGetLastError();
}

// Blocks of up to kPatchMaxK columns (the patches of P^d neighbouring subdomains): one workgroup
// of 256 threads per block (blocks blk0 + workgroup index), the matrices in global memory, nk x nk
// row-major at goff[b] in W (the factor) and G (the Gram block, then the inverse), panels of 16
// rows in LDS.  Cholesky R^T R = G_b + lambda I by right-looking block elimination: per panel the
// 16 x 16 diagonal block is factorised in LDS, the panel rows R[kb.., kb+16..] = R_kk^{-T} W[..]
// are solved one column per thread, and the trailing upper triangle loses Pn^T Pn.  Then
// X = R^{-1} block row by block row from the bottom: for column j,
// X[I, j] = R_II^{-1} (e_j - sum_{s > I} R[I, s] X[s, j]), with the block row of R in LDS and the
// rows of X below it read back from G.  X goes out column-packed at foff[b].  A failed
// factorisation is retried with a 100x larger shift up to 8 times; after that, or for an all-zero
// block, the block gets the identity and nfail counts it.
constexpr int kPanel = 16;
constexpr int kRows = 8;   // rows of a trailing update in flight per thread

__global__ void __launch_bounds__(256) k_bt_bj_factor_blocked(const DevBlock* __restrict__ blocks,
                                                              int blk0, double* __restrict__ G,
                                                              double* __restrict__ W,
                                                              const int64_t* __restrict__ goff,
                                                              const int64_t* __restrict__ foff,
                                                              double shift,
                                                              double* __restrict__ rc,
                                                              int32_t* __restrict__ nfail) {
  __shared__ double Pn[kPanel][kPatchMaxK];
  __shared__ double D[kPanel][kPanel + 1];
  __shared__ double part[4];
  const int b = blk0 + (int)blockIdx.x;
  const DevBlock B = blocks[b];
  const int K = B.nk;
  double* Gb = G + goff[b];
  double* Wb = W + goff[b];
  double* Pc = rc + foff[b];
  const int t = threadIdx.x;
  double tr = 0.0;
  for (int i = t; i < K; i += 256) tr += Gb[(int64_t)i * K + i];
  tr = wave_sum(tr);
  if ((t & 63) == 0) part[t >> 6] = tr;
  __syncthreads();
  tr = (part[0] + part[1]) + (part[2] + part[3]);
  double lam = shift * tr / K;
  bool ok = lam > 0.0;
  bool bad = true;
  for (int attempt = 0; attempt < 8 && ok; ++attempt) {
    __syncthreads();
    for (int64_t e = t; e < (int64_t)K * K; e += 256) {
      const int i = (int)(e / K), j = (int)(e - (int64_t)i * K);
      if (i <= j) Wb[e] = Gb[e] + (i == j ? lam : 0.0);
    }
    __syncthreads();
    bad = false;
    for (int kb = 0; kb < K; kb += kPanel) {
      const int nb = min(kPanel, K - kb);
      const int r16 = t >> 4, c16 = t & 15;
      if (r16 < nb && c16 < nb) D[r16][c16] = r16 <= c16 ? Wb[(int64_t)(kb + r16) * K + kb + c16] : 0.0;
      __syncthreads();
      for (int k = 0; k < nb; ++k) {
        const double d = D[k][k];      // the same value in every thread
        if (!(d > 0.0)) { bad = true; break; }
        const double rk = sqrt(d);
        __syncthreads();
        if (t > k && t < nb) D[k][t] /= rk;
        if (t == 0) D[k][k] = rk;
        __syncthreads();
        if (r16 > k && r16 < nb && c16 >= r16 && c16 < nb) D[r16][c16] -= D[k][r16] * D[k][c16];
        __syncthreads();
      }
      if (bad) break;
      if (r16 < nb && c16 < nb && r16 <= c16) Wb[(int64_t)(kb + r16) * K + kb + c16] = D[r16][c16];
      const int j0 = kb + nb;
      for (int j = j0 + t; j < K; j += 256) {
        double p[kPanel];
#pragma unroll
        for (int r = 0; r < kPanel; ++r) {
          if (r < nb) {
            double v = Wb[(int64_t)(kb + r) * K + j];
#pragma unroll
            for (int q = 0; q < r; ++q) v -= D[q][r] * p[q];
            p[r] = v / D[r][r];
            Pn[r][j] = p[r];
            Wb[(int64_t)(kb + r) * K + j] = p[r];
          }
        }
      }
      __syncthreads();
      // trailing update, kRows rows at a time so that their loads are in flight together
      for (int i0 = j0; i0 < K; i0 += kRows) {
        for (int j = i0 + t; j < K; j += 256) {
          double pj[kPanel], w[kRows];
#pragma unroll
          for (int r = 0; r < kPanel; ++r) pj[r] = r < nb ? Pn[r][j] : 0.0;
#pragma unroll
          for (int a = 0; a < kRows; ++a)
            w[a] = i0 + a <= j ? Wb[(int64_t)(i0 + a) * K + j] : 0.0;
#pragma unroll
          for (int a = 0; a < kRows; ++a) {
            if (i0 + a <= j) {
#pragma unroll
              for (int r = 0; r < kPanel; ++r)
                if (r < nb) w[a] -= Pn[r][i0 + a] * pj[r];
              Wb[(int64_t)(i0 + a) * K + j] = w[a];
            }
          }
        }
      }
      __syncthreads();
    }
    if (!bad) break;
    lam *= 100.0;
    ok = attempt < 7;
  }
  if (bad) {
    if (t == 0) atomicAdd(nfail, 1);
    for (int64_t e = t; e < (int64_t)K * (K + 1) / 2; e += 256) Pc[e] = 0.0;
    for (int i = t; i < K; i += 256) Pc[(int64_t)i * (i + 1) / 2 + i] = 1.0;
    return;
  }
  __syncthreads();
  for (int ib = ((K - 1) / kPanel) * kPanel; ib >= 0; ib -= kPanel) {
    const int nb = min(kPanel, K - ib);
    for (int e = t; e < nb * (K - ib); e += 256) {
      const int r = e / (K - ib), c = ib + (e - (e / (K - ib)) * (K - ib));
      Pn[r][c] = Wb[(int64_t)(ib + r) * K + c];
    }
    __syncthreads();
    for (int j = ib + t; j < K; j += 256) {
      double T[kPanel];
#pragma unroll
      for (int r = 0; r < kPanel; ++r) T[r] = (r < nb && ib + r == j) ? 1.0 : 0.0;
#pragma unroll 8
      for (int s2 = ib + nb; s2 <= j; ++s2) {
        const double x = Gb[(int64_t)s2 * K + j];
#pragma unroll
        for (int r = 0; r < kPanel; ++r)
          if (r < nb) T[r] -= Pn[r][s2] * x;
      }
#pragma unroll
      for (int r = kPanel - 1; r >= 0; --r) {
        if (r < nb) {
          double v = T[r];
#pragma unroll
          for (int q = r + 1; q < kPanel; ++q)
            if (q < nb) v -= Pn[r][ib + q] * T[q];
          T[r] = v / Pn[r][ib + r];
        }
      }
#pragma unroll
      for (int r = 0; r < kPanel; ++r) {
        if (r < nb && ib + r <= j) {
          Gb[(int64_t)(ib + r) * K + j] = T[r];
          Pc[(int64_t)j * (j + 1) / 2 + ib + r] = T[r];
        }
      }
    }
    __syncthreads();
  }
}

// Patch blocks from the assembled subdomain blocks: column c of patch b is feature c mod K of its
// member c / K (members[moff[b]..], lexicographic in the per-axis indices), on the patch's box,
// zero where the point lies outside the member's box and in the row padding.  One workgroup per
// run of 256 stored points of a patch (runs[].p0 < ld).
__global__ void __launch_bounds__(256) k_bt_expand(const Geo* __restrict__ geos,
                                                   const DevBlock* __restrict__ pblocks,
                                                   const Tile* __restrict__ runs,
                                                   const DevBlock* __restrict__ blocks,
                                                   const int32_t* __restrict__ members,
                                                   const int32_t* __restrict__ moff,
                                                   const double* __restrict__ A,
                                                   double* __restrict__ Ap) {
  const Tile r = runs[blockIdx.x];
  const DevBlock P = pblocks[r.blk];
  const int K = geos[P.inst].K;
  const int p = r.p0 + (int)threadIdx.x;
  if (p >= P.ld) return;
  const bool in = p < P.n;
  const int lx = in ? p / P.ny : 0;
  const int ix = P.ix0 + lx, iy = P.iy0 + (in ? p - lx * P.ny : 0);
  const int nm = P.nk / K;
  for (int m = 0; m < nm; ++m) {
    const DevBlock S = blocks[members[moff[r.blk] + m]];
    const bool inside = in && ix >= S.ix0 && ix < S.ix0 + S.nx && iy >= S.iy0 && iy < S.iy0 + S.ny;
    const int64_t src = inside ? S.a_off + (int64_t)(ix - S.ix0) * S.ny + (iy - S.iy0) : 0;
    double* dst = Ap + P.a_off + (int64_t)m * K * P.ld + p;
    for (int k = 0; k < K; ++k) dst[(int64_t)k * P.ld] = inside ? A[src + (int64_t)k * S.ld] : 0.0;
  }
}

hipError_t launch_bt_gram_diag(const DevBlock* blocks, const GramTask* tasks, int64_t n_tasks,
                               bool two_panels, const double* A, const int64_t* goff, double* G,
                               hipStream_t s) {
  if (n_tasks == 0) return hipSuccess;
  const size_t lds = (size_t)(two_panels ? 2 : 1) * kBatchMaxK * kGdStr * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_bt_gram_diag,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bt_gram_diag, dim3((unsigned)n_tasks), dim3(256), lds, s, blocks, tasks, A,
                     goff, G);
  return hipGetLastError();
}

hipError_t launch_bt_bj_factor(const DevBlock* blocks, int blk0, int64_t n_blocks,
                               const double* G, const int64_t* goff, const int64_t* foff, int kmax,
                               double shift, double* rc, int32_t* nfail, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  if (kmax < 1 || kmax > kBatchMaxK) return hipErrorInvalidValue;
  const size_t lds = (size_t)kmax * (kmax + 1) * sizeof(double);    // two packed triangles
  hipError_t e = hipFuncSetAttribute((const void*)k_bt_bj_factor,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bt_bj_factor, dim3((unsigned)n_blocks), dim3(kFacThreads), lds, s, blocks,
                     blk0, G, goff, foff, shift, rc, nfail);
  return hipGetLastError();
}

hipError_t launch_bt_bj_factor_blocked(const DevBlock* blocks, int blk0, int64_t n_blocks,
                                       double* G, double* W, const int64_t* goff,
                                       const int64_t* foff, double shift, double* rc,
                                       int32_t* nfail, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bt_bj_factor_blocked, dim3((unsigned)n_blocks), dim3(256), 0, s, blocks,
                     blk0, G, W, goff, foff, shift, rc, nfail);
  return hipGetLastError();
}

hipError_t launch_bt_expand(const Geo* geos, const DevBlock* pblocks, const Tile* runs,
                            int64_t n_runs, const DevBlock* blocks, const int32_t* members,
                            const int32_t* moff, const double* A, double* Ap, hipStream_t s) {
  if (n_runs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bt_expand, dim3((unsigned)n_runs), dim3(256), 0, s, geos, pblocks, runs,
                     blocks, members, moff, A, Ap);
  return hipGetLastError();
}

}  // namespace elmfb
