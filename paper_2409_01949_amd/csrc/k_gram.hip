// Gram blocks of the normal equations, G_ij = M_i^T M_j summed over the grid points the two
// supports share (the block decomposition of Sec. 3, eq. multilevel_domain_decomp, gives
// M^T M = sum_ij W_i^T M_i^T V_i V_j^T M_j W_j, nonzero only where I_i and I_j intersect).
//
// Each overlapping pair (i <= j) has a rectangular shared box; its points are split into chunks
// of kGramChunk consecutive points (box row-major).  One workgroup per (chunk, group of <= 64
// output tiles of 16 x 16) stages 32 points of both blocks ([K][32] each, feature-major) in LDS
// and accumulates X Y^T on the matrix cores:
//   FP64 blocks: v_mfma_f64_16x16x4_f64 (8 steps per stage),
//   FP32 blocks: v_mfma_f32_16x16x4_f32 (8 steps),
//   BF16 blocks: v_mfma_f32_16x16x32_bf16 (1 step), FP32 accumulation,
//   FP16 blocks: v_mfma_f32_16x16x32_f16 (1 step), FP32 accumulation.
// A pair with one chunk writes its block directly; a pair with several chunks writes chunk
// partials that a second kernel sums in chunk order (deterministic, no atomics).
#include "device.h"
#include "kernels.h"

namespace elmfb {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));

constexpr int kStage = 32;        // points per LDS stage
constexpr int kGramPf = 16;       // register-prefetched entries per thread (K <= 128)

template <int PREC> struct GramTypes;
template <> struct GramTypes<ELMFB_FP64> { typedef double in_t; typedef double acc_t; typedef d4_t v4; };
template <> struct GramTypes<ELMFB_FP32> { typedef float in_t; typedef float acc_t; typedef f4_t v4; };
template <> struct GramTypes<ELMFB_BF16> { typedef __bf16 in_t; typedef float acc_t; typedef f4_t v4; };
template <> struct GramTypes<ELMFB_FP16> { typedef _Float16 in_t; typedef float acc_t; typedef f4_t v4; };

template <int PREC>
__device__ __forceinline__ typename GramTypes<PREC>::in_t load_in(const void* A, int64_t i);
template <>
__device__ __forceinline__ double load_in<ELMFB_FP64>(const void* A, int64_t i) {
  return static_cast<const double*>(A)[i];
}
template <>
__device__ __forceinline__ float load_in<ELMFB_FP32>(const void* A, int64_t i) {
  return static_cast<const float*>(A)[i];
}
template <>
__device__ __forceinline__ __bf16 load_in<ELMFB_BF16>(const void* A, int64_t i) {
  const uint16_t bits = static_cast<const uint16_t*>(A)[i];
  return __builtin_bit_cast(__bf16, bits);
}
template <>
__device__ __forceinline__ _Float16 load_in<ELMFB_FP16>(const void* A, int64_t i) {
  return static_cast<const _Float16*>(A)[i];
}

// TPW output tiles of 16 x 16 per wave (4 TPW per workgroup): 4 for K <= 64, 9 for K <= 96,
// 16 above, so that the accumulators of small K leave room for the prefetch registers.
template <int PREC, int TPW>
__global__ void __launch_bounds__(256) k_gram(Geo g, const DevBlock* __restrict__ blocks,
                                              const GramPair* __restrict__ pairs,
                                              const GramChunk* __restrict__ chunks,
                                              const void* __restrict__ A,
                                              typename GramTypes<PREC>::acc_t* __restrict__ G,
                                              typename GramTypes<PREC>::acc_t* __restrict__ part) {
  typedef typename GramTypes<PREC>::in_t in_t;
  typedef typename GramTypes<PREC>::acc_t acc_t;
  typedef typename GramTypes<PREC>::v4 v4;
  constexpr bool k16 = PREC == ELMFB_BF16 || PREC == ELMFB_FP16;
  constexpr int STR = k16 ? (kStage + 8) : (kStage + 1);   // LDS row stride
  extern __shared__ __align__(16) unsigned char smem[];
  const int K = g.K;
  const int Kp = (K + 15) & ~15;
  in_t* X = reinterpret_cast<in_t*>(smem);
  in_t* Y = X + (size_t)Kp * STR;

  const GramChunk ck = chunks[blockIdx.x];
  const GramPair pr = pairs[ck.pair];
  const DevBlock Bi = blocks[pr.bi], Bj = blocks[pr.bj];
  const int nshared = pr.nx * pr.ny;
  const int s_end = min(ck.s0 + kGramChunk, nshared);
  const int nT = Kp / 16;
  const int ntiles = nT * nT;
  const int t_base = blockIdx.y * 4 * TPW;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  // a diagonal block G_jj multiplies the staged rows by themselves: stage them once
  const bool diag = pr.bi == pr.bj;
  const in_t* Yop = diag ? X : Y;

  v4 acc[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) acc[i] = v4{0, 0, 0, 0};

  // every thread stages one point slot (s_l) of the stage for features k_l, k_l + 8, ...; the
  // next stage's entries are loaded into registers while the matrix cores work on this one
  const int s_l = threadIdx.x & (kStage - 1), k_l = threadIdx.x >> 5;
  constexpr int kRows = 256 / kStage;            // feature rows per pass (8)
  in_t rx[kGramPf], ry[kGramPf];
  const int npf = Kp / kRows;                    // passes (<= kGramPf when prefetching)
  auto point_idx = [&](int s0, int& pi, int& pj) {
    const int s = s0 + s_l;
    pi = pj = -1;
    if (s < s_end) {
      const int sx = s / pr.ny, sy = s - sx * pr.ny;
      const int ix = pr.ix0 + sx, iy = pr.iy0 + sy;
      pi = (ix - Bi.ix0) * Bi.ny + (iy - Bi.iy0);
      pj = (ix - Bj.ix0) * Bj.ny + (iy - Bj.iy0);
    }
  };
  auto fetch = [&](int s0) {
    int pi, pj;
    point_idx(s0, pi, pj);
#pragma unroll
    for (int m = 0; m < kGramPf; ++m) {
      const int k = k_l + kRows * m;
      in_t xv = in_t(0.0f), yv = in_t(0.0f);
      if (m < npf && k < K && pi >= 0) {
        xv = load_in<PREC>(A, Bi.a_off + (int64_t)k * Bi.ld + pi);
        if (!diag) yv = load_in<PREC>(A, Bj.a_off + (int64_t)k * Bj.ld + pj);
      }
      rx[m] = xv;
      ry[m] = yv;
    }
  };
  const bool pf = npf <= kGramPf;
  if (pf) fetch(ck.s0);
  for (int s0 = ck.s0; s0 < s_end; s0 += kStage) {
    __syncthreads();   // the previous stage's products are done with X and Y
    if (pf) {
#pragma unroll
      for (int m = 0; m < kGramPf; ++m) {
        if (m < npf) {
          const int k = k_l + kRows * m;
          X[k * STR + s_l] = rx[m];
          if (!diag) Y[k * STR + s_l] = ry[m];
        }
      }
    } else {
      int pi, pj;
      point_idx(s0, pi, pj);
      for (int k = k_l; k < Kp; k += kRows) {
        in_t xv = in_t(0.0f), yv = in_t(0.0f);
        if (k < K && pi >= 0) {
          xv = load_in<PREC>(A, Bi.a_off + (int64_t)k * Bi.ld + pi);
          if (!diag) yv = load_in<PREC>(A, Bj.a_off + (int64_t)k * Bj.ld + pj);
        }
        X[k * STR + s_l] = xv;
        if (!diag) Y[k * STR + s_l] = yv;
      }
    }
    __syncthreads();
    if (pf && s0 + kStage < s_end) fetch(s0 + kStage);
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int t = t_base + wid + 4 * i;
      if (t < ntiles) {
        const int I = t / nT, J = t - (t / nT) * nT;
        const in_t* xr = X + (I * 16 + li) * STR;
        const in_t* yr = Yop + (J * 16 + li) * STR;
        if constexpr (PREC == ELMFB_BF16) {
          bf8_t a, b;
#pragma unroll
          for (int q = 0; q < 8; ++q) { a[q] = xr[8 * lq + q]; b[q] = yr[8 * lq + q]; }
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i], 0, 0, 0);
        } else if constexpr (PREC == ELMFB_FP16) {
          h8_t a, b;
#pragma unroll
          for (int q = 0; q < 8; ++q) { a[q] = xr[8 * lq + q]; b[q] = yr[8 * lq + q]; }
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc[i], 0, 0, 0);
        } else if constexpr (PREC == ELMFB_FP32) {
#pragma unroll
          for (int q = 0; q < kStage; q += 4)
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr[q + lq], yr[q + lq], acc[i], 0, 0, 0);
        } else {
#pragma unroll
          for (int q = 0; q < kStage; q += 4)
            acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[q + lq], yr[q + lq], acc[i], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // accumulator layout of a 16 x 16 tile: lane holds column li; rows 4*lq + v for the FP32
  // accumulating forms, rows lq + 4*v for v_mfma_f64_16x16x4_f64
  acc_t* out = (pr.nchunks == 1) ? G + pr.g_off
                                 : part + (int64_t)(blockIdx.x - pr.c0 + pr.p_off) * K * K;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int t = t_base + wid + 4 * i;
    if (t < ntiles) {
      const int I = t / nT, J = t - (t / nT) * nT;
      const int col = J * 16 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = (PREC == ELMFB_FP64) ? I * 16 + lq + 4 * v : I * 16 + 4 * lq + v;
        if (row < K && col < K) out[(int64_t)row * K + col] = acc[i][v];
      }
    }
  }
}

// Sum the chunk partials of every multi-chunk pair in chunk order.
template <typename acc_t>
__global__ void __launch_bounds__(256) k_gram_reduce(Geo g, const GramPair* __restrict__ pairs,
                                                     const int32_t* __restrict__ multi,
                                                     const acc_t* __restrict__ part,
                                                     acc_t* __restrict__ G) {
  const GramPair pr = pairs[multi[blockIdx.x]];
  const int KK = g.K * g.K;
  for (int e = blockIdx.y * 256 + threadIdx.x; e < KK; e += 256 * gridDim.y) {
    acc_t s = 0;
    for (int c = 0; c < pr.nchunks; ++c) s += part[(int64_t)(pr.p_off + c) * KK + e];
    G[pr.g_off + e] = s;
  }
}

static size_t gram_smem(int prec, int K) {
  const int Kp = (K + 15) & ~15;
  const size_t es = prec == ELMFB_FP64 ? 8 : (prec == ELMFB_FP32 ? 4 : 2);
  const int str = (prec == ELMFB_BF16 || prec == ELMFB_FP16) ? kStage + 8 : kStage + 1;
  return 2 * (size_t)Kp * str * es + 2 * kStage * sizeof(int) + 16;
}

template <int PREC, int TPW>
static hipError_t gram_launch(const Geo& g, const DevBlock* blocks, const GramPair* pairs,
                              const GramChunk* chunks, int64_t n_chunks, const void* A, void* G,
                              void* part, size_t sm, hipStream_t s) {
  typedef typename GramTypes<PREC>::acc_t acc_t;
  const int Kp = (g.K + 15) & ~15;
  const int nT = Kp / 16;
  const int groups = (nT * nT + 4 * TPW - 1) / (4 * TPW);
  if (sm > 64 * 1024) {
    const hipError_t ea = hipFuncSetAttribute((const void*)k_gram<PREC, TPW>,
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (ea != hipSuccess) return ea;
  }
  hipLaunchKernelGGL((k_gram<PREC, TPW>), dim3((unsigned)n_chunks, (unsigned)groups), dim3(256),
                     sm, s, g, blocks, pairs, chunks, A, (acc_t*)G, (acc_t*)part);
  return hipGetLastError();
}

template <int PREC>
static hipError_t gram_launch_k(const Geo& g, const DevBlock* blocks, const GramPair* pairs,
                                const GramChunk* chunks, int64_t n_chunks, const void* A, void* G,
                                void* part, size_t sm, hipStream_t s) {
  if (g.K <= 64) return gram_launch<PREC, 4>(g, blocks, pairs, chunks, n_chunks, A, G, part, sm, s);
  if (g.K <= 96) return gram_launch<PREC, 9>(g, blocks, pairs, chunks, n_chunks, A, G, part, sm, s);
  return gram_launch<PREC, 16>(g, blocks, pairs, chunks, n_chunks, A, G, part, sm, s);
}

hipError_t launch_gram(const Geo& g, int prec, const DevBlock* blocks, const GramPair* pairs,
                       const GramChunk* chunks, int64_t n_chunks, const int32_t* multi,
                       int64_t n_multi, const void* A, void* G, void* part, hipStream_t s) {
  if (n_chunks == 0) return hipSuccess;
  const size_t sm = gram_smem(prec, g.K);
  if (sm > 160 * 1024) return hipErrorInvalidValue;
  hipError_t e;
  if (prec == ELMFB_FP64)
    e = gram_launch_k<ELMFB_FP64>(g, blocks, pairs, chunks, n_chunks, A, G, part, sm, s);
  else if (prec == ELMFB_FP32)
    e = gram_launch_k<ELMFB_FP32>(g, blocks, pairs, chunks, n_chunks, A, G, part, sm, s);
  else if (prec == ELMFB_BF16)
    e = gram_launch_k<ELMFB_BF16>(g, blocks, pairs, chunks, n_chunks, A, G, part, sm, s);
  else
    e = gram_launch_k<ELMFB_FP16>(g, blocks, pairs, chunks, n_chunks, A, G, part, sm, s);
  if (e != hipSuccess || n_multi == 0) return e;
  const dim3 rgrid((unsigned)n_multi, (unsigned)((g.K * g.K + 255) / 256 < 16 ? (g.K * g.K + 255) / 256 : 16));
  if (prec == ELMFB_FP64)
    hipLaunchKernelGGL(k_gram_reduce<double>, rgrid, dim3(256), 0, s, g, pairs, multi,
                       (const double*)part, (double*)G);
  else
    hipLaunchKernelGGL(k_gram_reduce<float>, rgrid, dim3(256), 0, s, g, pairs, multi,
                       (const float*)part, (float*)G);
  return hipGetLastError();
}

size_t gram_smem_bytes(int prec, int K) { return gram_smem(prec, K); }

// ---- y = G p from the stored upper Gram blocks (the normal-equation operator of CG on G)
//
// G = M^T M is symmetric; only the blocks G_ij (i <= j) are stored.  Pass 1, one workgroup per
// stored block: the row products G_ij p_j (for block-row i) and, off the diagonal, the column
// products G_ij^T p_i (for block-row j), each written as a K-vector of partials.  A group of 16
// lanes owns one row at a time and reads it in 128-byte segments (lane s takes columns
// s, s + 16, ...), so G_ij is read from memory exactly once: each loaded entry feeds the row
// sum (a 16-lane butterfly) and the lane's running column sums, which are added over the 16
// row groups through LDS at the end.  Pass 2 (k_gmv_rows): every output coefficient sums the
// partials that belong to its block-row in a fixed order (a table built on the host), 4 lanes
// per coefficient, and the workgroup adds its share of p . y.  Deterministic; no atomics.
constexpr int kGmvMaxK = 256;
constexpr int kGmvCols = kGmvMaxK / 16;   // columns per lane

template <typename GT>
__global__ void __launch_bounds__(256) k_gmv_pairs(int K, const GramPair* __restrict__ pairs,
                                                   const GT* __restrict__ G,
                                                   const double* __restrict__ p,
                                                   const SolveState* __restrict__ st,
                                                   double* __restrict__ part) {
  __shared__ double pi_s[kGmvMaxK], pj_s[kGmvMaxK];
  __shared__ double csum[16][kGmvMaxK];
  if (st && st->done) return;
  const int pr = blockIdx.x;
  const GramPair P = pairs[pr];
  const int64_t qi = (int64_t)P.bi * K, qj = (int64_t)P.bj * K;
  for (int t = threadIdx.x; t < K; t += 256) {
    pi_s[t] = p[qi + t];
    pj_s[t] = p[qj + t];
  }
  __syncthreads();
  const GT* Gb = G + P.g_off;
  const bool offd = P.bi != P.bj;
  const int r = threadIdx.x >> 4, s = threadIdx.x & 15;
  const int nc = (K - s + 15) >> 4;          // columns s + 16 j < K of this lane
  double pjr[kGmvCols], cs[kGmvCols];
#pragma unroll
  for (int j = 0; j < kGmvCols; ++j) {
    pjr[j] = j < nc ? pj_s[s + 16 * j] : 0.0;
    cs[j] = 0.0;
  }
  for (int k = r; k < K; k += 16) {
    const GT* row = Gb + (int64_t)k * K + s;
    double gv[kGmvCols];
#pragma unroll
    for (int j = 0; j < kGmvCols; ++j) gv[j] = j < nc ? (double)row[16 * j] : 0.0;
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < kGmvCols; ++j) v += gv[j] * pjr[j];
    v += __shfl_xor(v, 8, 16);
    v += __shfl_xor(v, 4, 16);
    v += __shfl_xor(v, 2, 16);
    v += __shfl_xor(v, 1, 16);
    if (s == 0) part[(int64_t)(2 * pr) * K + k] = v;
    const double pk = pi_s[k];
#pragma unroll
    for (int j = 0; j < kGmvCols; ++j) cs[j] += gv[j] * pk;
  }
  if (!offd) return;
#pragma unroll
  for (int j = 0; j < kGmvCols; ++j)
    if (j < nc) csum[r][s + 16 * j] = cs[j];
  __syncthreads();
  for (int t = threadIdx.x; t < K; t += 256) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) v += csum[q][t];
    part[(int64_t)(2 * pr + 1) * K + t] = v;
  }
}

// y[b K + k] = sum over the partials listed for block-row b (row_ptr / idx, in table order),
// 4 lanes per coefficient taking every 4th partial, combined by a fixed butterfly;
// red[workgroup] = its share of p . y.
__global__ void __launch_bounds__(256) k_gmv_rows(int K, int64_t n_phi,
                                                  const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ idx,
                                                  const double* __restrict__ part,
                                                  const double* __restrict__ p,
                                                  double* __restrict__ y,
                                                  const SolveState* __restrict__ st,
                                                  double* __restrict__ red) {
  __shared__ double sh[4];
  if (st && st->done) return;
  const int sub = threadIdx.x & 3;
  double acc = 0.0;
  const int64_t n4 = n_phi * 4;
  for (int64_t t4 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t4 < n4;
       t4 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = t4 >> 2;
    const int b = (int)(t / K), k = (int)(t - (int64_t)b * K);
    const int e1 = row_ptr[b + 1];
    double v = 0.0;
    int e = row_ptr[b] + sub;
    for (; e + 12 < e1; e += 16) {   // 4 partials of this lane in flight
      double tv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) tv[q] = part[(int64_t)idx[e + 4 * q] * K + k];
#pragma unroll
      for (int q = 0; q < 4; ++q) v += tv[q];
    }
    for (; e < e1; e += 4) v += part[(int64_t)idx[e] * K + k];
    v += __shfl_xor(v, 1, 4);
    v += __shfl_xor(v, 2, 4);
    if (sub == 0) {
      y[t] = v;
      acc += p[t] * v;
    }
  }
  const double sum = block_sum256(acc, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = sum;
}

hipError_t launch_gram_mv_pairs_only(const Geo& g, int gram_prec, const GramPair* pairs,
                                     int64_t n_pairs, const void* G, const double* p, double* part,
                                     hipStream_t s) {
  if (g.K > kGmvMaxK) return hipErrorInvalidValue;
  if (n_pairs == 0) return hipSuccess;
  if (gram_prec == ELMFB_FP64)
    hipLaunchKernelGGL(k_gmv_pairs<double>, dim3((unsigned)n_pairs), dim3(256), 0, s, g.K, pairs,
                       (const double*)G, p, nullptr, part);
  else
    hipLaunchKernelGGL(k_gmv_pairs<float>, dim3((unsigned)n_pairs), dim3(256), 0, s, g.K, pairs,
                       (const float*)G, p, nullptr, part);
  return hipGetLastError();
}

hipError_t launch_gram_mv(const Geo& g, int gram_prec, const GramPair* pairs, int64_t n_pairs,
                          const void* G, const int32_t* row_ptr, const int32_t* idx,
                          const double* p, double* part, double* y, const SolveState* st,
                          double* red, int n_wg, hipStream_t s) {
  if (g.K > kGmvMaxK) return hipErrorInvalidValue;
  if (n_pairs > 0) {
    if (gram_prec == ELMFB_FP64)
      hipLaunchKernelGGL(k_gmv_pairs<double>, dim3((unsigned)n_pairs), dim3(256), 0, s, g.K,
                         pairs, (const double*)G, p, st, part);
    else
      hipLaunchKernelGGL(k_gmv_pairs<float>, dim3((unsigned)n_pairs), dim3(256), 0, s, g.K,
                         pairs, (const float*)G, p, st, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_gmv_rows, dim3(n_wg), dim3(256), 0, s, g.K, g.n_phi, row_ptr, idx, part,
                     p, y, st, red);   // n_wg <= kRedBlocks partials
  return hipGetLastError();
}

}  // namespace elmfb
