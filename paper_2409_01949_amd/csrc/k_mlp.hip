// Kernels of the warm-start MLP: a tanh network from problem parameters to a subdomain's
// coefficient block, trained with mean-squared error and Adam (the method's optimiser and
// learning rate, Sec. 4.1).  Products take bfloat16 operands on the matrix cores
// (v_mfma_f32_16x16x32_bf16) with FP32 accumulation; master weights, biases, moments and
// pre-activations are FP32.  Rounding to bfloat16 is round-to-nearest-even.
#include <algorithm>

#include "device.h"
#include "kernels.h"

namespace elmfb {

typedef __bf16 bf8v_t __attribute__((ext_vector_type(8)));
typedef float f4v_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

constexpr int kMT = 64, kNT = 64, kKT = 32, kLdsK = kKT + 8;

// How an operand tile is staged from global memory: OP_SCALAR element by element; OP_KVEC eight
// consecutive k of one row in one 16-byte load (k contiguous, rows 16-byte aligned); OP_MVEC eight
// consecutive rows at one k in one 16-byte load (rows contiguous, k stride 16-byte aligned),
// scattered into the k-contiguous LDS tile.
enum { OP_SCALAR = 0, OP_KVEC = 1, OP_MVEC = 2 };

typedef uint16_t u16x8_t __attribute__((ext_vector_type(8)));

// Loads the 8 elements of thread t's share of a 64 x 32 (rows x k) operand tile into r: OP_KVEC
// row t / 4, k 8 (t % 4) ..; otherwise k t / 8, rows 8 (t % 8) ...  X(row, k) = P[row sr + k sk].
template <int MODE>
__device__ __forceinline__ void tile_load(const uint16_t* __restrict__ P, int64_t sr, int64_t sk,
                                          int rows, int K, int r0, int k0, u16x8_t& r) {
  const int t = threadIdx.x;
  if constexpr (MODE == OP_KVEC) {
    const int row = r0 + (t >> 2), k = k0 + 8 * (t & 3);
    if (row < rows && k + 8 <= K) {
      r = *reinterpret_cast<const u16x8_t*>(P + (int64_t)row * sr + k);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q)
        r[q] = (row < rows && k + q < K) ? P[(int64_t)row * sr + k + q] : (uint16_t)0;
    }
  } else {
    const int k = k0 + (t >> 3), row = r0 + 8 * (t & 7);
    if (MODE == OP_MVEC && k < K && row + 8 <= rows) {
      r = *reinterpret_cast<const u16x8_t*>(P + (int64_t)k * sk + row);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q)
        r[q] = (k < K && row + q < rows) ? P[(int64_t)(row + q) * sr + (int64_t)k * sk]
                                         : (uint16_t)0;
    }
  }
}

template <int MODE>
__device__ __forceinline__ void tile_store(uint16_t (*S)[kLdsK], const u16x8_t& r) {
  const int t = threadIdx.x;
  if constexpr (MODE == OP_KVEC) {
    *reinterpret_cast<u16x8_t*>(&S[t >> 2][8 * (t & 3)]) = r;
  } else {
    const int k = t >> 3, row = 8 * (t & 7);
#pragma unroll
    for (int q = 0; q < 8; ++q) S[row + q][k] = r[q];
  }
}

// C[M][N] = sum_k A(m, k) B(k, n), A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn]
// (bfloat16), then the epilogue.  Workgroup tile 64 x 64, four waves of 32 x 32 (2 x 2 tiles of
// v_mfma_f32_16x16x32_bf16), k in stages of 32 through LDS (rows of A and columns of B with k
// contiguous, each lane's MFMA operand one 16-byte read); the next stage's global loads are in
// flight while the current stage is multiplied.  With gridDim.z = S > 1 workgroup z covers k in
// [z kc, (z + 1) kc) and writes its FP32 partial tile to ws[z][M][N]; k_mlp_gemm_reduce sums
// them in order and applies the epilogue.
template <int MA, int MB>
__global__ void __launch_bounds__(256) k_mlp_gemm(MlpGemm p, int kc, float* __restrict__ ws) {
  __shared__ __align__(16) uint16_t As[kMT][kLdsK];
  __shared__ __align__(16) uint16_t Bs[kNT][kLdsK];
  const int m0 = blockIdx.y * kMT, n0 = blockIdx.x * kNT;
  const int kb = blockIdx.z * kc, ke = min(p.K, kb + kc);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int li = lane & 15, lq = lane >> 4;
  f4v_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4v_t{0.f, 0.f, 0.f, 0.f};
  u16x8_t ra, rb;
  // operand B is staged as its transpose: rows n, X(n, k) = B[k sbk + n sbn]
  if (kb < ke) {
    tile_load<MA>(p.A, p.sam, p.sak, p.M, ke, m0, kb, ra);
    tile_load<MB>(p.B, p.sbn, p.sbk, p.N, ke, n0, kb, rb);
  }
  for (int k0 = kb; k0 < ke; k0 += kKT) {
    tile_store<MA>(As, ra);
    tile_store<MB>(Bs, rb);
    __syncthreads();
    if (k0 + kKT < ke) {
      tile_load<MA>(p.A, p.sam, p.sak, p.M, ke, m0, k0 + kKT, ra);
      tile_load<MB>(p.B, p.sbn, p.sbk, p.N, ke, n0, k0 + kKT, rb);
    }
    bf8v_t a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = *reinterpret_cast<const bf8v_t*>(&As[wm * 32 + i * 16 + li][8 * lq]);
      b[i] = *reinterpret_cast<const bf8v_t*>(&Bs[wn * 32 + i * 16 + li][8 * lq]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // accumulator of the FP32 16x16 forms: lane holds column li, rows 4 lq + v
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm * 32 + i * 16 + 4 * lq + v;
        const int n = n0 + wn * 32 + j * 16 + li;
        if (m >= p.M || n >= p.N) continue;
        const float c = acc[i][j][v];
        if (gridDim.z > 1) {
          ws[((int64_t)blockIdx.z * p.M + m) * p.N + n] = c;
          continue;
        }
        const int64_t o = (int64_t)m * p.ldo + n;
        if (p.epi == MLP_EPI_F32) {
          p.out_f32[o] = c;
        } else if (p.epi == MLP_EPI_BIAS) {
          p.out_f32[o] = c + p.bias[n];
        } else if (p.epi == MLP_EPI_BIAS_TANH) {
          p.out_bf16[o] = f32_to_bf16(tanhf(c + p.bias[n]));
        } else {   // MLP_EPI_DTANH
          const float a = bf16_to_f32(p.act[o]);
          p.out_bf16[o] = f32_to_bf16(c * (1.0f - a * a));
        }
      }
}

// Sum of the S partial tiles of a split-k product, in order of z (F32 epilogue).
__global__ void k_mlp_gemm_reduce(MlpGemm p, int S, const float* __restrict__ ws) {
  const int64_t MN = (int64_t)p.M * p.N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < MN;
       e += (int64_t)gridDim.x * blockDim.x) {
    float c = 0.0f;
    for (int z = 0; z < S; ++z) c += ws[z * MN + e];
    const int64_t m = e / p.N, n = e - m * p.N;
    p.out_f32[m * p.ldo + n] = c;
  }
}

__global__ void k_mlp_to_bf16(int64_t n, const float* __restrict__ x, uint16_t* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = f32_to_bf16(x[i]);
}

// g = bf16(2 (y - t) / n); per-workgroup partial sums of (y - t)^2 in FP64.
__global__ void __launch_bounds__(256) k_mlp_loss(int64_t n, const float* __restrict__ y,
                                                  const float* __restrict__ t,
                                                  uint16_t* __restrict__ g,
                                                  double* __restrict__ part) {
  __shared__ double sh[4];
  double acc = 0.0;
  const float sc = 2.0f / (float)n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float d = y[i] - t[i];
    g[i] = f32_to_bf16(sc * d);
    acc += (double)d * (double)d;
  }
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Modulated output y[b][k] = sum_i f[b][i] z[b][i K + k] (FP32).
__global__ void k_mlp_modulate(int64_t n, int K, int n_mod, const float* __restrict__ z,
                               const float* __restrict__ f, float* __restrict__ y) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / K;
    const int k = (int)(e - b * K);
    float s = 0.0f;
    for (int i = 0; i < n_mod; ++i) s += f[b * n_mod + i] * z[(b * n_mod + i) * K + k];
    y[e] = s;
  }
}

// Loss of the modulated output: d = y - t, g = 2 d / n, gz[b][i K + k] = bf16(f[b][i] g);
// per-workgroup partial sums of d^2 in FP64.
__global__ void __launch_bounds__(256) k_mlp_mod_loss(int64_t n, int K, int n_mod,
                                                      const float* __restrict__ z,
                                                      const float* __restrict__ f,
                                                      const float* __restrict__ t,
                                                      uint16_t* __restrict__ gz,
                                                      double* __restrict__ part) {
  __shared__ double sh[4];
  double acc = 0.0;
  const float sc = 2.0f / (float)n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / K;
    const int k = (int)(e - b * K);
    float y = 0.0f;
    for (int i = 0; i < n_mod; ++i) y += f[b * n_mod + i] * z[(b * n_mod + i) * K + k];
    const float d = y - t[e];
    const float g = sc * d;
    for (int i = 0; i < n_mod; ++i) gz[(b * n_mod + i) * K + k] = f32_to_bf16(f[b * n_mod + i] * g);
    acc += (double)d * (double)d;
  }
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_mlp_sum(int n, const double* __restrict__ part, double scale,
                          double* __restrict__ out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s * scale;
  }
}

// db[n] = sum_m g[m][n] in FP32, fixed order: partial sums over chunks of kColRows rows
// (part[c][n]), then their sum in order of c.
constexpr int kColRows = 256;

__global__ void k_mlp_colsum_part(int M, int N, const uint16_t* __restrict__ g,
                                  float* __restrict__ part) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int m0 = blockIdx.y * kColRows, m1 = min(M, m0 + kColRows);
  float s = 0.0f;
  for (int m = m0; m < m1; ++m) s += bf16_to_f32(g[(int64_t)m * N + n]);
  part[(int64_t)blockIdx.y * N + n] = s;
}

__global__ void k_mlp_colsum(int N, int n_chunks, const float* __restrict__ part,
                             float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.0f;
  for (int c = 0; c < n_chunks; ++c) s += part[(int64_t)c * N + n];
  db[n] = s;
}

// Adam on the flat FP32 parameters; refreshes their bfloat16 copy.
__global__ void k_mlp_adam(int64_t n, float* __restrict__ prm, const float* __restrict__ grad,
                           float* __restrict__ m1, float* __restrict__ m2,
                           uint16_t* __restrict__ pb, float lr, float b1, float b2, float eps,
                           float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float g = grad[i];
    const float a = b1 * m1[i] + (1.0f - b1) * g;
    const float b = b2 * m2[i] + (1.0f - b2) * g * g;
    m1[i] = a;
    m2[i] = b;
    const float p = prm[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
    prm[i] = p;
    pb[i] = f32_to_bf16(p);
  }
}

static unsigned flat_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

static bool aligned16(const void* q) { return ((uintptr_t)q & 15) == 0; }

// Staging mode of an operand X(row, k) = P[row sr + k sk].
static int op_mode(const uint16_t* P, int64_t sr, int64_t sk) {
  if (!aligned16(P)) return OP_SCALAR;
  if (sk == 1 && sr % 8 == 0) return OP_KVEC;
  if (sr == 1 && sk % 8 == 0) return OP_MVEC;
  return OP_SCALAR;
}

int64_t mlp_gemm_ws_floats(int M, int N, int K) {
  const int S = mlp_gemm_splits(M, N, K);
  return S > 1 ? (int64_t)S * M * N : 0;
}

// Split k when the output has too few tiles to fill the chip and k is long (the weight
// gradients: k = batch): about 256 workgroups, at least 256 k per split.
int mlp_gemm_splits(int M, int N, int K) {
  const int64_t tiles = (int64_t)((N + kNT - 1) / kNT) * ((M + kMT - 1) / kMT);
  if (tiles >= 256) return 1;
  int S = (int)std::min<int64_t>(256 / tiles, K / 256);
  return std::max(1, std::min(S, 64));
}

hipError_t launch_mlp_gemm(const MlpGemm& p, float* ws, hipStream_t s) {
  if (p.M <= 0 || p.N <= 0) return hipSuccess;
  int S = p.epi == MLP_EPI_F32 && ws ? mlp_gemm_splits(p.M, p.N, p.K) : 1;
  int kc = p.K;
  if (S > 1) {
    kc = ((p.K + S - 1) / S + kKT - 1) / kKT * kKT;
    S = (p.K + kc - 1) / kc;
  }
  const dim3 grid((unsigned)((p.N + kNT - 1) / kNT), (unsigned)((p.M + kMT - 1) / kMT),
                  (unsigned)S);
  const int ma = op_mode(p.A, p.sam, p.sak), mb = op_mode(p.B, p.sbn, p.sbk);
  float* w = S > 1 ? ws : nullptr;
#define GEMM(A_, B_) hipLaunchKernelGGL((k_mlp_gemm<A_, B_>), grid, dim3(256), 0, s, p, kc, w)
#define GEMM_B(A_)                                  \
  do {                                              \
    if (mb == OP_KVEC) GEMM(A_, OP_KVEC);           \
    else if (mb == OP_MVEC) GEMM(A_, OP_MVEC);      \
    else GEMM(A_, OP_SCALAR);                       \
  } while (0)
  if (ma == OP_KVEC) GEMM_B(OP_KVEC);
  else if (ma == OP_MVEC) GEMM_B(OP_MVEC);
  else GEMM_B(OP_SCALAR);
#undef GEMM_B
#undef GEMM
  if (S > 1) {
    const int64_t MN = (int64_t)p.M * p.N;
    hipLaunchKernelGGL(k_mlp_gemm_reduce, dim3(flat_grid(MN)), dim3(256), 0, s, p, S, ws);
  }
  return hipGetLastError();
}
hipError_t launch_mlp_to_bf16(int64_t n, const float* x, uint16_t* y, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_to_bf16, dim3(flat_grid(n)), dim3(256), 0, s, n, x, y);
  return hipGetLastError();
}
hipError_t launch_mlp_loss(int64_t n, const float* y, const float* t, uint16_t* g, double* part,
                           int n_part, double* loss, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<int64_t>(n_part, std::max<int64_t>(1, (n + 255) / 256));
  hipLaunchKernelGGL(k_mlp_loss, dim3(nb), dim3(256), 0, s, n, y, t, g, part);
  hipLaunchKernelGGL(k_mlp_sum, dim3(1), dim3(64), 0, s, (int)nb, part, 1.0 / (double)n, loss);
  return hipGetLastError();
}
hipError_t launch_mlp_modulate(int64_t n, int K, int n_mod, const float* z, const float* f,
                               float* y, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_modulate, dim3(flat_grid(n)), dim3(256), 0, s, n, K, n_mod, z, f, y);
  return hipGetLastError();
}
hipError_t launch_mlp_mod_loss(int64_t n, int K, int n_mod, const float* z, const float* f,
                               const float* t, uint16_t* gz, double* part, int n_part,
                               double* loss, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<int64_t>(n_part, std::max<int64_t>(1, (n + 255) / 256));
  hipLaunchKernelGGL(k_mlp_mod_loss, dim3(nb), dim3(256), 0, s, n, K, n_mod, z, f, t, gz, part);
  hipLaunchKernelGGL(k_mlp_sum, dim3(1), dim3(64), 0, s, (int)nb, part, 1.0 / (double)n, loss);
  return hipGetLastError();
}
int mlp_colsum_chunks(int M) { return std::max(1, (M + kColRows - 1) / kColRows); }

hipError_t launch_mlp_colsum(int M, int N, const uint16_t* g, float* part, float* db,
                             hipStream_t s) {
  const int nc = mlp_colsum_chunks(M);
  hipLaunchKernelGGL(k_mlp_colsum_part, dim3((unsigned)((N + 255) / 256), (unsigned)nc), dim3(256),
                     0, s, M, N, g, part);
  hipLaunchKernelGGL(k_mlp_colsum, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, nc, part,
                     db);
  return hipGetLastError();
}
hipError_t launch_mlp_adam(int64_t n, float* prm, const float* grad, float* m1, float* m2,
                           uint16_t* pb, float lr, float b1, float b2, float eps, float c1,
                           float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_adam, dim3(flat_grid(n)), dim3(256), 0, s, n, prm, grad, m1, m2, pb, lr,
                     b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace elmfb
