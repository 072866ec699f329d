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

// C[M][N] = sum_k A(m, k) B(k, n), A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn]
// (bfloat16), then the epilogue.  Workgroup tile 64 x 64, four waves of 32 x 32 (2 x 2 MFMA
// tiles), k in stages of 32 through LDS (rows of A and columns of B with k contiguous).
__global__ void __launch_bounds__(256) k_mlp_gemm(MlpGemm p) {
  __shared__ __align__(16) uint16_t As[kMT][kLdsK];
  __shared__ __align__(16) uint16_t Bs[kNT][kLdsK];
  const int m0 = blockIdx.y * kMT, n0 = blockIdx.x * kNT;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int li = lane & 15, lq = lane >> 4;
  f4v_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4v_t{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < p.K; k0 += kKT) {
    // stage A (64 x 32) and B (32 x 64); consecutive threads follow the unit stride
#pragma unroll
    for (int it = 0; it < (kMT * kKT) / 256; ++it) {
      const int e = threadIdx.x + 256 * it;
      int r, c;
      if (p.sak == 1) { r = e / kKT; c = e % kKT; } else { r = e % kMT; c = e / kMT; }
      const int m = m0 + r, k = k0 + c;
      As[r][c] = (m < p.M && k < p.K) ? p.A[(int64_t)m * p.sam + (int64_t)k * p.sak] : (uint16_t)0;
    }
#pragma unroll
    for (int it = 0; it < (kNT * kKT) / 256; ++it) {
      const int e = threadIdx.x + 256 * it;
      int r, c;   // r: n within the tile, c: k within the stage
      if (p.sbn == 1) { r = e % kNT; c = e / kNT; } else { r = e / kKT; c = e % kKT; }
      const int n = n0 + r, k = k0 + c;
      Bs[r][c] = (n < p.N && k < p.K) ? p.B[(int64_t)k * p.sbk + (int64_t)n * p.sbn] : (uint16_t)0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      bf8v_t a;
      const uint16_t* ar = &As[wm * 32 + i * 16 + li][8 * lq];
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = __builtin_bit_cast(__bf16, ar[q]);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        bf8v_t b;
        const uint16_t* br = &Bs[wn * 32 + j * 16 + li][8 * lq];
#pragma unroll
        for (int q = 0; q < 8; ++q) b[q] = __builtin_bit_cast(__bf16, br[q]);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
      }
    }
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
        const int64_t o = (int64_t)m * p.ldo + n;
        const float c = acc[i][j][v];
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

// db[n] = sum_m g[m][n] in FP32, fixed order.
__global__ void k_mlp_colsum(int M, int N, const uint16_t* __restrict__ g, float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.0f;
  for (int m = 0; m < M; ++m) s += bf16_to_f32(g[(int64_t)m * N + n]);
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

hipError_t launch_mlp_gemm(const MlpGemm& p, hipStream_t s) {
  if (p.M <= 0 || p.N <= 0) return hipSuccess;
  const dim3 grid((unsigned)((p.N + kNT - 1) / kNT), (unsigned)((p.M + kMT - 1) / kMT));
  hipLaunchKernelGGL(k_mlp_gemm, grid, dim3(256), 0, s, p);
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
hipError_t launch_mlp_colsum(int M, int N, const uint16_t* g, float* db, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_colsum, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, M, N, g, db);
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
