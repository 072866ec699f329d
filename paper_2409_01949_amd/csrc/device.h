// Device helpers shared by the kernel translation units.
#pragma once

#include "common.h"

namespace elmfb {

// Grid coordinate x_m = lo + m*step (last point = hi), each operation rounded on its own (the
// multiply and add must not be contracted into a fused multiply-add).
__device__ __forceinline__ double grid_coord(const Geo& g, int a, int m) {
#pragma clang fp contract(off)
  const int n = (a == 0) ? g.nx : g.ny;
  if (n == 1) return g.lo[a];
  if (m == n - 1) return g.hi[a];
  const double t = (double)m * g.step[a];
  return t + g.lo[a];
}

// Centre of subdomain j of level l along axis a: lo + j*h (J > 1) or the midpoint (J = 1).
__device__ __forceinline__ double centre(const Geo& g, int l, int a, int j) {
#pragma clang fp contract(off)
  if (g.J[l][a] == 1) return g.mid[l][a];
  const double t = (double)j * g.cen_h[l][a];
  return t + g.lo[a];
}

// Input of the random features along axis a of subdomain j of level l at coordinate x, and the
// divisor of its derivative: subdomain-local (x - mu_j)/sigma_l (ELMFB_INPUT_LOCAL) or the
// coordinate itself (ELMFB_INPUT_GLOBAL).
__device__ __forceinline__ double feat_in(const Geo& g, int l, int a, int j, double x) {
  return g.input_norm == ELMFB_INPUT_GLOBAL ? x : (x - centre(g, l, a, j)) / g.sigma[l][a];
}
__device__ __forceinline__ double feat_div(const Geo& g, int l, int a) {
  return g.input_norm == ELMFB_INPUT_GLOBAL ? 1.0 : g.sigma[l][a];
}

// Raw window factor (1 + cos(pi t))^2, t = (x - mu)/sigma, and its first two x-derivatives.
__device__ __forceinline__ void raw_window(double x, double mu, double sigma, double& w,
                                           double& w1, double& w2) {
  const double t = (x - mu) / sigma;
  if (!(fabs(t) < 1.0)) { w = 0.0; w1 = 0.0; w2 = 0.0; return; }
  double s, c;
  sincospi(t, &s, &c);
  const double oc = 1.0 + c;
  w = oc * oc;
  w1 = (-2.0 * M_PI * s * oc) / sigma;
  w2 = (2.0 * M_PI * M_PI * (s * s - c * oc)) / (sigma * sigma);
}

// Hard-constraint factor along one axis: value and two derivatives.
__device__ __forceinline__ void ansatz_axis(const Geo& g, int a, double x, double& v, double& v1,
                                            double& v2) {
  const double w = g.ansatz_omega;
  if (g.ansatz == ELMFB_ANSATZ_TANH_BOX && a < g.dim) {
    const double p = tanh(w * (x - g.lo[a]));
    const double r = tanh(w * (g.hi[a] - x));
    const double dp = w * (1.0 - p * p);
    const double dr = -w * (1.0 - r * r);
    const double ddp = -2.0 * w * p * dp;
    const double ddr = 2.0 * w * r * dr;
    v = p * r;
    v1 = dp * r + p * dr;
    v2 = ddp * r + 2.0 * dp * dr + p * ddr;
  } else if (g.ansatz == ELMFB_ANSATZ_TANH_ORIGIN && a == 0) {
    const double c = tanh(w * x);
    v = c;
    v1 = w * (1.0 - c * c);
    v2 = -2.0 * w * w * c * (1.0 - c * c);
  } else {
    v = 1.0; v1 = 0.0; v2 = 0.0;
  }
}

// Fixed-order (deterministic) sum over a wavefront of 64 lanes.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order sum over a workgroup of 256 threads; the result is valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double* sh /* >= 4 doubles */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// Sum 8 per-lane values over the 64 lanes of a wavefront with a transposing butterfly: after
// the exchanges across lanes 32, 16 and 8 apart each lane holds one of the 8 features (index
// 4*b5 + 2*b4 + b3 of its lane bits), then three plain steps finish the sums; 10 shuffles for
// 8 features instead of 48.  Fixed order, so deterministic.
__device__ __forceinline__ double butterfly8(const double a[8], int lane, int* feat) {
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
  double c[4], d[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double send = b5 ? a[i] : a[i + 4];
    const double keep = b5 ? a[i + 4] : a[i];
    c[i] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double send = b4 ? c[i] : c[i + 2];
    const double keep = b4 ? c[i + 2] : c[i];
    d[i] = keep + __shfl_xor(send, 16, 64);
  }
  const double send = b3 ? d[0] : d[1];
  const double keep = b3 ? d[1] : d[0];
  double v = keep + __shfl_xor(send, 8, 64);
  v += __shfl_xor(v, 4, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 1, 64);
  *feat = (b5 ? 4 : 0) + (b4 ? 2 : 0) + (b3 ? 1 : 0);
  return v;
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b to XCD b mod 8), and each XCD
// has its own L2.  Map workgroup b to a logical tile so that every XCD takes one contiguous range
// of tiles, in order: neighbouring tiles, which share the cache lines at their boundary, then
// run on the same L2 one after the other.  A bijection of 0..n-1 for any n.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  constexpr int kXcd = 8;
  const int x = b % kXcd, i = b / kXcd;
  const int q = n / kXcd, r = n % kXcd;
  return x * q + (x < r ? x : r) + i;
}

template <int PREC>
__device__ __forceinline__ double load_entry(const void* A, int64_t i);

template <>
__device__ __forceinline__ double load_entry<ELMFB_FP64>(const void* A, int64_t i) {
  return static_cast<const double*>(A)[i];
}
template <>
__device__ __forceinline__ double load_entry<ELMFB_FP32>(const void* A, int64_t i) {
  return (double)static_cast<const float*>(A)[i];
}
template <>
__device__ __forceinline__ double load_entry<ELMFB_BF16>(const void* A, int64_t i) {
  return bf16_to_f64(static_cast<const uint16_t*>(A)[i]);
}
template <>
__device__ __forceinline__ double load_entry<ELMFB_FP16>(const void* A, int64_t i) {
  // hardware conversion; exact, subnormals kept (FP16 denormals are on by default on gfx950)
  return (double)(float)static_cast<const _Float16*>(A)[i];
}

// Exact FP64 value of a 16-bit stored entry given as the low 16 bits of w.
template <int PREC>
__device__ __forceinline__ double half_bits_to_f64(uint32_t w) {
  if constexpr (PREC == ELMFB_BF16) return (double)__uint_as_float(w << 16);
  else return (double)(float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
}

// VEC consecutive stored entries from element i in one vector load (i a multiple of VEC; stored
// rows start on kRowAlign-element boundaries, so the load is naturally aligned), as FP64.
template <int PREC, int VEC>
__device__ __forceinline__ void load_vec(const void* A, int64_t i, double (&out)[VEC]) {
  static_assert(VEC == 1 || VEC == 2 || VEC == 4 || VEC == 8, "vector width");
  static_assert(kRowAlign % VEC == 0, "rows must be aligned to the vector width");
  if constexpr (VEC == 1) {
    out[0] = load_entry<PREC>(A, i);
  } else if constexpr (PREC == ELMFB_FP64) {
    static_assert(VEC == 2, "FP64 vectors hold 2 entries");
    const double2 x = *reinterpret_cast<const double2*>(static_cast<const double*>(A) + i);
    out[0] = x.x;
    out[1] = x.y;
  } else if constexpr (PREC == ELMFB_FP32) {
    const float* p = static_cast<const float*>(A) + i;
    if constexpr (VEC == 2) {
      const float2 x = *reinterpret_cast<const float2*>(p);
      out[0] = x.x; out[1] = x.y;
    } else {
      static_assert(VEC == 4, "FP32 vectors hold 2 or 4 entries");
      const float4 x = *reinterpret_cast<const float4*>(p);
      out[0] = x.x; out[1] = x.y; out[2] = x.z; out[3] = x.w;
    }
  } else {
    const uint16_t* p = static_cast<const uint16_t*>(A) + i;
    uint32_t w[VEC / 2];
    if constexpr (VEC == 2) {
      w[0] = *reinterpret_cast<const uint32_t*>(p);
    } else if constexpr (VEC == 4) {
      // streamed once per pass (the M^T u chunks): a non-temporal load leaves the caches to the
      // gathered vector (measured: 92 -> 87 us per FP16 M^T u pass inside the solve; the same
      // hint on the 4-byte loads of M v made that pass slower)
      typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
      const u32x2 x = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
      w[0] = x.x; w[1] = x.y;
    } else {
      const uint4 x = *reinterpret_cast<const uint4*>(p);
      w[0] = x.x; w[1] = x.y; w[2] = x.z; w[3] = x.w;
    }
#pragma unroll
    for (int h = 0; h < VEC / 2; ++h) {
      out[2 * h] = half_bits_to_f64<PREC>(w[h]);
      out[2 * h + 1] = half_bits_to_f64<PREC>(w[h] >> 16);
    }
  }
}

}  // namespace elmfb
