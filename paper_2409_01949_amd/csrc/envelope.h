// Per-axis envelope table entries of one subdomain along one axis, shared by the single-problem
// and batched assembly (Sec. 4.1 eq. window_func; hard constraint Sec. 4.3).
//
// For grid index m of the segment, with x the grid coordinate, w the subdomain's raw window
// factor and S the sum of the raw factors of every subdomain of the level covering m along the
// axis, the normalised factor is g = w / S, and with the ansatz factor a(x) the entries are
// E = a g, E' = a'g + a g', E'' = a''g + 2a'g' + a g''.  On an L-shaped domain the level sum of
// the kept 2D windows does not factor per axis: there the entries hold the raw factor (g = w)
// and the entry kernel divides by the 2D sum.
//
// Also shared: the staging of a block's features and the operator applied to the envelope times
// one feature, so the two assembly paths compute every entry by the same expressions.
#pragma once

#include "device.h"
#include "kernels.h"

namespace elmfb {

// Entries for grid indices sg.m0..sg.m1-1, strided over the workgroup's threads; cov gives, per
// (level, axis, grid index), the covering subdomain range [jlo, jhi].
__device__ inline void axis_segment_entries(const Geo& g, const AxisSeg& sg,
                                            const int32_t* __restrict__ cov,
                                            double* __restrict__ tab) {
  const int l = sg.level, a = sg.axis;
  const int J = g.J[l][a];
  const double sigma = g.sigma[l][a];
  const double muj = centre(g, l, a, sg.j);
  for (int m = sg.m0 + threadIdx.x; m < sg.m1; m += blockDim.x) {
    double e = 1.0, e1 = 0.0, e2 = 0.0;
    if (a < g.dim) {
      const double x = grid_coord(g, a, m);
      double gv = 1.0, g1 = 0.0, g2 = 0.0;
      if (J > 1) {
        double w, w1, w2;
        raw_window(x, muj, sigma, w, w1, w2);
        if (g.domain == ELMFB_DOMAIN_L) {
          gv = w;
          g1 = w1;
          g2 = w2;
        } else {
          const int jlo = cov[g.cov_off[l][a] + 2 * m], jhi = cov[g.cov_off[l][a] + 2 * m + 1];
          double S = 0.0, S1 = 0.0, S2 = 0.0;
          for (int jj = jlo; jj <= jhi; ++jj) {
            double v, v1, v2;
            raw_window(x, centre(g, l, a, jj), sigma, v, v1, v2);
            S += v; S1 += v1; S2 += v2;
          }
          gv = w / S;
          g1 = (w1 - gv * S1) / S;
          g2 = (w2 - 2.0 * g1 * S1 - gv * S2) / S;
        }
      }
      double c, c1, c2;
      ansatz_axis(g, a, x, c, c1, c2);
      e = c * gv;
      e1 = c1 * gv + c * g1;
      e2 = c2 * gv + 2.0 * c1 * g1 + c * g2;
    }
    const int64_t o = 3 * (int64_t)(sg.tab_off + (m - sg.m0));
    tab[o] = e;
    tab[o + 1] = e1;
    tab[o + 2] = e2;
  }
}

// The K features of the block whose first column is q0, staged for the entry loop (strided over
// the workgroup's threads): w = (W1, W2) and b as given, c = (W1/s_x, W2/s_y) with s the feature
// input scale of level l (the chain-rule factor of d/dx tanh(W xbar + b)), and c3 = |c|^2.
__device__ inline void stage_block_features(const Geo& g, int l, int64_t q0, int K,
                                            const double* __restrict__ W,
                                            const double* __restrict__ bias, double* w1s,
                                            double* w2s, double* c1s, double* c2s, double* c3s,
                                            double* bs) {
  const double sx = feat_div(g, l, 0), sy = feat_div(g, l, 1);
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double w1 = W[2 * (q0 + k)];
    const double w2 = (g.dim == 2) ? W[2 * (q0 + k) + 1] : 0.0;
    const double c1 = w1 / sx, c2 = (g.dim == 2) ? w2 / sy : 0.0;
    w1s[k] = w1;
    w2s[k] = w2;
    c1s[k] = c1;
    c2s[k] = c2;
    c3s[k] = c1 * c1 + c2 * c2;
    bs[k] = bias[q0 + k];
  }
}

// The problem's operator applied to P phi at one point, before the 1/(sqrt(N) L) scale, from the
// envelope P, its gradient (Px, Py) and Laplacian LP there, phi = tanh(z) and sd = 1 - phi^2 of
// one feature, and that feature's c1, c2, c3 (stage_block_features):
//   -Lap(P phi) (Poisson), d/dx (P phi) (first-order ODE), P phi (identity),
//   m (P phi)'' + mu (P phi)' + k P phi (damped oscillator, Sec. 4.2 eq. harm_oscillator; 1D, so
//   LP = P'' and c3 = c1^2), Lap(P phi) + k^2 P phi (Helmholtz, Sec. 4.4 eq. helmholtz_problem).
// With op a compile-time constant the branches fold away.
__device__ __forceinline__ double operator_entry(int op, const double* op_coef, double P,
                                                 double Px, double Py, double LP, double ph,
                                                 double sd, double c1, double c2, double c3) {
  if (op == ELMFB_OP_NEG_LAPLACE)
    return -(LP * ph + 2.0 * sd * (Px * c1 + Py * c2) - 2.0 * P * ph * sd * c3);
  if (op == ELMFB_OP_D1) return Px * ph + P * sd * c1;
  if (op == ELMFB_OP_OSCILLATOR) {
    const double d2 = LP * ph + 2.0 * sd * Px * c1 - 2.0 * P * ph * sd * c3;
    const double d1 = Px * ph + P * sd * c1;
    return op_coef[0] * d2 + op_coef[1] * d1 + op_coef[2] * P * ph;
  }
  if (op == ELMFB_OP_HELMHOLTZ)
    return LP * ph + 2.0 * sd * (Px * c1 + Py * c2) - 2.0 * P * ph * sd * c3 + op_coef[0] * P * ph;
  return P * ph;
}

// Store of an entry's rounded copy (FP32, BF16 or FP16, round to nearest even).
template <int PREC>
__device__ __forceinline__ void store_entry(void* A, int64_t i, double v);
template <>
__device__ __forceinline__ void store_entry<ELMFB_FP32>(void* A, int64_t i, double v) {
  static_cast<float*>(A)[i] = (float)v;
}
template <>
__device__ __forceinline__ void store_entry<ELMFB_BF16>(void* A, int64_t i, double v) {
  static_cast<uint16_t*>(A)[i] = f64_to_bf16_rne(v);
}
template <>
__device__ __forceinline__ void store_entry<ELMFB_FP16>(void* A, int64_t i, double v) {
  static_cast<uint16_t*>(A)[i] = f64_to_fp16_rne(v);
}

}  // namespace elmfb
