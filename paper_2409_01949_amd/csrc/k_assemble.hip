// Fused assembly of the block-sparse least-squares system (Sec. 3 "Definition of the system
// matrices"; windows Sec. 4.1 eq. window_func; features Sec. 3 with h = 1; hard constraint
// Sec. 4.3).
//
// On a tensor grid the windowed, hard-constrained envelope P = C * omega_j of a subdomain is a
// product of one factor per axis: C = a_x(x) a_y(y) and omega_j = g_jx(x) g_jy(y), where
// g_j = w_j / sum_{j'} w_{j'} along that axis (the level sum of the 2D windows factorises into
// the product of the per-axis sums).  So the envelope and its derivatives up to second order
// are tabulated once per (level, axis, subdomain, grid index): E = a g, E' = a'g + a g',
// E'' = a''g + 2a'g' + a g''.  The entry kernel then combines one x-entry and one y-entry per
// point with the K features of the block: phi = tanh(W1 xbar + W2 ybar + b),
//   -Lap(P phi) = -(Lap P phi + 2 (1-phi^2)(P_x W1/sx + P_y W2/sy)
//                   - 2 P phi (1-phi^2)((W1/sx)^2 + (W2/sy)^2)),
//   d/dx(P phi) = P_x phi + P (1-phi^2) W1/sx,    identity: P phi,
//   1D m (P phi)'' + mu (P phi)' + k P phi (the damped oscillator, Sec. 4.2 eq. harm_oscillator),
//   Lap(P phi) + k^2 P phi (the Helmholtz problem, Sec. 4.4 eq. helmholtz_problem),
// scaled by 1/(sqrt(N) L), in FP64, stored feature-major per block (A_blk[k][p]) so that a
// wavefront writes 64 consecutive points of one feature.
#include "device.h"
#include "envelope.h"
#include "kernels.h"

namespace elmfb {

// One workgroup per axis segment (level, axis, subdomain j).
__global__ void __launch_bounds__(256) k_axis_tables(Geo g, const AxisSeg* __restrict__ segs,
                                                     const int32_t* __restrict__ cov,
                                                     double* __restrict__ tab) {
  axis_segment_entries(g, segs[blockIdx.x], cov, tab);
}

// L-shaped domain: per (level, axis, grid index) the sum of the raw window factors of every
// subdomain along the axis covering that index, S_a, and of those whose centre lies above the
// domain's midpoint, D_a, each with two derivatives.  The discarded subdomains of a level are
// the product set {jx: mu_x > mid_x} x {jy: mu_y > mid_y}, so the level sum of the kept 2D
// windows is S = S_x S_y - D_x D_y (and its derivatives follow from the product rule).  An axis
// with a single subdomain has factor 1: S_a = 1, D_a = 0.
__global__ void __launch_bounds__(256) k_axis_sums(Geo g, const int32_t* __restrict__ cov,
                                                   double* __restrict__ lsum) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int l = 0; l < g.n_levels; ++l)
    for (int a = 0; a < 2; ++a) {
      const int n = a == 0 ? g.nx : g.ny;
      if (i >= n) {
        i -= n;
        continue;
      }
      const int m = (int)i;
      double S = 1.0, S1 = 0.0, S2 = 0.0, D = 0.0, D1 = 0.0, D2 = 0.0;
      if (g.J[l][a] > 1) {
        const double x = grid_coord(g, a, m);
        const double sigma = g.sigma[l][a];
        const int jlo = cov[g.cov_off[l][a] + 2 * m], jhi = cov[g.cov_off[l][a] + 2 * m + 1];
        S = 0.0;
        for (int jj = jlo; jj <= jhi; ++jj) {
          const double mu = centre(g, l, a, jj);
          double v, v1, v2;
          raw_window(x, mu, sigma, v, v1, v2);
          S += v; S1 += v1; S2 += v2;
          if (mu > g.lmid[a]) { D += v; D1 += v1; D2 += v2; }
        }
      }
      double* o = lsum + 6 * (int64_t)(g.lsum_off[l][a] + m);
      o[0] = S; o[1] = S1; o[2] = S2; o[3] = D; o[4] = D1; o[5] = D2;
      return;
    }
}

// Envelope P = P_hat / S of a point on an L-shaped domain from the raw product P_hat = X Y (X, Y
// the per-axis table entries, ansatz included) and the 2D level sum S = Sx Sy - Dx Dy, by the
// quotient rule: P_a = (P_hat_a - P S_a)/S, P_aa = (P_hat_aa - 2 P_a S_a - P S_aa)/S.
__device__ __forceinline__ void l_envelope(const Geo& g, int l, int ix, int iy, const double* tx,
                                           const double* ty, double& P, double& Px, double& Py,
                                           double& LP) {
  const double* sx = g.lsum + 6 * (int64_t)(g.lsum_off[l][0] + ix);
  const double* sy = g.lsum + 6 * (int64_t)(g.lsum_off[l][1] + iy);
  const double S = sx[0] * sy[0] - sx[3] * sy[3];
  const double Sx = sx[1] * sy[0] - sx[4] * sy[3];
  const double Sy = sx[0] * sy[1] - sx[3] * sy[4];
  const double Sxx = sx[2] * sy[0] - sx[5] * sy[3];
  const double Syy = sx[0] * sy[2] - sx[3] * sy[5];
  const double H = tx[0] * ty[0], Hx = tx[1] * ty[0], Hy = tx[0] * ty[1];
  const double Hxx = tx[2] * ty[0], Hyy = tx[0] * ty[2];
  P = H / S;
  Px = (Hx - P * Sx) / S;
  Py = (Hy - P * Sy) / S;
  const double Pxx = (Hxx - 2.0 * Px * Sx - P * Sxx) / S;
  const double Pyy = (Hyy - 2.0 * Py * Sy - P * Syy) / S;
  LP = Pxx + Pyy;
}

// One workgroup per tile of <= 256 points of one block; one thread per point, looping over K.
// LO < 0: FP64 matrix only; LO = FP32 / BF16 / FP16: also its rounded copy.
template <int LO, int OP>
__global__ void __launch_bounds__(256) k_assemble(Geo g, const DevBlock* __restrict__ blocks,
                                                  const Tile* __restrict__ tiles,
                                                  const double* __restrict__ tab,
                                                  const double* __restrict__ W,
                                                  const double* __restrict__ bias,
                                                  double* __restrict__ A,
                                                  void* __restrict__ A_lo) {
  __shared__ double w1s[256], w2s[256], c1s[256], c2s[256], c3s[256], bs[256];
  const Tile t = tiles[blockIdx.x];
  const DevBlock B = blocks[t.blk];
  const int K = g.K;
  const int l = B.level;
  stage_block_features(g, l, B.q0, K, W, bias, w1s, w2s, c1s, c2s, c3s, bs);
  __syncthreads();
  const int p = t.p0 + threadIdx.x;
  if (p >= B.n) return;
  const int lx = p / B.ny, ly = p - lx * B.ny;
  const double* tx = tab + 3 * (int64_t)(B.tabx + lx);
  const double* ty = tab + 3 * (int64_t)(B.taby + ly);
  double P, Px, Py, LP;
  bool outside = false;   // a grid point of the removed quarter of an L-shaped domain
  if (g.domain == ELMFB_DOMAIN_L) {
    l_envelope(g, l, B.ix0 + lx, B.iy0 + ly, tx, ty, P, Px, Py, LP);
    outside = grid_coord(g, 0, B.ix0 + lx) > g.lmid[0] && grid_coord(g, 1, B.iy0 + ly) > g.lmid[1];
  } else {
    const double X0 = tx[0], X1 = tx[1], X2 = tx[2];
    const double Y0 = ty[0], Y1 = ty[1], Y2 = ty[2];
    P = X0 * Y0;
    Px = X1 * Y0;
    Py = X0 * Y1;
    LP = X2 * Y0 + X0 * Y2;
  }
  // feature inputs: subdomain-local (x - mu)/sigma, or x with global inputs
  const int jx = B.jx, jy = B.jy;
  const double xb = feat_in(g, l, 0, jx, grid_coord(g, 0, B.ix0 + lx));
  const double yb = (g.dim == 2) ? feat_in(g, l, 1, jy, grid_coord(g, 1, B.iy0 + ly)) : 0.0;
  const double scale = g.inv_scale;
  const int64_t base = B.a_off + p;
  const int ld = B.ld;
  for (int k = 0; k < K; ++k) {
    const double z = w1s[k] * xb + w2s[k] * yb + bs[k];
    const double ph = tanh(z);
    const double sd = 1.0 - ph * ph;
    const double v = operator_entry(OP, g.op_coef, P, Px, Py, LP, ph, sd, c1s[k], c2s[k], c3s[k]);
    const double e = outside ? 0.0 : v * scale;
    A[base + (int64_t)k * ld] = e;
    if constexpr (LO >= 0) store_entry<LO>(A_lo, base + (int64_t)k * ld, e);
  }
}

// h = f / sqrt(N_I); on an L-shaped domain the rows of grid points in the removed quarter are
// zero (f is not read there).
__global__ void k_rhs(Geo g, const double* __restrict__ f, double* __restrict__ h,
                      int32_t* __restrict__ bad) {
  const double sq = sqrt((double)g.n_int);
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < g.n_rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    if (g.domain == ELMFB_DOMAIN_L) {
      const int ix = (int)(r / g.ny), iy = (int)(r - (int64_t)ix * g.ny);
      if (grid_coord(g, 0, ix) > g.lmid[0] && grid_coord(g, 1, iy) > g.lmid[1]) {
        h[r] = 0.0;
        continue;
      }
    }
    const double v = f[r];
    if (!isfinite(v)) atomicOr(bad, 1);
    h[r] = v / sq;
  }
}

__global__ void k_points(Geo g, double* __restrict__ xy) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < g.n_rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int ix = (int)(r / g.ny), iy = (int)(r - (int64_t)ix * g.ny);
    xy[r * g.dim] = grid_coord(g, 0, ix);
    if (g.dim == 2) xy[r * g.dim + 1] = grid_coord(g, 1, iy);
  }
}

hipError_t launch_axis_tables(const Geo& g, const AxisSeg* segs, int n_segs, const int32_t* cov,
                              double* tab, hipStream_t s) {
  if (n_segs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axis_tables, dim3(n_segs), dim3(256), 0, s, g, segs, cov, tab);
  return hipGetLastError();
}

template <int LO>
static hipError_t launch_assemble_p(const Geo& g, const DevBlock* blocks, const Tile* tiles,
                                    int64_t n_tiles, const double* tab, const double* W,
                                    const double* b, double* A, void* A_lo, hipStream_t s) {
  const dim3 grid((unsigned)n_tiles), blk(256);
  switch (g.op) {
    case ELMFB_OP_NEG_LAPLACE:
      hipLaunchKernelGGL((k_assemble<LO, ELMFB_OP_NEG_LAPLACE>), grid, blk, 0, s, g, blocks,
                         tiles, tab, W, b, A, A_lo);
      break;
    case ELMFB_OP_D1:
      hipLaunchKernelGGL((k_assemble<LO, ELMFB_OP_D1>), grid, blk, 0, s, g, blocks, tiles, tab,
                         W, b, A, A_lo);
      break;
    case ELMFB_OP_OSCILLATOR:
      hipLaunchKernelGGL((k_assemble<LO, ELMFB_OP_OSCILLATOR>), grid, blk, 0, s, g, blocks,
                         tiles, tab, W, b, A, A_lo);
      break;
    case ELMFB_OP_HELMHOLTZ:
      hipLaunchKernelGGL((k_assemble<LO, ELMFB_OP_HELMHOLTZ>), grid, blk, 0, s, g, blocks,
                         tiles, tab, W, b, A, A_lo);
      break;
    default:
      hipLaunchKernelGGL((k_assemble<LO, ELMFB_OP_IDENTITY>), grid, blk, 0, s, g, blocks, tiles,
                         tab, W, b, A, A_lo);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_assemble(const Geo& g, int lo_prec, const DevBlock* blocks, const Tile* tiles,
                           int64_t n_tiles, const double* tab, const double* W, const double* b,
                           double* A, void* A_lo, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  if (lo_prec == ELMFB_FP32)
    return launch_assemble_p<ELMFB_FP32>(g, blocks, tiles, n_tiles, tab, W, b, A, A_lo, s);
  if (lo_prec == ELMFB_BF16)
    return launch_assemble_p<ELMFB_BF16>(g, blocks, tiles, n_tiles, tab, W, b, A, A_lo, s);
  if (lo_prec == ELMFB_FP16)
    return launch_assemble_p<ELMFB_FP16>(g, blocks, tiles, n_tiles, tab, W, b, A, A_lo, s);
  return launch_assemble_p<-1>(g, blocks, tiles, n_tiles, tab, W, b, A, A_lo, s);
}

hipError_t launch_axis_sums(const Geo& g, const int32_t* cov, double* lsum, hipStream_t s) {
  int64_t n = 0;
  for (int l = 0; l < g.n_levels; ++l) n += g.nx + g.ny;
  hipLaunchKernelGGL(k_axis_sums, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, cov, lsum);
  return hipGetLastError();
}

hipError_t launch_rhs(const Geo& g, const double* f, double* h, int32_t* bad, hipStream_t s) {
  int64_t nb = (g.n_rows + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_rhs, dim3((unsigned)nb), dim3(256), 0, s, g, f, h, bad);
  return hipGetLastError();
}

hipError_t launch_points(const Geo& g, double* xy, hipStream_t s) {
  int64_t nb = (g.n_rows + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_points, dim3((unsigned)nb), dim3(256), 0, s, g, xy);
  return hipGetLastError();
}

}  // namespace elmfb
