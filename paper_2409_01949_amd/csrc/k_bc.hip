// Soft-constraint rows (Sec. 3 "Definition of the system matrices", the matrix B), stored densely
// over the columns after the collocation rows, and their part of the products:
//   - 1D conditions: row b is sqrt(lambda_b) (1/L) D^order[omega_j phi_q C](x_b), one point per
//     condition (the damped oscillator's initial conditions, Sec. 4.2);
//   - 2D Dirichlet rows at points: row b is w (1/L) omega_j phi_q C at x_b (the boundary term of
//     the Helmholtz loss, Sec. 4.4, with w = sqrt(lambda_bc / N_B)).
// Their part of M^T u is added by k_rmv_finish.
#include "device.h"
#include "kernels.h"

namespace elmfb {

// One workgroup per (block, condition): the block's K entries of the row, zero where x_b lies
// outside the block's support (the planner's strict test); the first block also writes the
// right-hand side entry h[n_rows + b] = sqrt(lambda_b) g_b.
__global__ void __launch_bounds__(256) k_bc_assemble(Geo g, BcSpec bc,
                                                     const DevBlock* __restrict__ blocks,
                                                     const double* __restrict__ W,
                                                     const double* __restrict__ bias,
                                                     double* __restrict__ Bm,
                                                     double* __restrict__ h) {
  const int j = blockIdx.x, b = blockIdx.y;
  const DevBlock B = blocks[j];
  const int l = B.level;
  const int J = g.J[l][0];
  const int jj = j - g.bbase[l];
  const double x = bc.x[b];
  const double sigma = g.sigma[l][0];
  const double mu = centre(g, l, 0, jj);
  // window normalised over the level, value and first derivative (J = 1: factor 1)
  bool in = true;
  double gv = 1.0, g1 = 0.0;
  if (J > 1) {
    in = fabs(x - mu) < sigma;
    double w, w1, w2;
    raw_window(x, mu, sigma, w, w1, w2);
    double S = 0.0, S1 = 0.0;
    for (int t = 0; t < J; ++t) {
      double v, v1, v2;
      raw_window(x, centre(g, l, 0, t), sigma, v, v1, v2);
      S += v;
      S1 += v1;
    }
    gv = w / S;
    g1 = (w1 - gv * S1) / S;
  }
  double c, c1, c2;
  ansatz_axis(g, 0, x, c, c1, c2);
  const double P = c * gv, P1 = c1 * gv + c * g1;
  const double xb = feat_in(g, l, 0, jj, x);
  const double fd = feat_div(g, l, 0);
  const double scale = bc.w[b] * g.inv_levels;
  for (int k = threadIdx.x; k < g.K; k += blockDim.x) {
    double v = 0.0;
    if (in) {
      const int64_t q = B.q0 + k;
      const double w1 = W[2 * q];
      const double ph = tanh(w1 * xb + bias[q]);
      v = bc.order[b] == 0 ? P * ph : P1 * ph + P * (1.0 - ph * ph) * (w1 / fd);
      v *= scale;
    }
    Bm[(int64_t)b * g.n_phi + B.q0 + k] = v;
  }
  if (j == 0 && threadIdx.x == 0) h[g.n_rows + b] = bc.w[b] * bc.val[b];
}

// Dirichlet rows at points of a 2D problem: one workgroup per point x_b.  Row b is
// w (1/L) omega_j(x_b) phi_q(x_b) C(x_b) over every column q (zero where x_b lies outside
// subdomain j's support, the strict test of the planner), each window normalised over the kept
// subdomains of its level at x_b; the right-hand side entry is h[n_rows + b] = w g_b.
__global__ void __launch_bounds__(256) k_bc_assemble_pts(Geo g, const DevBlock* __restrict__ blocks,
                                                         const double* __restrict__ W,
                                                         const double* __restrict__ bias,
                                                         double* __restrict__ Bm,
                                                         double* __restrict__ h) {
  __shared__ double inv_s[kMaxLevels];
  const int b = blockIdx.x;
  const double p[2] = {g.bcpts[2 * b], g.bcpts[2 * b + 1]};
  // the raw 2D window of block j at p: the product of its per-axis factors (factor 1 along an
  // axis with a single subdomain), zero outside the support
  auto window = [&](const DevBlock& B) {
    const int l = B.level;
    double w = 1.0;
    const int jj[2] = {B.jx, B.jy};
    for (int a = 0; a < 2; ++a) {
      if (g.J[l][a] == 1) continue;
      const double mu = centre(g, l, a, jj[a]);
      if (!(fabs(p[a] - mu) < g.sigma[l][a])) return 0.0;
      double v, v1, v2;
      raw_window(p[a], mu, g.sigma[l][a], v, v1, v2);
      w *= v;
    }
    return w;
  };
  if (threadIdx.x < g.n_levels) {
    const int l = threadIdx.x;
    const int j1 = l + 1 < g.n_levels ? g.bbase[l + 1] : g.n_blocks;
    double S = 0.0;
    for (int j = g.bbase[l]; j < j1; ++j) S += window(blocks[j]);
    inv_s[l] = S > 0.0 ? 1.0 / S : 0.0;
  }
  __syncthreads();
  double c0, c1, c2, d0;
  ansatz_axis(g, 0, p[0], c0, c1, c2);
  ansatz_axis(g, 1, p[1], d0, c1, c2);
  const double scale = g.bc_w * g.inv_levels * (c0 * d0);
  for (int64_t q = threadIdx.x; q < g.n_phi; q += blockDim.x) {
    const int j = (int)(q / g.K);
    const DevBlock B = blocks[j];
    const double w = window(B);
    double v = 0.0;
    if (w != 0.0) {
      const int l = B.level;
      const double xb = feat_in(g, l, 0, B.jx, p[0]);
      const double yb = feat_in(g, l, 1, B.jy, p[1]);
      const double ph = tanh(W[2 * q] * xb + W[2 * q + 1] * yb + bias[q]);
      v = scale * (w * inv_s[l]) * ph;
    }
    Bm[(int64_t)b * g.n_phi + q] = v;
  }
  if (threadIdx.x == 0) h[g.n_rows + b] = g.bc_w * g.bcpts[2 * (int64_t)g.n_bc + b];
}

// y_b = sum_q Bm[b][q] v_q (v scaled by *vscale when given) for the soft-constraint rows, one
// wavefront per row and 4 rows per workgroup, then the row mode at row n_rows + b as
// k_gather_rows applies it; each workgroup writes one partial squared norm to red[blockIdx.x]
// (its rows' in order).  Fixed-order sums: deterministic.
__global__ void __launch_bounds__(256) k_bc_rows(Geo g, const double* __restrict__ Bm,
                                                 const double* __restrict__ v,
                                                 const double* __restrict__ vscale, int mode,
                                                 double* __restrict__ out,
                                                 const double* __restrict__ bvec,
                                                 const SolveState* __restrict__ st,
                                                 double* __restrict__ red) {
  __shared__ double sh[4];
  if (st && st->done) return;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int b = blockIdx.x * 4 + wid;
  const double sc = vscale ? *vscale : 1.0;
  double acc = 0.0;
  if (b < g.n_bc) {
    const double* row = Bm + (int64_t)b * g.n_phi;
    double d = 0.0;
    for (int64_t q = lane; q < g.n_phi; q += 64) d += row[q] * v[q];
    const double y = wave_sum(d) * sc;
    if (lane == 0) {
      const int64_t r = g.n_rows + b;
      if (mode == ROW_STORE) {
        out[r] = y;
      } else if (mode == ROW_LSQR_U) {
        const double u = y - st->alpha * st->su * out[r];
        out[r] = u;
        acc = u * u;
      } else if (mode == ROW_RESID) {
        const double u = bvec[r] - y;
        out[r] = u;
        acc = u * u;
      } else {
        out[r] = y;
        acc = y * y;
      }
    }
  }
  if (lane == 0) sh[wid] = acc;
  __syncthreads();
  if (mode != ROW_STORE && threadIdx.x == 0) red[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

int bc_row_wgs(const Geo& g) { return (g.n_bc + 3) / 4; }

hipError_t launch_bc_assemble(const Geo& g, const BcSpec& bc, const DevBlock* blocks,
                              const double* W, const double* b, double* Bm, double* h,
                              hipStream_t s) {
  if (g.n_bc == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bc_assemble, dim3((unsigned)g.n_blocks, (unsigned)g.n_bc), dim3(256), 0,
                     s, g, bc, blocks, W, b, Bm, h);
  return hipGetLastError();
}

hipError_t launch_bc_assemble_pts(const Geo& g, const DevBlock* blocks, const double* W,
                                  const double* b, double* Bm, double* h, hipStream_t s) {
  if (g.n_bc == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bc_assemble_pts, dim3((unsigned)g.n_bc), dim3(256), 0, s, g, blocks, W, b,
                     Bm, h);
  return hipGetLastError();
}

hipError_t launch_bc_rows(const Geo& g, const double* Bm, const double* v, const double* vscale,
                          int mode, double* out, const double* bvec, const SolveState* st,
                          double* red, hipStream_t s) {
  if (g.n_bc == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bc_rows, dim3((unsigned)bc_row_wgs(g)), dim3(256), 0, s, g, Bm, v, vscale,
                     mode, out, bvec, st, red);
  return hipGetLastError();
}

}  // namespace elmfb
