// Soft-constraint rows of the 1D problems (Sec. 3 "Definition of the system matrices", the matrix
// B): row b is sqrt(lambda_b) (1/L) D^order[omega_j phi_q C](x_b) with one point per condition,
// stored densely over the columns (a handful of rows next to N_I collocation rows), and their part
// of the products.  Their part of M^T u is added by k_rmv_finish.
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
  const double xb = (x - mu) / sigma;
  const double scale = bc.w[b] * g.inv_levels;
  for (int k = threadIdx.x; k < g.K; k += blockDim.x) {
    double v = 0.0;
    if (in) {
      const int64_t q = B.q0 + k;
      const double w1 = W[2 * q];
      const double ph = tanh(w1 * xb + bias[q]);
      v = bc.order[b] == 0 ? P * ph : P1 * ph + P * (1.0 - ph * ph) * (w1 / sigma);
      v *= scale;
    }
    Bm[(int64_t)b * g.n_phi + B.q0 + k] = v;
  }
  if (j == 0 && threadIdx.x == 0) h[g.n_rows + b] = bc.w[b] * bc.val[b];
}

// y_b = sum_q Bm[b][q] v_q (v scaled by *vscale when given), for every condition in order, then
// the row mode at row n_rows + b as k_gather_rows applies it; one partial squared norm to *red.
__global__ void __launch_bounds__(256) k_bc_rows(Geo g, const double* __restrict__ Bm,
                                                 const double* __restrict__ v,
                                                 const double* __restrict__ vscale, int mode,
                                                 double* __restrict__ out,
                                                 const double* __restrict__ bvec,
                                                 const SolveState* __restrict__ st,
                                                 double* __restrict__ red) {
  __shared__ double sh[4];
  if (st && st->done) return;
  const double sc = vscale ? *vscale : 1.0;
  const double coef_u = mode == ROW_LSQR_U ? st->alpha * st->su : 0.0;
  double acc = 0.0;
  for (int b = 0; b < g.n_bc; ++b) {
    double d = 0.0;
    for (int64_t q = threadIdx.x; q < g.n_phi; q += blockDim.x)
      d += Bm[(int64_t)b * g.n_phi + q] * v[q];
    const double y = block_sum256(d, sh) * sc;   // thread 0 holds the sum
    if (threadIdx.x == 0) {
      const int64_t r = g.n_rows + b;
      if (mode == ROW_STORE) {
        out[r] = y;
      } else if (mode == ROW_LSQR_U) {
        const double u = y - coef_u * out[r];
        out[r] = u;
        acc += u * u;
      } else if (mode == ROW_RESID) {
        const double u = bvec[r] - y;
        out[r] = u;
        acc += u * u;
      } else {
        out[r] = y;
        acc += y * y;
      }
    }
  }
  if (mode != ROW_STORE && threadIdx.x == 0) *red = acc;
}

hipError_t launch_bc_assemble(const Geo& g, const BcSpec& bc, const DevBlock* blocks,
                              const double* W, const double* b, double* Bm, double* h,
                              hipStream_t s) {
  if (g.n_bc == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bc_assemble, dim3((unsigned)g.n_blocks, (unsigned)g.n_bc), dim3(256), 0,
                     s, g, bc, blocks, W, b, Bm, h);
  return hipGetLastError();
}

hipError_t launch_bc_rows(const Geo& g, const double* Bm, const double* v, const double* vscale,
                          int mode, double* out, const double* bvec, const SolveState* st,
                          double* red, hipStream_t s) {
  if (g.n_bc == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bc_rows, dim3(1), dim3(256), 0, s, g, Bm, v, vscale, mode, out, bvec, st,
                     red);
  return hipGetLastError();
}

}  // namespace elmfb
