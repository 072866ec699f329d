// Batched assembly and Krylov kernels: many independent least-squares problems (instances) of
// the multilevel ELM-FBPINN method (Sec. 3), each with up to 8 right-hand sides that share its
// matrix, processed by every kernel in a single launch.
//
// The instances are concatenated: global row, column, block and block-point ranges with offsets
// per instance; each block records its instance, whose geometry (grid, levels, half-widths,
// scaling) is read from a device table.  Vectors hold the right-hand sides interleaved
// ([row][rhs], [column][rhs]), so one pass over a matrix block serves every right-hand side.
// Row and column work comes in tiles of one instance, which makes every workgroup's partial
// sums belong to a single instance; the per-(instance, rhs) scalar kernels sum their own
// instance's partials in a fixed order.  LSQR recurrences are independent per
// (instance, rhs) (Paige & Saunders 1982, damp 0), their scalars in one SolveState each.
#include "device.h"
#include "kernels.h"

namespace elmfb {

// ---------------------------------------------------------------- assembly

__global__ void __launch_bounds__(256) k_bt_tables(const Geo* __restrict__ geos,
                                                   const BSeg* __restrict__ segs,
                                                   const int32_t* __restrict__ cov,
                                                   double* __restrict__ tab) {
  const BSeg bs = segs[blockIdx.x];
  const AxisSeg sg = bs.s;
  const Geo& g = geos[bs.inst];
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

template <int LO>
__global__ void __launch_bounds__(256) k_bt_assemble(const Geo* __restrict__ geos,
                                                     const DevBlock* __restrict__ blocks,
                                                     const Tile* __restrict__ tiles,
                                                     const double* __restrict__ tab,
                                                     const double* __restrict__ W,
                                                     const double* __restrict__ bias,
                                                     double* __restrict__ A,
                                                     void* __restrict__ A_lo) {
  __shared__ double w1s[kBatchMaxK], w2s[kBatchMaxK], c1s[kBatchMaxK], c2s[kBatchMaxK],
      c3s[kBatchMaxK], bs[kBatchMaxK];
  const Tile t = tiles[blockIdx.x];
  const DevBlock B = blocks[t.blk];
  const Geo& g = geos[B.inst];
  const int K = g.K;
  const int l = B.level;
  const double sx = g.sigma[l][0], sy = g.sigma[l][1];
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double w1 = W[2 * (int64_t)(B.q0 + k)];
    const double w2 = (g.dim == 2) ? W[2 * (int64_t)(B.q0 + k) + 1] : 0.0;
    const double c1 = w1 / sx, c2 = (g.dim == 2) ? w2 / sy : 0.0;
    w1s[k] = w1;
    w2s[k] = w2;
    c1s[k] = c1;
    c2s[k] = c2;
    c3s[k] = c1 * c1 + c2 * c2;
    bs[k] = bias[B.q0 + k];
  }
  __syncthreads();
  const int p = t.p0 + threadIdx.x;
  if (p >= B.n) return;
  const int lx = p / B.ny, ly = p - lx * B.ny;
  const double* tx = tab + 3 * (int64_t)(B.tabx + lx);
  const double* ty = tab + 3 * (int64_t)(B.taby + ly);
  const double X0 = tx[0], X1 = tx[1], X2 = tx[2];
  const double Y0 = ty[0], Y1 = ty[1], Y2 = ty[2];
  const double P = X0 * Y0, Px = X1 * Y0, Py = X0 * Y1, LP = X2 * Y0 + X0 * Y2;
  const int jl = t.blk - g.bbase[l];
  const int jx = jl / g.J[l][1];
  const int jy = jl - jx * g.J[l][1];
  const double xb = (grid_coord(g, 0, B.ix0 + lx) - centre(g, l, 0, jx)) / sx;
  const double yb = (g.dim == 2) ? (grid_coord(g, 1, B.iy0 + ly) - centre(g, l, 1, jy)) / sy : 0.0;
  const double scale = g.inv_scale;
  const int64_t base = B.a_off + p;
  const int n = B.n;
  const int op = g.op;
  for (int k = 0; k < K; ++k) {
    const double z = w1s[k] * xb + w2s[k] * yb + bs[k];
    const double ph = tanh(z);
    const double sd = 1.0 - ph * ph;
    double v;
    if (op == ELMFB_OP_NEG_LAPLACE)
      v = -(LP * ph + 2.0 * sd * (Px * c1s[k] + Py * c2s[k]) - 2.0 * P * ph * sd * c3s[k]);
    else if (op == ELMFB_OP_D1)
      v = Px * ph + P * sd * c1s[k];
    else
      v = P * ph;
    const double e = v * scale;
    A[base + (int64_t)k * n] = e;
    if constexpr (LO == ELMFB_FP32) static_cast<float*>(A_lo)[base + (int64_t)k * n] = (float)e;
    if constexpr (LO == ELMFB_BF16)
      static_cast<uint16_t*>(A_lo)[base + (int64_t)k * n] = f64_to_bf16_rne(e);
  }
}

// h[row][rhs] = f / sqrt(N_inst), f given per instance right-hand-side-major [R][N_i].
__global__ void __launch_bounds__(256) k_bt_rhs(const Geo* __restrict__ geos,
                                                const InstInfo* __restrict__ insts,
                                                const RowTile* __restrict__ rtiles, int R,
                                                const double* __restrict__ f,
                                                double* __restrict__ h, int32_t* __restrict__ bad) {
  const RowTile t = rtiles[blockIdx.x];
  const Geo& g = geos[t.inst];
  const InstInfo I = insts[t.inst];
  const int64_t r = t.r0 + threadIdx.x;
  if (r >= I.row_off + g.n_rows) return;
  const int64_t rl = r - I.row_off;
  const double sq = sqrt((double)g.n_rows);
  for (int j = 0; j < R; ++j) {
    const double v = f[I.row_off * R + (int64_t)j * g.n_rows + rl];
    if (!isfinite(v)) atomicOr(bad, 1);
    h[r * R + j] = v / sq;
  }
}

// ---------------------------------------------------------------- products

// per (instance, rhs) scale of the vector being read: 1/alpha (v) or 1/beta (u); 0 once done
__device__ __forceinline__ double pair_scale(const SolveState* st, int idx, bool use_v) {
  if (!st) return 1.0;
  const SolveState& s = st[idx];
  if (s.done) return 0.0;
  return use_v ? s.sv : s.su;
}

template <int PREC>
__global__ void __launch_bounds__(256) k_bt_mv(const Geo* __restrict__ geos,
                                               const DevBlock* __restrict__ blocks,
                                               const Tile* __restrict__ tiles,
                                               const void* __restrict__ A,
                                               const double* __restrict__ v, int R,
                                               const SolveState* __restrict__ st,
                                               double* __restrict__ tpart) {
  const Tile t = tiles[blockIdx.x];
  const DevBlock B = blocks[t.blk];
  const int p = t.p0 + threadIdx.x;
  if (p >= B.n) return;
  const int K = geos[B.inst].K;
  const int n = B.n;
  const int64_t base = B.a_off + p;
  double acc[kMaxRhs];
#pragma unroll
  for (int j = 0; j < kMaxRhs; ++j) acc[j] = 0.0;
  for (int k = 0; k < K; ++k) {
    const double a = load_entry<PREC>(A, base + (int64_t)k * n);
    const double* vk = v + (int64_t)(B.q0 + k) * R;
#pragma unroll
    for (int j = 0; j < kMaxRhs; ++j)
      if (j < R) acc[j] += a * vk[j];
  }
  double* out = tpart + (B.p_off + p) * R;
  for (int j = 0; j < R; ++j) out[j] = acc[j] * pair_scale(st, B.inst * R + j, true);
}

__global__ void __launch_bounds__(256) k_bt_gather(const Geo* __restrict__ geos,
                                                   const InstInfo* __restrict__ insts,
                                                   const DevBlock* __restrict__ blocks,
                                                   const int32_t* __restrict__ cov,
                                                   const RowTile* __restrict__ rtiles,
                                                   const double* __restrict__ tpart, int mode,
                                                   int R, double* __restrict__ out,
                                                   const double* __restrict__ bvec,
                                                   const SolveState* __restrict__ st,
                                                   double* __restrict__ red) {
  __shared__ double sh[4];
  const RowTile t = rtiles[blockIdx.x];
  const Geo& g = geos[t.inst];
  const InstInfo I = insts[t.inst];
  const int64_t r = t.r0 + threadIdx.x;
  const bool valid = r < I.row_off + g.n_rows;
  double y[kMaxRhs];
#pragma unroll
  for (int j = 0; j < kMaxRhs; ++j) y[j] = 0.0;
  if (valid) {
    const int64_t rl = r - I.row_off;
    const int ix = (int)(rl / g.ny), iy = (int)(rl - (int64_t)ix * g.ny);
    for (int l = 0; l < g.n_levels; ++l) {
      const int jx0 = cov[g.cov_off[l][0] + 2 * ix], jx1 = cov[g.cov_off[l][0] + 2 * ix + 1];
      const int jy0 = cov[g.cov_off[l][1] + 2 * iy], jy1 = cov[g.cov_off[l][1] + 2 * iy + 1];
      const int Jy = g.J[l][1];
      for (int jx = jx0; jx <= jx1; ++jx)
        for (int jy = jy0; jy <= jy1; ++jy) {
          const DevBlock& B = blocks[g.bbase[l] + jx * Jy + jy];
          const int p = (ix - B.ix0) * B.ny + (iy - B.iy0);
          const double* tp = tpart + (B.p_off + p) * R;
#pragma unroll
          for (int j = 0; j < kMaxRhs; ++j)
            if (j < R) y[j] += tp[j];
        }
    }
  }
  for (int j = 0; j < R; ++j) {
    double acc = 0.0;
    if (valid) {
      const int64_t o = r * R + j;
      if (mode == ROW_STORE) {
        out[o] = y[j];
      } else if (mode == ROW_LSQR_U) {
        const SolveState& s = st[t.inst * R + j];
        const double c = s.done ? 0.0 : s.alpha * s.su;
        const double u = y[j] - c * out[o];
        out[o] = s.done ? 0.0 : u;
        acc = s.done ? 0.0 : u * u;
      } else if (mode == ROW_RESID) {
        const double u = bvec[o] - y[j];
        out[o] = u;
        acc = u * u;
      } else {
        out[o] = y[j];
        acc = y[j] * y[j];
      }
    }
    if (mode != ROW_STORE) {
      const double s = block_sum256(acc, sh);
      if (threadIdx.x == 0) red[(int64_t)blockIdx.x * kMaxRhs + j] = s;
    }
  }
}

template <int PREC>
__global__ void __launch_bounds__(256) k_bt_rmv(const Geo* __restrict__ geos,
                                                const InstInfo* __restrict__ insts,
                                                const DevBlock* __restrict__ blocks,
                                                const Tile* __restrict__ chunks,
                                                const void* __restrict__ A,
                                                const double* __restrict__ u, int R,
                                                const SolveState* __restrict__ st,
                                                double* __restrict__ part) {
  constexpr int PPT = kBChunkPts / 256;
  __shared__ double sred[4][kBatchMaxK][kMaxRhs];
  const Tile c = chunks[blockIdx.x];
  const DevBlock B = blocks[c.blk];
  const Geo& g = geos[B.inst];
  const InstInfo I = insts[B.inst];
  const int K = g.K;
  double sc[kMaxRhs];
#pragma unroll
  for (int j = 0; j < kMaxRhs; ++j) sc[j] = j < R ? pair_scale(st, B.inst * R + j, false) : 0.0;
  double uv[PPT][kMaxRhs];
  int64_t idx[PPT];
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int p = c.p0 + i * 256 + threadIdx.x;
    if (p < B.n) {
      const int lx = p / B.ny, ly = p - lx * B.ny;
      const int64_t r = I.row_off + (int64_t)(B.ix0 + lx) * g.ny + (B.iy0 + ly);
#pragma unroll
      for (int j = 0; j < kMaxRhs; ++j) uv[i][j] = j < R ? u[r * R + j] * sc[j] : 0.0;
      idx[i] = B.a_off + p;
    } else {
#pragma unroll
      for (int j = 0; j < kMaxRhs; ++j) uv[i][j] = 0.0;
      idx[i] = B.a_off;   // in bounds; multiplied by zero weights
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int n = B.n;
  const int K8 = (K + 7) & ~7;
  for (int k0 = 0; k0 < K8; k0 += 8) {
    double a[8][PPT];
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const int k = k0 + jj < K ? k0 + jj : K - 1;
#pragma unroll
      for (int i = 0; i < PPT; ++i) a[jj][i] = load_entry<PREC>(A, idx[i] + (int64_t)k * n);
    }
    for (int j = 0; j < R; ++j) {
      double acc[8];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < PPT; ++i) s += a[jj][i] * uv[i][j];
        acc[jj] = s;
      }
      int f;
      const double v = butterfly8(acc, lane, &f);
      if ((lane & 7) == 0) sred[wid][k0 + f][j] = v;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < K * R; e += 256) {
    const int k = e / R, j = e - (e / R) * R;
    part[((int64_t)blockIdx.x * kBatchMaxK + k) * R + j] =
        (sred[0][k][j] + sred[1][k][j]) + (sred[2][k][j] + sred[3][k][j]);
  }
}

__global__ void __launch_bounds__(256) k_bt_finish(const Geo* __restrict__ geos,
                                                   const InstInfo* __restrict__ insts,
                                                   const ColTile* __restrict__ ctiles,
                                                   const int32_t* __restrict__ cstart,
                                                   const double* __restrict__ part, int mode,
                                                   int R, double* __restrict__ out,
                                                   const SolveState* __restrict__ st,
                                                   double* __restrict__ red) {
  __shared__ double sh[4];
  const ColTile t = ctiles[blockIdx.x];
  const Geo& g = geos[t.inst];
  const InstInfo I = insts[t.inst];
  const int64_t q = t.q0 + threadIdx.x;
  const bool valid = q < I.col_off + g.n_phi;
  const int K = g.K;
  int b = 0, k = 0;
  if (valid) {
    const int64_t ql = q - I.col_off;
    b = g.bbase[0] + (int)(ql / K);
    k = (int)(ql - (ql / K) * K);
  }
  for (int j = 0; j < R; ++j) {
    double acc = 0.0;
    if (valid) {
      double x = 0.0;
      for (int c = cstart[b]; c < cstart[b + 1]; ++c)
        x += part[((int64_t)c * kBatchMaxK + k) * R + j];
      const int64_t o = q * R + j;
      if (mode == COL_STORE) {
        out[o] = x;
      } else if (mode == COL_LSQR_V) {
        const SolveState& s = st[t.inst * R + j];
        double v = out[o];
        if (s.done) {
          v = 0.0;
        } else if (s.beta > 0.0) {
          v = x - s.beta * s.sv * v;
        }
        out[o] = v;
        acc = v * v;
      } else {
        out[o] = x;
        acc = x * x;
      }
    }
    if (mode != COL_STORE) {
      const double s = block_sum256(acc, sh);
      if (threadIdx.x == 0) red[(int64_t)blockIdx.x * kMaxRhs + j] = s;
    }
  }
}

// ---------------------------------------------------------------- recurrences

// sum of an instance's tile partials for one right-hand side, in tile order
__device__ __forceinline__ double seg_sum(const double* red, int t0, int t1, int j) {
  double s = 0.0;
  for (int t = t0; t < t1; ++t) s += red[(int64_t)t * kMaxRhs + j];
  return s;
}

// bnorm = ||h||, beta = ||u||, su = 1/beta  (row partials)
__global__ void k_bt_lsqr_init(SolveState* st, const InstInfo* __restrict__ insts, int n_inst,
                               int R, const double* __restrict__ red_b,
                               const double* __restrict__ red_u, double atol, double btol,
                               int iter_lim) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_inst * R) return;
  const int i = idx / R, j = idx - (idx / R) * R;
  const InstInfo I = insts[i];
  SolveState s{};
  const double beta = sqrt(seg_sum(red_u, I.rt0, I.rt1, j));
  s.bnorm = sqrt(seg_sum(red_b, I.rt0, I.rt1, j));
  s.beta = beta;
  s.su = beta > 0.0 ? 1.0 / beta : 0.0;
  s.atol = atol;
  s.btol = btol;
  s.iter_lim = iter_lim;
  s.rel_l2 = -1.0;
  st[idx] = s;
}

// alpha = ||A^T u||, phibar = beta, rhobar = alpha  (column partials)
__global__ void k_bt_lsqr_init_alpha(SolveState* st, const InstInfo* __restrict__ insts,
                                     int n_inst, int R, const double* __restrict__ red) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_inst * R) return;
  const int i = idx / R, j = idx - (idx / R) * R;
  const InstInfo I = insts[i];
  SolveState& s = st[idx];
  const double beta = s.beta;
  const double alpha = beta > 0.0 ? sqrt(seg_sum(red, I.ct0, I.ct1, j)) : 0.0;
  s.alpha = alpha;
  s.sv = alpha > 0.0 ? 1.0 / alpha : 0.0;
  s.phibar = beta;
  s.rhobar = alpha;
  s.rnorm = beta;
  s.arnorm = alpha * beta;
  if (s.bnorm == 0.0) s.bnorm = beta;
  if (alpha * beta == 0.0) { s.istop = 0; s.done = 1; }
  if (s.iter_lim <= 0 && !s.done) { s.istop = 7; s.done = 1; }
}

__global__ void k_bt_lsqr_beta(SolveState* st, const InstInfo* __restrict__ insts, int n_inst,
                               int R, const double* __restrict__ red) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_inst * R) return;
  SolveState& s = st[idx];
  if (s.done) return;
  const InstInfo I = insts[idx / R];
  const double beta = sqrt(seg_sum(red, I.rt0, I.rt1, idx - (idx / R) * R));
  s.beta = beta;
  if (beta > 0.0) {
    s.su = 1.0 / beta;
    s.anorm = sqrt(s.anorm * s.anorm + s.alpha * s.alpha + beta * beta);
  }
}

__global__ void k_bt_lsqr_alpha(SolveState* st, const InstInfo* __restrict__ insts, int n_inst,
                                int R, const double* __restrict__ red) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_inst * R) return;
  SolveState& s = st[idx];
  if (s.done) return;
  const InstInfo I = insts[idx / R];
  const double beta = s.beta;
  double alpha = s.alpha;
  if (beta > 0.0) {
    alpha = sqrt(seg_sum(red, I.ct0, I.ct1, idx - (idx / R) * R));
    s.alpha = alpha;
    if (alpha > 0.0) s.sv = 1.0 / alpha;
  }
  const double rho = sqrt(s.rhobar * s.rhobar + beta * beta);
  const double c = s.rhobar / rho, sn = beta / rho;
  const double theta = sn * alpha;
  s.rhobar = -c * alpha;
  const double phi = c * s.phibar;
  s.phibar = sn * s.phibar;
  s.t1 = phi / rho;
  s.t2 = -theta / rho;
  s.rnorm = s.phibar;
  s.arnorm = alpha * fabs(c) * s.phibar;
}

__global__ void __launch_bounds__(256) k_bt_update(const Geo* __restrict__ geos,
                                                   const InstInfo* __restrict__ insts,
                                                   const ColTile* __restrict__ ctiles, int R,
                                                   double* __restrict__ x,
                                                   double* __restrict__ w,
                                                   const double* __restrict__ v,
                                                   const SolveState* __restrict__ st,
                                                   double* __restrict__ red) {
  __shared__ double sh[4];
  const ColTile t = ctiles[blockIdx.x];
  const InstInfo I = insts[t.inst];
  const int64_t q = t.q0 + threadIdx.x;
  const bool valid = q < I.col_off + geos[t.inst].n_phi;
  for (int j = 0; j < R; ++j) {
    const SolveState& s = st[t.inst * R + j];
    double acc = 0.0;
    if (valid) {
      const int64_t o = q * R + j;
      double xq = x[o];
      if (!s.done) {
        const double wq = w[o];
        xq = xq + s.t1 * wq;
        x[o] = xq;
        w[o] = v[o] * s.sv + s.t2 * wq;
      }
      acc = xq * xq;
    }
    const double sum = block_sum256(acc, sh);
    if (threadIdx.x == 0) red[(int64_t)blockIdx.x * kMaxRhs + j] = sum;
  }
}

__global__ void k_bt_lsqr_stop(SolveState* st, const InstInfo* __restrict__ insts, int n_inst,
                               int R, const double* __restrict__ red) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_inst * R) return;
  SolveState& s = st[idx];
  if (s.done) return;
  const InstInfo I = insts[idx / R];
  const double eps = 2.220446049250313e-16;
  const double xnorm = sqrt(seg_sum(red, I.ct0, I.ct1, idx - (idx / R) * R));
  s.xnorm = xnorm;
  s.itn += 1;
  const double test1 = s.rnorm / s.bnorm;
  const double test2 = s.arnorm / (s.anorm * s.rnorm + eps);
  const double t1 = test1 / (1.0 + s.anorm * xnorm / s.bnorm);
  const double rtol = s.btol + s.atol * s.anorm * xnorm / s.bnorm;
  int istop = 0;
  if (1.0 + test2 <= 1.0) istop = 5;
  if (1.0 + t1 <= 1.0) istop = 4;
  if (test2 <= s.atol) istop = 2;
  if (test1 <= rtol) istop = 1;
  if (istop == 0 && s.itn >= s.iter_lim) istop = 7;
  if (istop != 0) { s.istop = istop; s.done = 1; }
}

// number of (instance, rhs) pairs still iterating, fixed-order sum by one workgroup
__global__ void __launch_bounds__(256) k_bt_count_active(const SolveState* __restrict__ st,
                                                         int n, int32_t* __restrict__ out) {
  __shared__ double sh[4];
  double c = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) c += st[i].done ? 0.0 : 1.0;
  const double s = block_sum256(c, sh);
  if (threadIdx.x == 0) *out = (int32_t)s;
}

// pack / unpack between the ABI layout (per instance [R][n_i]) and the interleaved [global][R]
__global__ void k_bt_pack(const InstInfo* __restrict__ insts, const int64_t* __restrict__ sizes,
                          int n_inst, int R, int64_t total, const double* __restrict__ src,
                          double* __restrict__ dst, int to_interleaved, int use_cols) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    // find the instance of global index g (binary search on the offsets)
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      const int64_t off = use_cols ? insts[mid].col_off : insts[mid].row_off;
      if (off <= g) lo = mid; else hi = mid - 1;
    }
    const int64_t off = use_cols ? insts[lo].col_off : insts[lo].row_off;
    const int64_t n = sizes[lo];
    const int64_t loc = g - off;
    for (int j = 0; j < R; ++j) {
      const int64_t a = g * R + j;                      // interleaved
      const int64_t b = off * R + (int64_t)j * n + loc;  // per instance, rhs-major
      if (to_interleaved) dst[a] = src[b]; else dst[b] = src[a];
    }
  }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_bt_tables(const Geo* geos, const BSeg* segs, int n_segs, const int32_t* cov,
                            double* tab, hipStream_t s) {
  if (n_segs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bt_tables, dim3(n_segs), dim3(256), 0, s, geos, segs, cov, tab);
  return hipGetLastError();
}

hipError_t launch_bt_assemble(int lo_prec, const Geo* geos, const DevBlock* blocks,
                              const Tile* tiles, int64_t n_tiles, const double* tab,
                              const double* W, const double* b, double* A, void* A_lo,
                              hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  const dim3 grid((unsigned)n_tiles), blk(256);
  if (lo_prec == ELMFB_FP32)
    hipLaunchKernelGGL(k_bt_assemble<ELMFB_FP32>, grid, blk, 0, s, geos, blocks, tiles, tab, W, b, A, A_lo);
  else if (lo_prec == ELMFB_BF16)
    hipLaunchKernelGGL(k_bt_assemble<ELMFB_BF16>, grid, blk, 0, s, geos, blocks, tiles, tab, W, b, A, A_lo);
  else
    hipLaunchKernelGGL(k_bt_assemble<-1>, grid, blk, 0, s, geos, blocks, tiles, tab, W, b, A, A_lo);
  return hipGetLastError();
}

hipError_t launch_bt_rhs(const Geo* geos, const InstInfo* insts, const RowTile* rt, int64_t n_rt,
                         int R, const double* f, double* h, int32_t* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_bt_rhs, dim3((unsigned)n_rt), dim3(256), 0, s, geos, insts, rt, R, f, h, bad);
  return hipGetLastError();
}

hipError_t launch_bt_mv(int prec, const Geo* geos, const DevBlock* blocks, const Tile* tiles,
                        int64_t n_tiles, const void* A, const double* v, int R,
                        const SolveState* st, double* tpart, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  const dim3 grid((unsigned)n_tiles), blk(256);
  if (prec == ELMFB_FP32)
    hipLaunchKernelGGL(k_bt_mv<ELMFB_FP32>, grid, blk, 0, s, geos, blocks, tiles, A, v, R, st, tpart);
  else if (prec == ELMFB_BF16)
    hipLaunchKernelGGL(k_bt_mv<ELMFB_BF16>, grid, blk, 0, s, geos, blocks, tiles, A, v, R, st, tpart);
  else
    hipLaunchKernelGGL(k_bt_mv<ELMFB_FP64>, grid, blk, 0, s, geos, blocks, tiles, A, v, R, st, tpart);
  return hipGetLastError();
}

hipError_t launch_bt_gather(const Geo* geos, const InstInfo* insts, const DevBlock* blocks,
                            const int32_t* cov, const RowTile* rt, int64_t n_rt,
                            const double* tpart, int mode, int R, double* out, const double* bvec,
                            const SolveState* st, double* red, hipStream_t s) {
  hipLaunchKernelGGL(k_bt_gather, dim3((unsigned)n_rt), dim3(256), 0, s, geos, insts, blocks, cov,
                     rt, tpart, mode, R, out, bvec, st, red);
  return hipGetLastError();
}

hipError_t launch_bt_rmv(int prec, const Geo* geos, const InstInfo* insts, const DevBlock* blocks,
                         const Tile* chunks, int64_t n_chunks, const void* A, const double* u,
                         int R, const SolveState* st, double* part, hipStream_t s) {
  if (n_chunks == 0) return hipSuccess;
  const dim3 grid((unsigned)n_chunks), blk(256);
  if (prec == ELMFB_FP32)
    hipLaunchKernelGGL(k_bt_rmv<ELMFB_FP32>, grid, blk, 0, s, geos, insts, blocks, chunks, A, u, R, st, part);
  else if (prec == ELMFB_BF16)
    hipLaunchKernelGGL(k_bt_rmv<ELMFB_BF16>, grid, blk, 0, s, geos, insts, blocks, chunks, A, u, R, st, part);
  else
    hipLaunchKernelGGL(k_bt_rmv<ELMFB_FP64>, grid, blk, 0, s, geos, insts, blocks, chunks, A, u, R, st, part);
  return hipGetLastError();
}

hipError_t launch_bt_finish(const Geo* geos, const InstInfo* insts, const ColTile* ct,
                            int64_t n_ct, const int32_t* cstart, const double* part, int mode,
                            int R, double* out, const SolveState* st, double* red, hipStream_t s) {
  hipLaunchKernelGGL(k_bt_finish, dim3((unsigned)n_ct), dim3(256), 0, s, geos, insts, ct, cstart,
                     part, mode, R, out, st, red);
  return hipGetLastError();
}

static dim3 pairs_grid(int n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_bt_lsqr_init(SolveState* st, const InstInfo* insts, int n_inst, int R,
                               const double* red_b, const double* red_u, double atol, double btol,
                               int iter_lim, hipStream_t s) {
  hipLaunchKernelGGL(k_bt_lsqr_init, pairs_grid(n_inst * R), dim3(256), 0, s, st, insts, n_inst, R,
                     red_b, red_u, atol, btol, iter_lim);
  return hipGetLastError();
}
hipError_t launch_bt_lsqr_init_alpha(SolveState* st, const InstInfo* insts, int n_inst, int R,
                                     const double* red, hipStream_t s) {
  hipLaunchKernelGGL(k_bt_lsqr_init_alpha, pairs_grid(n_inst * R), dim3(256), 0, s, st, insts,
                     n_inst, R, red);
  return hipGetLastError();
}
hipError_t launch_bt_lsqr_beta(SolveState* st, const InstInfo* insts, int n_inst, int R,
                               const double* red, hipStream_t s) {
  hipLaunchKernelGGL(k_bt_lsqr_beta, pairs_grid(n_inst * R), dim3(256), 0, s, st, insts, n_inst, R, red);
  return hipGetLastError();
}
hipError_t launch_bt_lsqr_alpha(SolveState* st, const InstInfo* insts, int n_inst, int R,
                                const double* red, hipStream_t s) {
  hipLaunchKernelGGL(k_bt_lsqr_alpha, pairs_grid(n_inst * R), dim3(256), 0, s, st, insts, n_inst, R, red);
  return hipGetLastError();
}
hipError_t launch_bt_update(const Geo* geos, const InstInfo* insts, const ColTile* ct, int64_t n_ct,
                            int R, double* x, double* w, const double* v, const SolveState* st,
                            double* red, hipStream_t s) {
  hipLaunchKernelGGL(k_bt_update, dim3((unsigned)n_ct), dim3(256), 0, s, geos, insts, ct, R, x, w,
                     v, st, red);
  return hipGetLastError();
}
hipError_t launch_bt_lsqr_stop(SolveState* st, const InstInfo* insts, int n_inst, int R,
                               const double* red, hipStream_t s) {
  hipLaunchKernelGGL(k_bt_lsqr_stop, pairs_grid(n_inst * R), dim3(256), 0, s, st, insts, n_inst, R, red);
  return hipGetLastError();
}
hipError_t launch_bt_count_active(const SolveState* st, int n, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_bt_count_active, dim3(1), dim3(256), 0, s, st, n, out);
  return hipGetLastError();
}
hipError_t launch_bt_pack(const InstInfo* insts, const int64_t* sizes, int n_inst, int R,
                          int64_t total, const double* src, double* dst, int to_interleaved,
                          int use_cols, hipStream_t s) {
  int64_t nb = (total + 255) / 256;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_bt_pack, dim3((unsigned)nb), dim3(256), 0, s, insts, sizes, n_inst, R,
                     total, src, dst, to_interleaved, use_cols);
  return hipGetLastError();
}

}  // namespace elmfb
