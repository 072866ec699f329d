// Block-sparse products with the assembled matrix M = sum_j V_j^T M_j W_j (Sec. 3
// eq. multilevel_domain_decomp), each block M_j stored feature-major [K][ld_j] (rows padded with
// zeros to a multiple of 8 entries, so vector loads stay aligned).
//
// y = M v runs in two passes that stream the matrix exactly once:
//   1. per block point (consecutive points on consecutive lanes; 16-bit copies take two points
//      per lane in one 4-byte load): t_j[p] = sum_k M_j[k][p] v[q0_j + k] -- the K coefficients
//      of the block are wavefront-uniform, so they come from the scalar cache;
//   2. per row (grid point): y_r = sum over the blocks covering it of t_j[p_j(r)], the covering
//      blocks found arithmetically from per-axis index ranges; no atomics, fixed order.
// x = M^T u also streams the matrix once:
//   1. per chunk of <= 2048 consecutive points of one block: each thread holds 8 gathered
//      u values (in vector-load groups of 2 or 4 consecutive points for FP32 and 16-bit
//      copies); for every group of 8 features the 256 lanes form their dot products, a
//      transposing butterfly across the wavefront reduces the 8 features at once (10 cross-lane
//      shuffles) and a 4-wave LDS sum gives the chunk partials;
//   2. per column: sum of the chunk partials of its block in chunk order.
// All reductions are deterministic (fixed order, no floating-point atomics).
#include "device.h"
#include "kernels.h"

namespace elmfb {

// PTS consecutive points per thread (one vector load per feature row); a tile of 256 points
// runs on 256 / PTS threads.  Per point the sum order does not depend on PTS.
template <int PREC, int PTS>
__global__ void __launch_bounds__(256) k_mv_blocks(Geo g, const DevBlock* __restrict__ blocks,
                                                   const Tile* __restrict__ tiles,
                                                   const void* __restrict__ A,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ vscale,
                                                   double* __restrict__ tpart,
                                                   const SolveState* __restrict__ st) {
  if (st && st->done) return;
  const Tile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const DevBlock B = blocks[t.blk];
  const int p = t.p0 + threadIdx.x * PTS;
  if (p >= B.n) return;
  const double* vb = v + B.q0;
  const int K = g.K;
  const int ld = B.ld;
  const int64_t base = B.a_off + p;
  double acc[4][PTS];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < PTS; ++q) acc[u][q] = 0.0;
  int k = 0;
  for (; k + 4 <= K; k += 4) {
    double a[4][PTS];
#pragma unroll
    for (int u = 0; u < 4; ++u) load_vec<PREC, PTS>(A, base + (int64_t)(k + u) * ld, a[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < PTS; ++q) acc[u][q] += a[u][q] * vb[k + u];
  }
  for (; k < K; ++k) {
    double a[PTS];
    load_vec<PREC, PTS>(A, base + (int64_t)k * ld, a);
#pragma unroll
    for (int q = 0; q < PTS; ++q) acc[0][q] += a[q] * vb[k];
  }
  const double sc = vscale ? *vscale : 1.0;
#pragma unroll
  for (int q = 0; q < PTS; ++q)
    if (p + q < B.n)
      tpart[B.p_off + p + q] = ((acc[0][q] + acc[1][q]) + (acc[2][q] + acc[3][q])) * sc;
}

__global__ void __launch_bounds__(256) k_gather_rows(Geo g, const DevBlock* __restrict__ blocks,
                                                     const int32_t* __restrict__ cov,
                                                     const double* __restrict__ tpart, int mode,
                                                     double* __restrict__ out,
                                                     const double* __restrict__ bvec,
                                                     const SolveState* __restrict__ st,
                                                     double* __restrict__ red) {
  __shared__ double sh[4];
  if (st && st->done) return;
  double coef_u = 0.0;
  if (mode == ROW_LSQR_U) coef_u = st->alpha * st->su;
  double acc = 0.0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < g.n_rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int ix = (int)(r / g.ny), iy = (int)(r - (int64_t)ix * g.ny);
    double y = 0.0;
    for (int l = 0; l < g.n_levels; ++l) {
      const int jx0 = cov[g.cov_off[l][0] + 2 * ix], jx1 = cov[g.cov_off[l][0] + 2 * ix + 1];
      const int jy0 = cov[g.cov_off[l][1] + 2 * iy], jy1 = cov[g.cov_off[l][1] + 2 * iy + 1];
      const int Jy = g.J[l][1];
      const int ncx = jx1 - jx0 + 1, ncy = jy1 - jy0 + 1;
      if (g.domain == ELMFB_DOMAIN_L) {
        // an L-shaped domain discards subdomains: covering blocks through the block map
        for (int jx = jx0; jx <= jx1; ++jx)
          for (int jy = jy0; jy <= jy1; ++jy) {
            const int bi = g.bmap[g.bmap_off[l] + jx * Jy + jy];
            if (bi < 0) continue;
            const DevBlock& B = blocks[bi];
            y += tpart[B.p_off + (ix - B.ix0) * B.ny + (iy - B.iy0)];
          }
      } else if (ncx <= 3 && ncy <= 3) {
        // up to 3 x 3 covering blocks (width ratio < 3): every load issued before the sums,
        // which keep the order jx-major, jy-minor; absent slots read the first block and add 0
        double tv[9];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const bool ok = a < ncx && c < ncy;
            const DevBlock& B = blocks[g.bbase[l] + (jx0 + (ok ? a : 0)) * Jy + jy0 + (ok ? c : 0)];
            const int p = (ix - B.ix0) * B.ny + (iy - B.iy0);
            const double t = tpart[B.p_off + p];
            tv[a * 3 + c] = ok ? t : 0.0;
          }
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) y += tv[q];
      } else {
        for (int jx = jx0; jx <= jx1; ++jx) {
          for (int jy = jy0; jy <= jy1; ++jy) {
            const DevBlock& B = blocks[g.bbase[l] + jx * Jy + jy];
            const int p = (ix - B.ix0) * B.ny + (iy - B.iy0);
            y += tpart[B.p_off + p];
          }
        }
      }
    }
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
  if (mode != ROW_STORE) {
    const double s = block_sum256(acc, sh);
    if (threadIdx.x == 0) red[blockIdx.x] = s;
  }
}

// VEC consecutive points per vector load; each thread holds NG groups of them, the groups of a
// chunk interleaved across the workgroup (group i of thread t starts at i*256*VEC + t*VEC).
template <int PREC, int VEC>
__global__ void __launch_bounds__(256) k_rmv_chunks(Geo g, const DevBlock* __restrict__ blocks,
                                                    const Tile* __restrict__ chunks,
                                                    const void* __restrict__ A,
                                                    const double* __restrict__ u,
                                                    const double* __restrict__ uscale,
                                                    double* __restrict__ part,
                                                    const SolveState* __restrict__ st) {
  constexpr int NG = kChunkPts / (256 * VEC);
  static_assert(NG * 256 * VEC == kChunkPts, "chunk size");
  __shared__ double sred[4][264];
  if (st && st->done) return;
  const int ci = xcd_tile(blockIdx.x, gridDim.x);
  const Tile c = chunks[ci];
  const DevBlock B = blocks[c.blk];
  const int K = g.K;
  const double sc = uscale ? *uscale : 1.0;
  double uv[NG][VEC];
  int64_t idx[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    const int p0 = c.p0 + i * 256 * VEC + threadIdx.x * VEC;
    // a group past the block reads the block's first entries with zero weights (in bounds);
    // a group that straddles the end reads padding (zeros, p0 + VEC <= ld) with zero weights
    idx[i] = B.a_off + (p0 < B.n ? p0 : 0);
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      const int p = p0 + q;
      if (p < B.n) {
        const int lx = p / B.ny, ly = p - lx * B.ny;
        const int64_t r = (int64_t)(B.ix0 + lx) * g.ny + (B.iy0 + ly);
        uv[i][q] = u[r] * sc;
      } else {
        uv[i][q] = 0.0;
      }
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int ld = B.ld;
  const int K8 = (K + 7) & ~7;
  for (int k0 = 0; k0 < K8; k0 += 8) {
    double acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      acc[j] = 0.0;
      const int k = k0 + j < K ? k0 + j : K - 1;     // padded features reread the last one
#pragma unroll
      for (int i = 0; i < NG; ++i) {
        double a[VEC];
        load_vec<PREC, VEC>(A, idx[i] + (int64_t)k * ld, a);
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[j] += a[q] * uv[i][q];
      }
    }
    int f;
    const double v = butterfly8(acc, lane, &f);
    if ((lane & 7) == 0) sred[wid][k0 + f] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += 256)
    part[(int64_t)ci * K + k] = (sred[0][k] + sred[1][k]) + (sred[2][k] + sred[3][k]);
}

// bc (may be NULL): the dense soft-constraint rows [n_bc][n_phi]; their part of column q,
// sum_b bc[b][q] u[n_rows + b] (u scaled by *uscale when given), is added after the chunk
// partials.
__global__ void __launch_bounds__(256) k_rmv_finish(Geo g, const int32_t* __restrict__ cstart,
                                                    const double* __restrict__ part, int mode,
                                                    double* __restrict__ out,
                                                    const SolveState* __restrict__ st,
                                                    double* __restrict__ red,
                                                    const double* __restrict__ bc,
                                                    const double* __restrict__ u,
                                                    const double* __restrict__ uscale) {
  __shared__ double sh[4];
  if (st && st->done) return;
  const int K = g.K;
  double coef_v = 0.0;
  bool keep = false;
  if (mode == COL_LSQR_V) {
    coef_v = st->beta * st->sv;
    keep = !(st->beta > 0.0);   // beta == 0: v and alpha stay as they are
  }
  double acc = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < g.n_phi;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(q / K), k = (int)(q - (int64_t)b * K);
    double x = 0.0;
    int c = cstart[b];
    const int ce = cstart[b + 1];
    for (; c + 8 <= ce; c += 8) {   // 8 partials in flight, summed in chunk order
      double t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = part[(int64_t)(c + q) * K + k];
#pragma unroll
      for (int q = 0; q < 8; ++q) x += t[q];
    }
    for (; c < ce; ++c) x += part[(int64_t)c * K + k];
    if (bc) {
      const double usc = uscale ? *uscale : 1.0;
      for (int r = 0; r < g.n_bc; ++r) x += bc[(int64_t)r * g.n_phi + q] * (u[g.n_rows + r] * usc);
    }
    if (mode == COL_STORE) {
      out[q] = x;
    } else if (mode == COL_LSQR_V) {
      double v = out[q];
      if (!keep) {
        v = x - coef_v * v;
        out[q] = v;
      }
      acc += v * v;
    } else {
      out[q] = x;
      acc += x * x;
    }
  }
  if (mode != COL_STORE) {
    const double s = block_sum256(acc, sh);
    if (threadIdx.x == 0) red[blockIdx.x] = s;
  }
}

int rows_wg(const Geo& g) {
  int64_t nb = (g.n_rows + 255) / 256;
  return (int)(nb < kRedBlocks ? nb : kRedBlocks);
}
int cols_wg(const Geo& g) {
  int64_t nb = (g.n_phi + 255) / 256;
  return (int)(nb < kRedBlocks ? nb : kRedBlocks);
}

// Points per thread of the y = M v pass and points per vector load of the M^T u pass, per
// stored precision (16-bit rows are read 4 or 8 bytes per lane).
template <int PREC> struct MvShape { static constexpr int pts = 1, vec = 1; };
template <> struct MvShape<ELMFB_FP32> { static constexpr int pts = 1, vec = 2; };
template <> struct MvShape<ELMFB_BF16> { static constexpr int pts = 2, vec = 4; };
template <> struct MvShape<ELMFB_FP16> { static constexpr int pts = 2, vec = 4; };

template <int PREC>
static void mv_launch(const Geo& g, const DevBlock* blocks, const Tile* tiles, int64_t n_tiles,
                      const void* A, const double* v, const double* vscale, double* tpart,
                      const SolveState* st, hipStream_t s) {
  constexpr int P = MvShape<PREC>::pts;
  hipLaunchKernelGGL((k_mv_blocks<PREC, P>), dim3((unsigned)n_tiles), dim3(kTile / P), 0, s, g,
                     blocks, tiles, A, v, vscale, tpart, st);
}

hipError_t launch_mv_blocks(const Geo& g, int prec, const DevBlock* blocks, const Tile* tiles,
                            int64_t n_tiles, const void* A, const double* v, const double* vscale,
                            double* tpart, const SolveState* st, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  if (prec == ELMFB_FP32) mv_launch<ELMFB_FP32>(g, blocks, tiles, n_tiles, A, v, vscale, tpart, st, s);
  else if (prec == ELMFB_BF16) mv_launch<ELMFB_BF16>(g, blocks, tiles, n_tiles, A, v, vscale, tpart, st, s);
  else if (prec == ELMFB_FP16) mv_launch<ELMFB_FP16>(g, blocks, tiles, n_tiles, A, v, vscale, tpart, st, s);
  else mv_launch<ELMFB_FP64>(g, blocks, tiles, n_tiles, A, v, vscale, tpart, st, s);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const Geo& g, const DevBlock* blocks, const int32_t* cov,
                              const double* tpart, int mode, double* out, const double* bvec,
                              const SolveState* st, double* red, int n_wg, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_rows, dim3(n_wg), dim3(256), 0, s, g, blocks, cov, tpart, mode, out,
                     bvec, st, red);
  return hipGetLastError();
}

template <int PREC>
static void rmv_launch(const Geo& g, const DevBlock* blocks, const Tile* chunks, int64_t n_chunks,
                       const void* A, const double* u, const double* uscale, double* part,
                       const SolveState* st, hipStream_t s) {
  hipLaunchKernelGGL((k_rmv_chunks<PREC, MvShape<PREC>::vec>), dim3((unsigned)n_chunks), dim3(256),
                     0, s, g, blocks, chunks, A, u, uscale, part, st);
}

hipError_t launch_rmv_chunks(const Geo& g, int prec, const DevBlock* blocks, const Tile* chunks,
                             int64_t n_chunks, const void* A, const double* u,
                             const double* uscale, double* part, const SolveState* st,
                             hipStream_t s) {
  if (n_chunks == 0) return hipSuccess;
  if (prec == ELMFB_FP32) rmv_launch<ELMFB_FP32>(g, blocks, chunks, n_chunks, A, u, uscale, part, st, s);
  else if (prec == ELMFB_BF16) rmv_launch<ELMFB_BF16>(g, blocks, chunks, n_chunks, A, u, uscale, part, st, s);
  else if (prec == ELMFB_FP16) rmv_launch<ELMFB_FP16>(g, blocks, chunks, n_chunks, A, u, uscale, part, st, s);
  else rmv_launch<ELMFB_FP64>(g, blocks, chunks, n_chunks, A, u, uscale, part, st, s);
  return hipGetLastError();
}

hipError_t launch_rmv_finish(const Geo& g, const int32_t* chunk_start, const double* part,
                             int mode, double* out, const SolveState* st, double* red, int n_wg,
                             const double* bc, const double* u, const double* uscale,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_rmv_finish, dim3(n_wg), dim3(256), 0, s, g, chunk_start, part, mode, out,
                     st, red, g.n_bc > 0 ? bc : nullptr, u, uscale);
  return hipGetLastError();
}
hipError_t launch_rmv_finish(const Geo& g, const int32_t* chunk_start, const double* part,
                             int mode, double* out, const SolveState* st, double* red, int n_wg,
                             hipStream_t s) {
  return launch_rmv_finish(g, chunk_start, part, mode, out, st, red, n_wg, nullptr, nullptr,
                           nullptr, s);
}

}  // namespace elmfb
