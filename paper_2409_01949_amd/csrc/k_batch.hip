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
#include "envelope.h"
#include "kernels.h"

namespace elmfb {

// ---------------------------------------------------------------- assembly

// One workgroup per axis segment of one instance (instances are boxes: normalised factors).
__global__ void __launch_bounds__(256) k_bt_tables(const Geo* __restrict__ geos,
                                                   const BSeg* __restrict__ segs,
                                                   const int32_t* __restrict__ cov,
                                                   double* __restrict__ tab) {
  const BSeg bs = segs[blockIdx.x];
  axis_segment_entries(geos[bs.inst], bs.s, cov, tab);
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
  stage_block_features(g, l, B.q0, K, W, bias, w1s, w2s, c1s, c2s, c3s, bs);
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
  const double xb = feat_in(g, l, 0, jx, grid_coord(g, 0, B.ix0 + lx));
  const double yb = (g.dim == 2) ? feat_in(g, l, 1, jy, grid_coord(g, 1, B.iy0 + ly)) : 0.0;
  const double scale = g.inv_scale;
  const int64_t base = B.a_off + p;
  const int ld = B.ld;
  const int op = g.op;
  for (int k = 0; k < K; ++k) {
    const double z = w1s[k] * xb + w2s[k] * yb + bs[k];
    const double ph = tanh(z);
    const double sd = 1.0 - ph * ph;
    const double e =
        operator_entry(op, g.op_coef, P, Px, Py, LP, ph, sd, c1s[k], c2s[k], c3s[k]) * scale;
    A[base + (int64_t)k * ld] = e;
    if constexpr (LO >= 0) store_entry<LO>(A_lo, base + (int64_t)k * ld, e);
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
//
// Both matrix passes run one workgroup per subdomain block, so each workgroup's results belong
// to one block of one instance.  Block-Jacobi preconditioning needs no extra work here: its
// factors are folded into a preconditioned copy of the matrix once (k_bt_precond.hip), and the
// same kernels run on that copy.

// per (instance, rhs) scale of the vector being read: 1/alpha (v) or 1/beta (u); 0 once done
__device__ __forceinline__ double pair_scale(const SolveState* st, int idx, bool use_v) {
  if (!st) return 1.0;
  const SolveState& s = st[idx];
  if (s.done) return 0.0;
  return use_v ? s.sv : s.su;
}

// True when every right-hand side of the instance has stopped: the Krylov kernels then skip the
// instance's blocks, rows and columns (their values are read only for pairs still iterating),
// so a batch costs what its active instances cost.
__device__ __forceinline__ bool inst_all_done(const SolveState* st, int inst, int R) {
  if (!st) return false;
  for (int j = 0; j < R; ++j)
    if (!st[inst * R + j].done) return false;
  return true;
}

// Sum 8 per-thread values over the NW waves of a workgroup: transposing butterfly in each wave,
// then the NW wave sums in fixed order.  Value j is returned in thread j (j < 8); every thread
// must call it.
template <int NW = 4>
__device__ __forceinline__ double block_sum8(const double a[kMaxRhs], double (*sh)[kMaxRhs]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int f;
  const double v = butterfly8(a, lane, &f);
  if ((lane & 7) == 0) sh[wid][f] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x < kMaxRhs) {
    const int j = threadIdx.x;
    if constexpr (NW == 4) r = (sh[0][j] + sh[1][j]) + (sh[2][j] + sh[3][j]);
    else if constexpr (NW == 2) r = sh[0][j] + sh[1][j];
    else r = sh[0][j];
  }
  __syncthreads();
  return r;
}

__device__ __forceinline__ int64_t packed_col(int i, int k) { return (int64_t)k * (k + 1) / 2 + i; }

// Load / store the R values of one row or column (R == 8: four 16-byte accesses; the vectors
// are 64-byte aligned then).  Missing entries read as zero.
__device__ __forceinline__ void load_r(const double* __restrict__ p, int R, double v[kMaxRhs]) {
  if (R == kMaxRhs) {
    const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const double2 t = q[m];
      v[2 * m] = t.x;
      v[2 * m + 1] = t.y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < kMaxRhs; ++j) v[j] = j < R ? p[j] : 0.0;
  }
}
__device__ __forceinline__ void store_r(double* __restrict__ p, int R, const double v[kMaxRhs]) {
  if (R == kMaxRhs) {
    double2* q = reinterpret_cast<double2*>(p);
#pragma unroll
    for (int m = 0; m < 4; ++m) q[m] = double2{v[2 * m], v[2 * m + 1]};
  } else {
#pragma unroll
    for (int j = 0; j < kMaxRhs; ++j)
      if (j < R) p[j] = v[j];
  }
}

// y = R_b^{-1} c for the block's coefficients c in LDS (cs[k][rhs], K <= 512); the result
// replaces cs.  The column-packed factor is streamed through LDS (fs, nfs doubles) in runs of
// whole columns with coalesced loads; thread t accumulates outputs i = t and t + 256 (i < K) over
// the staged columns k >= i.
__device__ __forceinline__ void bj_apply_lds(const double* __restrict__ rc, int K,
                                             double (*cs)[kMaxRhs], double* fs, int nfs) {
  double acc[2][kMaxRhs];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int j = 0; j < kMaxRhs; ++j) acc[h][j] = 0.0;
  int k0 = 0;
  while (k0 < K) {
    const int64_t base = packed_col(0, k0);
    int k1 = k0 + 1;
    while (k1 < K && packed_col(0, k1 + 1) - base <= nfs) ++k1;
    const int cnt = (int)(packed_col(0, k1) - base);
    for (int e = threadIdx.x; e < cnt; e += 256) fs[e] = rc[base + e];
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = threadIdx.x + 256 * h;
      if (i < K) {
        for (int k = (i > k0 ? i : k0); k < k1; ++k) {
          const double r = fs[packed_col(i, k) - base];
#pragma unroll
          for (int j = 0; j < kMaxRhs; ++j) acc[h][j] += r * cs[k][j];
        }
      }
    }
    __syncthreads();
    k0 = k1;
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = threadIdx.x + 256 * h;
    if (i < K) {
#pragma unroll
      for (int j = 0; j < kMaxRhs; ++j) cs[i][j] = acc[h][j];
    }
  }
  __syncthreads();
}

constexpr int kFacStage = 2048;   // doubles of a packed factor staged per round in A.v

// Partial rows of Y = A V: per block point, the block's contribution for every right-hand side,
// tpart[(p_off + p) * R + rhs] (V scaled per pair by 1/alpha, or 0 once the pair is done).  The
// waves take 64-point runs of the block in turn; each lane loads FA feature entries ahead of
// their products (the autotuner's choice; the sum order over features does not depend on it).
// The block's coefficients are staged in dynamic LDS, cs[k][rhs] for k < nk (the launch sizes it
// for the largest block).  Without runs a workgroup takes a whole block; with runs (patch blocks,
// several hundred points over up to 512 columns) it takes one run of at most 256 points, so its
// four waves get one 64-point group each (runs of a block are dealt to one XCD; blk = -1 pads).
template <int PREC, int FA>
__global__ void __launch_bounds__(256) k_bt_mvb(const DevBlock* __restrict__ blocks,
                                                const Tile* __restrict__ runs,
                                                const void* __restrict__ A,
                                                const double* __restrict__ v, int R,
                                                const SolveState* __restrict__ st,
                                                double* __restrict__ tpart) {
  extern __shared__ double cs_dyn[];
  double (*cs)[kMaxRhs] = reinterpret_cast<double (*)[kMaxRhs]>(cs_dyn);
  const Tile run = runs ? runs[blockIdx.x] : Tile{(int32_t)blockIdx.x, 0};
  if (run.blk < 0) return;
  const DevBlock B = blocks[run.blk];
  if (inst_all_done(st, B.inst, R)) return;
  const int K = B.nk;
  for (int e = threadIdx.x; e < K * kMaxRhs; e += 256) {
    const int k = e >> 3, j = e & 7;
    cs[k][j] = j < R ? v[(int64_t)(B.q0 + k) * R + j] * pair_scale(st, B.inst * R + j, true) : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int n = runs ? min(B.n, run.p0 + 256) : B.n, ld = B.ld;
  for (int p0 = run.p0 + wid * 64; p0 < n; p0 += 256) {
    const int p = p0 + lane;
    if (p < n) {
      double acc[kMaxRhs];
#pragma unroll
      for (int j = 0; j < kMaxRhs; ++j) acc[j] = 0.0;
      const int64_t base = B.a_off + p;
      int k = 0;
      for (; k + FA <= K; k += FA) {
        double a[FA];
#pragma unroll
        for (int q = 0; q < FA; ++q) a[q] = load_entry<PREC>(A, base + (int64_t)(k + q) * ld);
#pragma unroll
        for (int q = 0; q < FA; ++q)
#pragma unroll
          for (int j = 0; j < kMaxRhs; ++j) acc[j] += a[q] * cs[k + q][j];
      }
      for (; k < K; ++k) {
        const double a = load_entry<PREC>(A, base + (int64_t)k * ld);
#pragma unroll
        for (int j = 0; j < kMaxRhs; ++j) acc[j] += a * cs[k][j];
      }
      store_r(tpart + (B.p_off + p) * R, R, acc);
    }
  }
}

// One workgroup per row tile of 256 rows, RPT rows per thread (the autotuner's choice: 256/RPT
// threads); the rows' own sums do not depend on RPT, the per-tile norm partial adds its rows in
// another order when RPT changes.
template <int RPT>
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
  constexpr int NT = 256 / RPT;
  __shared__ double sh[4][kMaxRhs];
  const RowTile t = rtiles[blockIdx.x];
  if (mode == ROW_LSQR_U && inst_all_done(st, t.inst, R)) return;
  const Geo& g = geos[t.inst];
  const InstInfo I = insts[t.inst];
  double acc[kMaxRhs];
#pragma unroll
  for (int j = 0; j < kMaxRhs; ++j) acc[j] = 0.0;
  for (int ri = 0; ri < RPT; ++ri) {
  const int64_t r = t.r0 + threadIdx.x + ri * NT;
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
      const int ncx = jx1 - jx0 + 1, ncy = jy1 - jy0 + 1;
      if (ncx <= 3 && ncy <= 3) {
        // up to 3 x 3 covering blocks (width ratio < 3): block records first, then the
        // partial rows, summed jx-major, jy-minor; absent slots read the first block, add 0
        int64_t off[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const bool ok = a < ncx && c < ncy;
            const DevBlock& B = blocks[g.bbase[l] + (jx0 + (ok ? a : 0)) * Jy + jy0 + (ok ? c : 0)];
            off[a * 3 + c] = ok ? (B.p_off + (ix - B.ix0) * B.ny + (iy - B.iy0)) * R : -1;
          }
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          if (off[q] >= 0) {
            double tv[kMaxRhs];
            load_r(tpart + off[q], R, tv);
#pragma unroll
            for (int j = 0; j < kMaxRhs; ++j) y[j] += tv[j];
          }
        }
      } else {
        for (int jx = jx0; jx <= jx1; ++jx)
          for (int jy = jy0; jy <= jy1; ++jy) {
            const DevBlock& B = blocks[g.bbase[l] + jx * Jy + jy];
            const int p = (ix - B.ix0) * B.ny + (iy - B.iy0);
            double tv[kMaxRhs];
            load_r(tpart + (B.p_off + p) * R, R, tv);
#pragma unroll
            for (int j = 0; j < kMaxRhs; ++j) y[j] += tv[j];
          }
      }
    }
    double* o = out + r * R;
    if (mode == ROW_STORE) {
#pragma unroll
      for (int j = 0; j < kMaxRhs; ++j)
        if (j < R) o[j] = y[j];
    } else if (mode == ROW_LSQR_U) {
#pragma unroll
      for (int j = 0; j < kMaxRhs; ++j) {
        if (j < R) {
          const SolveState& s = st[t.inst * R + j];
          const double u = s.done ? 0.0 : y[j] - s.alpha * s.su * o[j];
          o[j] = u;
          acc[j] += u * u;
        }
      }
    } else if (mode == ROW_RESID) {
      const double* bv = bvec + r * R;
#pragma unroll
      for (int j = 0; j < kMaxRhs; ++j) {
        if (j < R) {
          const double u = bv[j] - y[j];
          o[j] = u;
          acc[j] += u * u;
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < kMaxRhs; ++j) {
        if (j < R) {
          o[j] = y[j];
          acc[j] += y[j] * y[j];
        }
      }
    }
  }
  }   // rows of this thread
  if (mode != ROW_STORE) {
    const double sum = block_sum8<NT / 64>(acc, sh);
    if (threadIdx.x < kMaxRhs) red[(int64_t)blockIdx.x * kMaxRhs + threadIdx.x] = sum;
  }
}

template <int PREC> struct StoreT;
template <> struct StoreT<ELMFB_FP64> { typedef double t; };
template <> struct StoreT<ELMFB_FP32> { typedef float t; };
template <> struct StoreT<ELMFB_BF16> { typedef uint16_t t; };
template <> struct StoreT<ELMFB_FP16> { typedef _Float16 t; };

template <int PREC>
__device__ __forceinline__ double to_f64(typename StoreT<PREC>::t x) {
  if constexpr (PREC == ELMFB_BF16) return bf16_to_f64(x);
  else return (double)x;
}

// Column epilogue of the A^T U passes for one block: thread with column kk >= 0 holds the
// block's column kk in x; COL_STORE stores it, COL_LSQR_V applies v = x - beta sv v, COL_STORE_SQ
// stores and squares; per-block partial squared norms go to red[block][rhs].  Every thread of
// the workgroup must call it.
__device__ __forceinline__ void col_epilogue(int q0, int inst, int R, int kk,
                                             const double x[kMaxRhs], int mode,
                                             const SolveState* __restrict__ st,
                                             double* __restrict__ out, double* __restrict__ red,
                                             double (*sh)[kMaxRhs]) {
  double sq[kMaxRhs];
#pragma unroll
  for (int j = 0; j < kMaxRhs; ++j) sq[j] = 0.0;
  if (kk >= 0) {
    double* o = out + (int64_t)(q0 + kk) * R;
    if (mode == COL_STORE) {
      store_r(o, R, x);
    } else if (mode == COL_LSQR_V) {
      double vv[kMaxRhs];
      load_r(o, R, vv);
#pragma unroll
      for (int j = 0; j < kMaxRhs; ++j) {
        if (j < R) {
          const SolveState& ps = st[inst * R + j];
          if (ps.done) vv[j] = 0.0;
          else if (ps.beta > 0.0) vv[j] = x[j] - ps.beta * ps.sv * vv[j];
          sq[j] = vv[j] * vv[j];
        }
      }
      store_r(o, R, vv);
    } else {
      store_r(o, R, x);
#pragma unroll
      for (int j = 0; j < kMaxRhs; ++j) sq[j] = x[j] * x[j];
    }
  }
  if (mode != COL_STORE) {
    const double sum = block_sum8(sq, sh);
    if (threadIdx.x < kMaxRhs) red[(int64_t)blockIdx.x * kMaxRhs + threadIdx.x] = sum;
  }
}

// X = A^T U for one slice of <= 128 columns of a block and every right-hand side (a subdomain
// block is one slice; a patch block of the block-Jacobi preconditioner has several, each reading
// the patch's rows of U).  Tiles of TP points
// are staged in LDS (the block's K feature rows, and U on the tile's rows gathered from the
// grid), the next tile's loads in flight while the current one is reduced; thread (k, s) owns
// feature k and half s of the tile's points, so no cross-lane reduction is needed.  The
// epilogue stores the block's columns (COL_STORE), applies the LSQR step v = x - beta sv v
// (COL_LSQR_V) or stores and squares (COL_STORE_SQ); per-block partial squared norms go to
// red[slice][rhs].
template <int PREC, int TP>
__global__ void __launch_bounds__(256) k_bt_rmvb(const Geo* __restrict__ geos,
                                                 const InstInfo* __restrict__ insts,
                                                 const DevBlock* __restrict__ blocks,
                                                 const ColSlice* __restrict__ slices,
                                                 const void* __restrict__ A,
                                                 const double* __restrict__ u, int R,
                                                 const SolveState* __restrict__ st, int mode,
                                                 double* __restrict__ out,
                                                 double* __restrict__ red) {
  typedef typename StoreT<PREC>::t in_t;
  typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
  constexpr int VEC = 16 / (int)sizeof(in_t);        // entries per 16-byte load
  constexpr int NV = kBatchMaxK * TP / VEC / 256;    // 16-byte loads of A per thread per tile
  constexpr int TV = TP / VEC;                       // loads per feature row of a tile
  constexpr int NU = (TP * kMaxRhs + 255) / 256;     // U entries per thread per tile
  static_assert(NV >= 1 && NV * 256 * VEC == kBatchMaxK * TP, "tile shape");
  __shared__ __align__(16) in_t At[kBatchMaxK][TP + 1];
  __shared__ double us[TP][kMaxRhs];
  __shared__ double xs[kBatchMaxK][kMaxRhs];
  __shared__ double sh[4][kMaxRhs];
  const ColSlice S = slices[blockIdx.x];
  const DevBlock B = blocks[S.blk];
  if (inst_all_done(st, B.inst, R)) return;
  const Geo& g = geos[B.inst];
  const int64_t row0 = insts[B.inst].row_off;
  const int K = min(kBatchMaxK, B.nk - S.k0), n = B.n, gny = g.ny;
  const in_t* Ab = static_cast<const in_t*>(A) + B.a_off + (int64_t)S.k0 * B.ld;

  // every U entry a thread stages has right-hand side threadIdx.x & 7: its pair scale is read
  // once, and applied when the tile is written to LDS, so the loads of the next tile stay in
  // flight while the current one is reduced
  const int ju = threadIdx.x & 7;
  const double usc = ju < R ? pair_scale(st, B.inst * R + ju, false) : 0.0;
  // A is read 16 bytes at a time: VEC consecutive points of one feature row (rows start on
  // 8-entry boundaries and ld is a multiple of 8, so a load lies wholly before or after ld; the
  // row padding between n and ld holds zeros)
  u32x4_t ra[NV];
  double ru[NU];
  auto fetch = [&](int p0) {
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      const int g4 = threadIdx.x + 256 * m;
      const int k = g4 / TV, p = p0 + (g4 - (g4 / TV) * TV) * VEC;
      ra[m] = (k < K && p + VEC <= B.ld)
                  ? *reinterpret_cast<const u32x4_t*>(Ab + (int64_t)k * B.ld + p)
                  : u32x4_t{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      const int e = threadIdx.x + 256 * m;
      const int c = e >> 3, j = e & 7;
      const int p = p0 + c;
      double val = 0.0;
      if (c < TP && j < R && p < n) {
        const int lx = p / B.ny, ly = p - (p / B.ny) * B.ny;
        const int64_t r = row0 + (int64_t)(B.ix0 + lx) * gny + (B.iy0 + ly);
        val = u[r * R + j];
      }
      ru[m] = val;
    }
  };

  const int k = threadIdx.x & 127, s = threadIdx.x >> 7;
  double acc[kMaxRhs];
#pragma unroll
  for (int j = 0; j < kMaxRhs; ++j) acc[j] = 0.0;
  fetch(0);
  for (int p0 = 0; p0 < n; p0 += TP) {
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      const int g4 = threadIdx.x + 256 * m;
      const int k = g4 / TV, c = (g4 - (g4 / TV) * TV) * VEC;
      in_t v[VEC];
      __builtin_memcpy(v, &ra[m], 16);
#pragma unroll
      for (int i = 0; i < VEC; ++i) At[k][c + i] = v[i];
    }
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      const int e = threadIdx.x + 256 * m;
      if ((e >> 3) < TP) us[e >> 3][e & 7] = ru[m] * usc;
    }
    __syncthreads();
    if (p0 + TP < n) fetch(p0 + TP);
    if (k < K) {
#pragma unroll
      for (int cc = 0; cc < TP / 2; ++cc) {
        const int c = s * (TP / 2) + cc;
        const double a = to_f64<PREC>(At[k][c]);
#pragma unroll
        for (int j = 0; j < kMaxRhs; ++j) acc[j] += a * us[c][j];
      }
    }
    __syncthreads();
  }
  // combine the two halves: thread (k, 0) ends with column k of the block
  if (s == 1 && k < K) {
#pragma unroll
    for (int j = 0; j < kMaxRhs; ++j) xs[k][j] = acc[j];
  }
  __syncthreads();
  if (s == 0 && k < K) {
#pragma unroll
    for (int j = 0; j < kMaxRhs; ++j) acc[j] += xs[k][j];
  }
  col_epilogue(B.q0 + S.k0, B.inst, R, s == 0 && k < K ? k : -1, acc, mode, st, out, red, sh);
}

// x = x0 + R^{-1} y per block and right-hand side (x0 may be NULL; x may alias x0).  y is in
// the blocks' column order; with perm (patch blocks) column q of that order is column perm[q] of
// x and x0, else the two orders agree.
__global__ void __launch_bounds__(256) k_bt_bj_recover(const DevBlock* __restrict__ blocks,
                                                       const double* __restrict__ rc,
                                                       const int64_t* __restrict__ foff,
                                                       const int32_t* __restrict__ perm, int R,
                                                       const double* __restrict__ y,
                                                       const double* x0, double* x) {
  __shared__ double cs[kPatchMaxK][kMaxRhs];
  __shared__ double fs[kFacStage];
  const DevBlock B = blocks[blockIdx.x];
  const int K = B.nk;
  for (int e = threadIdx.x; e < K * kMaxRhs; e += 256) {
    const int k = e >> 3, j = e & 7;
    cs[k][j] = j < R ? y[(int64_t)(B.q0 + k) * R + j] : 0.0;
  }
  __syncthreads();
  bj_apply_lds(rc + foff[blockIdx.x], K, cs, fs, kFacStage);
  for (int e = threadIdx.x; e < K * R; e += 256) {
    const int k = e / R, j = e - (e / R) * R;
    const int64_t q = perm ? (int64_t)perm[B.q0 + k] : (int64_t)(B.q0 + k);
    const int64_t o = q * R + j;
    x[o] = (x0 ? x0[o] : 0.0) + cs[k][j];
  }
}

// ---------------------------------------------------------------- recurrences

// The per-pair scalar kernels run one wavefront per (instance, rhs) pair: pair
// blockIdx.x * 4 + wave.  Sum of an instance's tile partials for one right-hand side: each lane
// sums tiles lane, lane + 64, ..., then a fixed butterfly over the wavefront (lane 0's value is
// the one used).
__device__ __forceinline__ double seg_sum(const double* red, int t0, int t1, int j) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int t = t0 + lane; t < t1; t += 64) s += red[(int64_t)t * kMaxRhs + j];
  return wave_sum(s);
}

__device__ __forceinline__ int pair_index() { return blockIdx.x * 4 + (threadIdx.x >> 6); }

// bnorm = ||h||, beta = ||u||, su = 1/beta  (row partials)
__global__ void k_bt_lsqr_init(SolveState* st, const InstInfo* __restrict__ insts, int n_inst,
                               int R, const double* __restrict__ red_b,
                               const double* __restrict__ red_u, double atol, double btol,
                               int iter_lim, const BtOuter* __restrict__ ot, double inner_rel) {
  const int idx = pair_index();
  if (idx >= n_inst * R) return;
  const int i = idx / R, j = idx - (idx / R) * R;
  const InstInfo I = insts[i];
  const double su2 = seg_sum(red_u, I.rt0, I.rt1, j), sb2 = seg_sum(red_b, I.rt0, I.rt1, j);
  if ((threadIdx.x & 63) != 0) return;
  SolveState s{};
  const double beta = sqrt(su2);
  s.bnorm = sqrt(sb2);
  s.beta = beta;
  s.su = beta > 0.0 ? 1.0 / beta : 0.0;
  s.atol = atol;
  s.btol = btol;
  s.iter_lim = iter_lim;
  s.rel_l2 = -1.0;
  if (ot) {
    const BtOuter o = ot[idx];
    if (o.done) {
      s.done = 1;
      s.istop = 1;
    } else if (beta > 0.0) {
      s.btol = inner_rel * o.btol * o.hnorm / beta;
    }
  }
  st[idx] = s;
}

// Outer FP64 residual check of a refined solve from the row partials of the current residual.
// mode 1: the partials are those of h; record ||h|| (fresh state).  mode 2: the residual of a
// warm start; no step is counted.  mode 0: after a refinement step, whose inner iterations are
// added.  A pair stops once ||h - M c|| <= btol ||h|| (istop 1), once ||A^T r|| <= atol ||A|| ||r||
// (istop 2: least-squares optimality; red_a holds the per-block partials of ||A^T r||^2 and ||A||
// is the inner LSQR's estimate), or after outer_lim steps (istop 7).
__global__ void k_bt_outer_check(BtOuter* ot, const SolveState* __restrict__ st,
                                 const InstInfo* __restrict__ insts, int n_inst, int R,
                                 const double* __restrict__ red_r,
                                 const double* __restrict__ red_a, double atol, int mode,
                                 double btol, int outer_lim) {
  const int idx = pair_index();
  if (idx >= n_inst * R) return;
  const InstInfo I = insts[idx / R];
  const double rn = sqrt(seg_sum(red_r, I.rt0, I.rt1, idx - (idx / R) * R));
  const bool use_a = mode == 0 && red_a && atol > 0.0;
  const double an = use_a ? sqrt(seg_sum(red_a, I.b0, I.b1, idx - (idx / R) * R)) : 0.0;
  if ((threadIdx.x & 63) != 0) return;
  BtOuter o = mode == 1 ? BtOuter{} : ot[idx];
  if (mode == 1) {
    o.hnorm = rn;
    o.btol = btol;
  } else if (mode == 0 && !o.done) {
    o.iters += st[idx].itn;
    o.outer += 1;
  }
  o.rnorm = rn;
  if (!o.done) {
    if (o.hnorm == 0.0) {
      o.done = 1;
      o.istop = 0;
    } else if (rn <= o.btol * o.hnorm) {
      o.done = 1;
      o.istop = 1;
    } else if (use_a && an <= atol * st[idx].anorm * rn) {
      o.done = 1;
      o.istop = 2;
    } else if (o.outer >= outer_lim) {
      o.done = 1;
      o.istop = 7;
    }
  }
  ot[idx] = o;
}

// alpha = ||A^T u||, phibar = beta, rhobar = alpha  (column partials)
__global__ void k_bt_lsqr_init_alpha(SolveState* st, const InstInfo* __restrict__ insts,
                                     int n_inst, int R, const double* __restrict__ red) {
  const int idx = pair_index();
  if (idx >= n_inst * R) return;
  const int i = idx / R, j = idx - (idx / R) * R;
  const InstInfo I = insts[i];
  const double sa2 = seg_sum(red, I.b0, I.b1, j);
  if ((threadIdx.x & 63) != 0) return;
  SolveState& s = st[idx];
  const double beta = s.beta;
  const double alpha = beta > 0.0 ? sqrt(sa2) : 0.0;
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
  const int idx = pair_index();
  if (idx >= n_inst * R) return;
  SolveState& s = st[idx];
  if (s.done) return;
  const InstInfo I = insts[idx / R];
  const double beta = sqrt(seg_sum(red, I.rt0, I.rt1, idx - (idx / R) * R));
  if ((threadIdx.x & 63) != 0) return;
  s.beta = beta;
  if (beta > 0.0) {
    s.su = 1.0 / beta;
    s.anorm = sqrt(s.anorm * s.anorm + s.alpha * s.alpha + beta * beta);
  }
}

__global__ void k_bt_lsqr_alpha(SolveState* st, const InstInfo* __restrict__ insts, int n_inst,
                                int R, const double* __restrict__ red) {
  const int idx = pair_index();
  if (idx >= n_inst * R) return;
  SolveState& s = st[idx];
  if (s.done) return;
  const InstInfo I = insts[idx / R];
  const double sa2 = seg_sum(red, I.b0, I.b1, idx - (idx / R) * R);
  if ((threadIdx.x & 63) != 0) return;
  const double beta = s.beta;
  double alpha = s.alpha;
  if (beta > 0.0) {
    alpha = sqrt(sa2);
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

// x += t1 w, w = v sv + t2 w per (column, rhs) of a column tile: consecutive threads take
// consecutive elements of the interleaved vectors; per-rhs partials of ||x||^2.
__global__ void __launch_bounds__(256) k_bt_update(const Geo* __restrict__ geos,
                                                   const InstInfo* __restrict__ insts,
                                                   const ColTile* __restrict__ ctiles, int R,
                                                   double* __restrict__ x,
                                                   double* __restrict__ w,
                                                   const double* __restrict__ v,
                                                   const SolveState* __restrict__ st,
                                                   double* __restrict__ red) {
  __shared__ double sh[4][kMaxRhs];
  const ColTile t = ctiles[blockIdx.x];
  if (inst_all_done(st, t.inst, R)) return;
  const InstInfo I = insts[t.inst];
  const int64_t q_end = I.col_off + geos[t.inst].n_phi;
  const int64_t ncol = (q_end - t.q0) < 256 ? (q_end - t.q0) : 256;
  const int64_t e0 = (int64_t)t.q0 * R, ne = ncol * R;
  double acc[kMaxRhs];
#pragma unroll
  for (int j = 0; j < kMaxRhs; ++j) acc[j] = 0.0;
  for (int m = 0; m < kMaxRhs; ++m) {
    const int64_t e = threadIdx.x + 256 * (int64_t)m;
    if (e < ne) {
      const int j = (int)((e0 + e) % R);
      const SolveState& s = st[t.inst * R + j];
      double xv = x[e0 + e];
      if (!s.done) {
        const double wv = w[e0 + e];
        xv = xv + s.t1 * wv;
        x[e0 + e] = xv;
        w[e0 + e] = v[e0 + e] * s.sv + s.t2 * wv;
      }
#pragma unroll
      for (int jj = 0; jj < kMaxRhs; ++jj) acc[jj] += (jj == j) ? xv * xv : 0.0;
    }
  }
  const double sum = block_sum8(acc, sh);
  if (threadIdx.x < kMaxRhs) red[(int64_t)blockIdx.x * kMaxRhs + threadIdx.x] = sum;
}

__global__ void k_bt_lsqr_stop(SolveState* st, const InstInfo* __restrict__ insts, int n_inst,
                               int R, const double* __restrict__ red) {
  const int idx = pair_index();
  if (idx >= n_inst * R) return;
  SolveState& s = st[idx];
  if (s.done) return;
  const InstInfo I = insts[idx / R];
  const double eps = 2.220446049250313e-16;
  const double xnorm = sqrt(seg_sum(red, I.ct0, I.ct1, idx - (idx / R) * R));
  if ((threadIdx.x & 63) != 0) return;
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

__global__ void __launch_bounds__(256) k_bt_count_outer(const BtOuter* __restrict__ ot, int n,
                                                        int32_t* __restrict__ out) {
  __shared__ double sh[4];
  double c = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) c += ot[i].done ? 0.0 : 1.0;
  const double s = block_sum256(c, sh);
  if (threadIdx.x == 0) *out = (int32_t)s;
}

// x = x0 + y (x0 may be NULL)
__global__ void k_bt_recover_plain(int64_t n, const double* __restrict__ y,
                                   const double* __restrict__ x0, double* __restrict__ x) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = (x0 ? x0[i] : 0.0) + y[i];
}

__global__ void k_bt_axpy(int64_t n, const double* __restrict__ y, double* __restrict__ x) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] += y[i];
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
  else if (lo_prec == ELMFB_FP16)
    hipLaunchKernelGGL(k_bt_assemble<ELMFB_FP16>, grid, blk, 0, s, geos, blocks, tiles, tab, W, b, A, A_lo);
  else
    hipLaunchKernelGGL(k_bt_assemble<-1>, grid, blk, 0, s, geos, blocks, tiles, tab, W, b, A, A_lo);
  return hipGetLastError();
}

hipError_t launch_bt_rhs(const Geo* geos, const InstInfo* insts, const RowTile* rt, int64_t n_rt,
                         int R, const double* f, double* h, int32_t* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_bt_rhs, dim3((unsigned)n_rt), dim3(256), 0, s, geos, insts, rt, R, f, h, bad);
  return hipGetLastError();
}

template <int FA>
static void mvb_fa(int prec, dim3 grid, size_t lds, const DevBlock* blocks, const Tile* runs,
                   const void* A, const double* v, int R, const SolveState* st, double* tpart,
                   hipStream_t s) {
  const dim3 blk(256);
  if (prec == ELMFB_FP32)
    hipLaunchKernelGGL((k_bt_mvb<ELMFB_FP32, FA>), grid, blk, lds, s, blocks, runs, A, v, R, st,
                       tpart);
  else if (prec == ELMFB_BF16)
    hipLaunchKernelGGL((k_bt_mvb<ELMFB_BF16, FA>), grid, blk, lds, s, blocks, runs, A, v, R, st,
                       tpart);
  else if (prec == ELMFB_FP16)
    hipLaunchKernelGGL((k_bt_mvb<ELMFB_FP16, FA>), grid, blk, lds, s, blocks, runs, A, v, R, st,
                       tpart);
  else
    hipLaunchKernelGGL((k_bt_mvb<ELMFB_FP64, FA>), grid, blk, lds, s, blocks, runs, A, v, R, st,
                       tpart);
}

hipError_t launch_bt_mvb(int prec, const DevBlock* blocks, const Tile* runs, int64_t n_grid,
                         int kmax, const void* A, const double* v, int R, const SolveState* st,
                         double* tpart, hipStream_t s, int fa) {
  if (n_grid == 0) return hipSuccess;
  if (kmax < 1 || kmax > kPatchMaxK) return hipErrorInvalidValue;
  const dim3 grid((unsigned)n_grid);
  const size_t lds = (size_t)kmax * kMaxRhs * sizeof(double);
  if (fa == 4) mvb_fa<4>(prec, grid, lds, blocks, runs, A, v, R, st, tpart, s);
  else if (fa == 8) mvb_fa<8>(prec, grid, lds, blocks, runs, A, v, R, st, tpart, s);
  else if (fa == 16) mvb_fa<16>(prec, grid, lds, blocks, runs, A, v, R, st, tpart, s);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_bt_gather(const Geo* geos, const InstInfo* insts, const DevBlock* blocks,
                            const int32_t* cov, const RowTile* rt, int64_t n_rt,
                            const double* tpart, int mode, int R, double* out, const double* bvec,
                            const SolveState* st, double* red, hipStream_t s, int rpt) {
  if (rpt == 1)
    hipLaunchKernelGGL(k_bt_gather<1>, dim3((unsigned)n_rt), dim3(256), 0, s, geos, insts, blocks,
                       cov, rt, tpart, mode, R, out, bvec, st, red);
  else if (rpt == 2)
    hipLaunchKernelGGL(k_bt_gather<2>, dim3((unsigned)n_rt), dim3(128), 0, s, geos, insts, blocks,
                       cov, rt, tpart, mode, R, out, bvec, st, red);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_bt_rmvb(int prec, int tp, const Geo* geos, const InstInfo* insts,
                          const DevBlock* blocks, const ColSlice* slices, int64_t n_slices,
                          const void* A, const double* u, int R, const SolveState* st, int mode,
                          double* out, double* red, hipStream_t s) {
  if (n_slices == 0) return hipSuccess;
  const dim3 grid((unsigned)n_slices), blk(256);
#define RMVB(P, T)                                                                          \
  hipLaunchKernelGGL((k_bt_rmvb<P, T>), grid, blk, 0, s, geos, insts, blocks, slices, A, u, R, st, \
                     mode, out, red)
  if (prec == ELMFB_FP32) {
    if (tp == 16) RMVB(ELMFB_FP32, 16); else if (tp == 32) RMVB(ELMFB_FP32, 32);
    else if (tp == 64) RMVB(ELMFB_FP32, 64); else return hipErrorInvalidValue;
  } else if (prec == ELMFB_BF16) {
    if (tp == 16) RMVB(ELMFB_BF16, 16); else if (tp == 32) RMVB(ELMFB_BF16, 32);
    else if (tp == 64) RMVB(ELMFB_BF16, 64); else return hipErrorInvalidValue;
  } else if (prec == ELMFB_FP16) {
    if (tp == 16) RMVB(ELMFB_FP16, 16); else if (tp == 32) RMVB(ELMFB_FP16, 32);
    else if (tp == 64) RMVB(ELMFB_FP16, 64); else return hipErrorInvalidValue;
  } else {
    // FP64 stages of 64 points exceed the static LDS limit
    if (tp == 16) RMVB(ELMFB_FP64, 16); else if (tp == 32) RMVB(ELMFB_FP64, 32);
    else return hipErrorInvalidValue;
  }
#undef RMVB
  return hipGetLastError();
}

hipError_t launch_bt_bj_recover(const DevBlock* blocks, int64_t n_blocks, const double* rc,
                                const int64_t* foff, const int32_t* perm, int R, const double* y,
                                const double* x0, double* x, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bt_bj_recover, dim3((unsigned)n_blocks), dim3(256), 0, s, blocks, rc,
                     foff, perm, R, y, x0, x);
  return hipGetLastError();
}

hipError_t launch_bt_recover_plain(int64_t n, const double* y, const double* x0, double* x,
                                   hipStream_t s) {
  int64_t nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_bt_recover_plain, dim3((unsigned)nb), dim3(256), 0, s, n, y, x0, x);
  return hipGetLastError();
}

hipError_t launch_bt_axpy(int64_t n, const double* y, double* x, hipStream_t s) {
  int64_t nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_bt_axpy, dim3((unsigned)nb), dim3(256), 0, s, n, y, x);
  return hipGetLastError();
}

static dim3 pairs_grid(int n) { return dim3((unsigned)((n + 3) / 4)); }   // a wavefront per pair

hipError_t launch_bt_lsqr_init(SolveState* st, const InstInfo* insts, int n_inst, int R,
                               const double* red_b, const double* red_u, double atol, double btol,
                               int iter_lim, const BtOuter* ot, double inner_rel, hipStream_t s) {
  hipLaunchKernelGGL(k_bt_lsqr_init, pairs_grid(n_inst * R), dim3(256), 0, s, st, insts, n_inst, R,
                     red_b, red_u, atol, btol, iter_lim, ot, inner_rel);
  return hipGetLastError();
}
hipError_t launch_bt_outer_check(BtOuter* ot, const SolveState* st, const InstInfo* insts,
                                 int n_inst, int R, const double* red_r, const double* red_a,
                                 double atol, int mode, double btol, int outer_lim,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_bt_outer_check, pairs_grid(n_inst * R), dim3(256), 0, s, ot, st, insts,
                     n_inst, R, red_r, red_a, atol, mode, btol, outer_lim);
  return hipGetLastError();
}
hipError_t launch_bt_count_outer(const BtOuter* ot, int n, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_bt_count_outer, dim3(1), dim3(256), 0, s, ot, n, out);
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
