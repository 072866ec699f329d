// Internal structures shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "elmfb.h"

namespace elmfb {

constexpr int kMaxLevels = ELMFB_MAX_LEVELS;
constexpr int kTile = 256;          // points per assembly / A.v tile (one per thread)
constexpr int kRowAlign = 8;        // stored rows start on 8-element boundaries (16 B in FP16)
constexpr int kChunkPts = 2048;     // points per A^T u chunk (8 per thread of 256)
constexpr int kHistCap = 32768;     // bidiagonalisation steps an LSQR run records
constexpr int kRedBlocks = 1024;    // upper bound on per-workgroup partial sums of a reduction
// Iterations per captured graph: a graph of a Krylov loop is one chain of ~10 kernels per step,
// and instantiating very long chains exhausts the runtime (a 15,000-step capture ended the
// process); a longer run between host checks replays graphs of at most this many steps.
constexpr int kGraphMaxSteps = 1000;

// One subdomain's block of the matrix: K rows (features) x n points of its box, feature-major.
struct DevBlock {
  int64_t a_off;    // element offset of the block in the stored matrix (a multiple of kRowAlign)
  int64_t p_off;    // offset of the block's points in the per-block-point arrays
  int32_t q0;       // first global column
  int32_t n;        // points in the box = nx * ny
  int32_t ld;       // row stride of the stored block [K][ld]: n rounded up to kRowAlign; the
                    // padding entries hold zeros
  int32_t ix0, nx;  // box along x (grid indices)
  int32_t iy0, ny;  // box along y
  int32_t tabx;     // offset of the x-axis envelope table entries for ix0..ix0+nx-1
  int32_t taby;     // offset of the y-axis envelope table entries for iy0..iy0+ny-1
  int32_t level;
  int32_t inst;     // instance of a batch (0 for a single problem)
  int32_t jx, jy;   // subdomain indices along the axes within the level (patch indices for a
                    // patch block)
  int32_t nk;       // columns of the block: K for a subdomain; for a patch of the batched
                    // block-Jacobi preconditioner, the columns of all its member subdomains
};

constexpr int kGramChunk = 4096;  // shared points per Gram chunk

// One overlapping pair (bi <= bj) of subdomain blocks and its shared box of grid points.
struct GramPair {
  int32_t bi, bj;
  int32_t ix0, nx, iy0, ny;   // shared box
  int64_t g_off;              // element offset of G_ij [K][K] in the Gram storage
  int32_t c0, nchunks;        // first global chunk, number of chunks
  int64_t p_off;              // first partial slot (pairs with several chunks)
};

struct GramChunk {
  int32_t pair;
  int32_t s0;                 // first shared point of the chunk (box row-major)
};

// ---- batches of independent instances with several right-hand sides
constexpr int kMaxRhs = 8;
constexpr int kBatchMaxK = 128;      // features per subdomain in a batch
// Columns of a patch block (P^d neighbouring subdomains of a level taken as one block of the
// batched block-Jacobi preconditioner).
constexpr int kPatchMaxK = 512;

// <= kBatchMaxK consecutive columns of one block: the unit of work of the batched M^T U pass
// (a subdomain block is one slice, a patch block several).
struct ColSlice {
  int32_t blk;
  int32_t k0;       // first column of the slice within the block
};

// One tile of <= 128 x 128 entries of a block's diagonal Gram block G_b = M_b^T M_b: rows
// [i0, i0 + 128) and columns [j0, j0 + 128), i0 <= j0 (the factorisation reads the upper
// triangle only).
struct GramTask {
  int32_t blk;
  int32_t i0, j0;
};
// Points per LDS stage of the batched A^T U pass; the autotuner picks one of these.
constexpr int kBtTileChoices[3] = {16, 32, 64};

struct RowTile {    // <= 256 consecutive rows of one instance
  int32_t inst;
  int32_t r0;       // first global row
};

struct ColTile {    // <= 256 consecutive columns of one instance
  int32_t inst;
  int32_t q0;       // first global column
};

struct InstInfo {
  int64_t row_off, col_off;   // global offsets of the instance's rows and columns
  int32_t rt0, rt1;           // its row tiles
  int32_t ct0, ct1;           // its column tiles
  int32_t b0, b1;             // its blocks
};

struct Tile {       // a run of <= kTile consecutive points of one block
  int32_t blk;
  int32_t p0;
};

// Everything a kernel needs to locate rows, blocks and subdomains.
struct Geo {
  int32_t dim;
  int32_t nx, ny;                 // grid (ny = 1 for dim 1)
  int32_t n_levels;
  int32_t K;
  int32_t n_blocks;
  int64_t n_rows;
  int64_t n_phi;
  double lo[2], hi[2], step[2];   // grid
  double inv_scale;               // 1 / (sqrt(N) L)
  double inv_sqrt_n;              // 1 / sqrt(N)
  double inv_levels;              // 1 / L
  int32_t op, ansatz;
  int32_t input_norm;             // ELMFB_INPUT_LOCAL or ELMFB_INPUT_GLOBAL
  double ansatz_omega;
  // per level and axis
  int32_t J[kMaxLevels][2];
  int32_t bbase[kMaxLevels];      // first block index of the level
  double cen_h[kMaxLevels][2];    // centre spacing (J > 1)
  double sigma[kMaxLevels][2];    // half-width
  double mid[kMaxLevels][2];      // centre for J == 1
  int32_t cov_off[kMaxLevels][2]; // offset into the covering table (per grid index: jlo, jhi)
  int32_t n_bc;                   // soft-constraint rows after the n_rows collocation rows
  int32_t domain;                 // ELMFB_DOMAIN_BOX or ELMFB_DOMAIN_L
  double op_coef[3];              // (m, mu, k) of the oscillator operator; k^2 of Helmholtz
  // L-shaped domain: the removed quarter starts at mid (points x > mid_x and y > mid_y); per
  // level the first entry of the block map (kept block index or -1 for every (jx, jy) of the
  // full grid) and of the per-axis window-sum tables (6 doubles per grid index: the sum over
  // every subdomain along the axis and over those with centre above mid, each with two
  // derivatives)
  double lmid[2];
  int64_t n_int;                  // grid points of the domain (interior rows)
  int32_t bmap_off[kMaxLevels];
  int32_t lsum_off[kMaxLevels][2];
  double bc_w;                    // weight of the Dirichlet rows at points
  // device tables of a single problem (unused by batches)
  const int32_t* bmap;            // block map
  const double* lsum;             // per-axis window sums (L domain)
  const double* bcpts;            // Dirichlet points [n_bc][2], then their values [n_bc]
};

// Soft-constraint conditions of a 1D problem: row b = w[b] (1/L) D^order[b][psi_q](x[b]),
// right-hand side w[b] val[b].
struct BcSpec {
  int32_t n;
  int32_t order[4];
  double x[4], w[4], val[4];
};

// Device-side scalar state of one Krylov solve (LSQR or CGLS), FP64 throughout.
struct SolveState {
  double alpha, beta;      // LSQR: current alpha, beta
  double su, sv;           // scale of the stored (unnormalised) u and v
  double rhobar, phibar;
  double anorm, bnorm, xnorm, rnorm, arnorm;
  double t1, t2;           // x += t1 w, w = v + t2 w
  double gamma;            // CGLS: ||s||^2
  double cg_a, cg_b;       // CGLS step sizes
  double rel_l2;           // last solution-error check
  double atol, btol;
  double target;           // rel-L2 target (0: off)
  int32_t itn, istop, done, iter_lim;
  int32_t target_hit;      // the rel-L2 check met the target
  int32_t pad_;
};

// FP64 outer state of an iteratively refined batched solve, one per (instance, rhs).
struct BtOuter {
  double hnorm;      // ||h||
  double rnorm;      // ||h - M c|| at the last check
  double btol;       // stop when rnorm <= btol hnorm
  int32_t done, outer, iters, istop;
};

// Convert an FP64 value to the bits of a 16-bit IEEE-style format with MB stored significand
// bits and EB exponent bits (bias 2^(EB-1) - 1) by round-to-nearest-even in one step: keep
// MB + 1 significant bits, or the fixed spacing 2^(emin - MB) below 2^emin; overflow to
// infinity.  bfloat16 is <7, 8>, IEEE binary16 is <10, 5>.
template <int MB, int EB>
__host__ __device__ inline uint16_t f64_to_small_rne(double x) {
  constexpr int kEmax = (1 << (EB - 1)) - 1;       // also the bias
  constexpr int kEmin = 1 - kEmax;
  constexpr int kSub = kEmin - MB;                 // exponent of the subnormal spacing
  constexpr uint64_t kMant = (1ull << MB) - 1;
  constexpr uint64_t kInf = ((1ull << EB) - 1) << MB;
  union { double d; uint64_t u; } dv;
  dv.d = x;
  const uint64_t sign = (dv.u >> 63) << 15;
  const uint64_t mag = dv.u & 0x7fffffffffffffffull;
  if (mag >= 0x7ff0000000000000ull) {               // inf or nan
    if (mag > 0x7ff0000000000000ull) return (uint16_t)(sign | kInf | (1ull << (MB - 1)));
    return (uint16_t)(sign | kInf);
  }
  const int e = (int)(mag >> 52);                    // biased FP64 exponent
  const uint64_t frac = mag & 0xfffffffffffffull;
  const int exp2v = (e == 0) ? -1022 : e - 1023;
  const uint64_t sig = (e == 0) ? frac : (frac | (1ull << 52));   // value = sig 2^(exp2v-52)
  int ulp_e = exp2v - MB;                            // spacing of the target at this binade
  if (ulp_e < kSub) ulp_e = kSub;
  const int sh = ulp_e - exp2v + 52;                 // q = sig / 2^sh, rounded
  uint64_t q, rem, half;
  if (sh >= 64) {
    return (uint16_t)sign;                           // far below half the smallest spacing
  } else if (sh <= 0) {
    q = sig << (-sh); rem = 0; half = 1;
  } else {
    q = sig >> sh;
    rem = sig & ((1ull << sh) - 1);
    half = 1ull << (sh - 1);
  }
  if (rem > half || (rem == half && (q & 1))) q += 1;
  if (q == 0) return (uint16_t)sign;
  // q is an integer multiple of 2^ulp_e; find the binade of q 2^ulp_e and rebuild the bits
  const int msb = 63 - __builtin_clzll(q);
  const int vexp = ulp_e + msb;
  if (vexp < kEmin) return (uint16_t)(sign | (q & kMant));     // subnormal: exponent field 0
  if (vexp > kEmax) return (uint16_t)(sign | kInf);
  const uint64_t mant = (msb >= MB) ? (q >> (msb - MB)) : (q << (MB - msb));
  return (uint16_t)(sign | ((uint64_t)(vexp + kEmax) << MB) | (mant & kMant));
}

__host__ __device__ inline uint16_t f64_to_bf16_rne(double x) { return f64_to_small_rne<7, 8>(x); }
__host__ __device__ inline uint16_t f64_to_fp16_rne(double x) { return f64_to_small_rne<10, 5>(x); }

__host__ __device__ inline double bf16_to_f64(uint16_t b) {
  union { float f; uint32_t u; } v;
  v.u = ((uint32_t)b) << 16;
  return (double)v.f;
}

// Exact value of IEEE binary16 bits (subnormals included).
__host__ __device__ inline double fp16_to_f64(uint16_t h) {
  const int e = (h >> 10) & 0x1f;
  const int m = h & 0x3ff;
  union { double d; uint64_t u; } v;
  if (e == 0x1f) {
    v.u = 0x7ff0000000000000ull | (m ? 0x8000000000000ull : 0);
  } else if (e == 0) {
    v.d = (double)m * 0x1p-24;                    // m 2^-24, exact
  } else {
    v.u = ((uint64_t)(e - 15 + 1023) << 52) | ((uint64_t)m << 42);
  }
  if (h & 0x8000) v.u |= 0x8000000000000000ull;
  return v.d;
}

}  // namespace elmfb
