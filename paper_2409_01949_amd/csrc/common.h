// Internal structures shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "elmfb.h"

namespace elmfb {

constexpr int kMaxLevels = ELMFB_MAX_LEVELS;
constexpr int kTile = 256;          // points per assembly / A.v tile (one per thread)
constexpr int kChunkPts = 2048;     // points per A^T u chunk (8 per thread of 256)
constexpr int kRedBlocks = 1024;    // upper bound on per-workgroup partial sums of a reduction

// One subdomain's block of the matrix: K rows (features) x n points of its box, feature-major.
struct DevBlock {
  int64_t a_off;    // element offset of the block in the stored matrix
  int64_t p_off;    // offset of the block's points in the per-block-point arrays
  int32_t q0;       // first global column
  int32_t n;        // points in the box = nx * ny
  int32_t ix0, nx;  // box along x (grid indices)
  int32_t iy0, ny;  // box along y
  int32_t tabx;     // offset of the x-axis envelope table entries for ix0..ix0+nx-1
  int32_t taby;     // offset of the y-axis envelope table entries for iy0..iy0+ny-1
  int32_t level;
  int32_t inst;     // instance of a batch (0 for a single problem)
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
  double ansatz_omega;
  // per level and axis
  int32_t J[kMaxLevels][2];
  int32_t bbase[kMaxLevels];      // first block index of the level
  double cen_h[kMaxLevels][2];    // centre spacing (J > 1)
  double sigma[kMaxLevels][2];    // half-width
  double mid[kMaxLevels][2];      // centre for J == 1
  int32_t cov_off[kMaxLevels][2]; // offset into the covering table (per grid index: jlo, jhi)
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

// Convert an FP64 value to bfloat16 bits with round-to-nearest-even (IEEE definition: keep
// 8 significant bits, or the fixed 2^-133 spacing below 2^-126; overflow to infinity).
__host__ __device__ inline uint16_t f64_to_bf16_rne(double x) {
  // Integer rounding of the 53-bit significand to the bf16 spacing, half to even.
  union { double d; uint64_t u; } dv;
  dv.d = x;
  uint64_t sign = dv.u >> 63;
  uint64_t mag = dv.u & 0x7fffffffffffffffull;
  if (mag >= 0x7ff0000000000000ull) {               // inf or nan
    if (mag > 0x7ff0000000000000ull) return (uint16_t)((sign << 15) | 0x7fc0);
    return (uint16_t)((sign << 15) | 0x7f80);
  }
  int e = (int)(mag >> 52);                          // biased exponent
  uint64_t frac = mag & 0xfffffffffffffull;
  // value = 1.frac * 2^(e-1023) (normal) ; doubles here are never subnormal in practice but
  // handle them as zero-exponent values below.
  int exp2v = (e == 0) ? -1022 : e - 1023;
  uint64_t sig = (e == 0) ? frac : (frac | (1ull << 52));   // 53-bit significand
  // target spacing exponent: normal bf16 keeps 8 bits -> ulp = 2^(exp2v-7); below 2^-126 the
  // spacing is 2^-133.
  int ulp_e = exp2v - 7;
  if (ulp_e < -133) ulp_e = -133;
  // sig * 2^(exp2v-52) / 2^ulp_e = sig >> (ulp_e - exp2v + 52)
  int sh = ulp_e - exp2v + 52;
  uint64_t q, rem, half;
  if (sh >= 64) {
    return (uint16_t)(sign << 15);                   // far below half the smallest spacing
  } else if (sh <= 0) {
    q = sig << (-sh); rem = 0; half = 1;
  } else {
    q = sig >> sh;
    rem = sig & ((1ull << sh) - 1);
    half = 1ull << (sh - 1);
  }
  if (rem > half || (rem == half && (q & 1))) q += 1;
  // q is the integer multiple of 2^ulp_e; rebuild the bf16 bits
  if (q == 0) return (uint16_t)(sign << 15);
  // normalise: find the exponent of q * 2^ulp_e
  int msb = 63 - __builtin_clzll(q);
  int vexp = ulp_e + msb;                            // value in [2^vexp, 2^(vexp+1))
  uint16_t bits;
  if (vexp < -126) {
    // subnormal bf16: mantissa = q (spacing 2^-133), exponent field 0
    bits = (uint16_t)(q & 0x7f);
  } else {
    if (vexp > 127) return (uint16_t)((sign << 15) | 0x7f80);
    uint64_t mant = (msb >= 7) ? (q >> (msb - 7)) : (q << (7 - msb));
    bits = (uint16_t)(((uint64_t)(vexp + 127) << 7) | (mant & 0x7f));
  }
  return (uint16_t)((sign << 15) | bits);
}

__host__ __device__ inline double bf16_to_f64(uint16_t b) {
  union { float f; uint32_t u; } v;
  v.u = ((uint32_t)b) << 16;
  return (double)v.f;
}

}  // namespace elmfb
