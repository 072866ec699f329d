// Host runtime behind the C ABI: descriptor checks, decomposition planner (subdomain boxes on
// the grid, covering ranges, tiles, chunks, overlapping pairs), device memory, assembly,
// block-sparse products, copies and evaluation.  The solvers live in solve.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "handle.h"

// Geometry decisions (grid coordinates, centres, support membership) must reproduce the same
// doubles on every implementation: no contraction of a*b+c into fused multiply-adds here.
#pragma clang fp contract(off)

static thread_local std::string g_thread_error;

namespace elmfb {

elmfb_status fail(elmfb_problem h, elmfb_status code, const std::string& msg) {
  if (h) h->err = msg;
  g_thread_error = msg;
  return code;
}

hipError_t dalloc_bytes(elmfb_problem h, void** p, int64_t bytes) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, (size_t)(bytes > 0 ? bytes : 16));
  if (e != hipSuccess) return e;
  h->allocs.push_back(q);
  *p = q;
  return hipSuccess;
}

void dfree(elmfb_problem h, void* p) {
  if (!p) return;
  for (auto it = h->allocs.begin(); it != h->allocs.end(); ++it)
    if (*it == p) {
      hipFree(p);
      h->allocs.erase(it);
      return;
    }
}

}  // namespace elmfb

namespace {

double grid_x(double lo, double hi, int n, int m) {
  if (n == 1) return lo;
  if (m == n - 1) return hi;
  const double step = (hi - lo) / (double)(n - 1);
  const double t = (double)m * step;
  return t + lo;
}

double centre_x(double lo, double hi, int J, int j) {
  if (J == 1) return 0.5 * (lo + hi);
  const double h = (hi - lo) / (double)(J - 1);
  const double t = (double)j * h;
  return t + lo;
}

std::string validate_impl(const elmfb_problem_desc* d) {
  if (!d) return "descriptor is NULL";
  if (d->abi_version != ELMFB_ABI_VERSION) return "abi_version mismatch";
  if (d->dim != 1 && d->dim != 2) return "dim must be 1 or 2";
  if (d->op == ELMFB_OP_D1 && d->dim != 1) return "ELMFB_OP_D1 needs dim = 1";
  if (d->op == ELMFB_OP_NEG_LAPLACE && d->dim != 2) return "ELMFB_OP_NEG_LAPLACE needs dim = 2";
  if (d->op == ELMFB_OP_OSCILLATOR && d->dim != 1) return "ELMFB_OP_OSCILLATOR needs dim = 1";
  if (d->op == ELMFB_OP_HELMHOLTZ && d->dim != 2) return "ELMFB_OP_HELMHOLTZ needs dim = 2";
  if (d->op != ELMFB_OP_D1 && d->op != ELMFB_OP_NEG_LAPLACE && d->op != ELMFB_OP_IDENTITY &&
      d->op != ELMFB_OP_OSCILLATOR && d->op != ELMFB_OP_HELMHOLTZ)
    return "unknown operator";
  if (d->op == ELMFB_OP_HELMHOLTZ && !std::isfinite(d->op_coef[0]))
    return "op_coef[0] (k^2) must be finite";
  if (d->domain != ELMFB_DOMAIN_BOX && d->domain != ELMFB_DOMAIN_L) return "unknown domain";
  if (d->domain == ELMFB_DOMAIN_L && d->dim != 2) return "ELMFB_DOMAIN_L needs dim = 2";
  if (d->n_bc_pts < 0 || d->n_bc_pts > ELMFB_MAX_BC_PTS) return "n_bc_pts out of range";
  if (d->n_bc_pts > 0) {
    if (d->dim != 2) return "Dirichlet rows at points need dim = 2";
    if (d->n_bc > 0) return "n_bc and n_bc_pts cannot both be set";
    if (!d->bc_pts_host || !d->bc_pts_val_host) return "bc_pts_host and bc_pts_val_host are required";
    if (!(std::isfinite(d->bc_pts_weight) && d->bc_pts_weight > 0.0))
      return "bc_pts_weight must be finite and > 0";
    for (int i = 0; i < d->n_bc_pts; ++i) {
      for (int a = 0; a < 2; ++a) {
        const double x = d->bc_pts_host[2 * i + a];
        if (!(std::isfinite(x) && x >= d->lo[a] && x <= d->hi[a]))
          return "bc_pts must lie in the box";
      }
      if (!std::isfinite(d->bc_pts_val_host[i])) return "bc_pts_val must be finite";
    }
  }
  if (d->op == ELMFB_OP_OSCILLATOR &&
      !(std::isfinite(d->op_coef[0]) && std::isfinite(d->op_coef[1]) &&
        std::isfinite(d->op_coef[2])))
    return "op_coef must be finite";
  if (d->n_bc < 0 || d->n_bc > ELMFB_MAX_BC) return "n_bc out of range";
  if (d->n_bc > 0 && d->dim != 1) return "soft-constraint rows need dim = 1";
  for (int i = 0; i < d->n_bc; ++i) {
    if (d->bc_order[i] != 0 && d->bc_order[i] != 1) return "bc_order must be 0 or 1";
    if (!(std::isfinite(d->bc_x[i]) && d->bc_x[i] >= d->lo[0] && d->bc_x[i] <= d->hi[0]))
      return "bc_x must lie in [lo, hi]";
    if (!(std::isfinite(d->bc_weight[i]) && d->bc_weight[i] > 0.0))
      return "bc_weight must be finite and > 0";
    if (!std::isfinite(d->bc_value[i])) return "bc_value must be finite";
  }
  if (d->ansatz != ELMFB_ANSATZ_NONE && d->ansatz != ELMFB_ANSATZ_TANH_ORIGIN &&
      d->ansatz != ELMFB_ANSATZ_TANH_BOX)
    return "unknown ansatz";
  if (d->ansatz == ELMFB_ANSATZ_TANH_ORIGIN && d->dim != 1) return "TANH_ORIGIN needs dim = 1";
  if (!std::isfinite(d->ansatz_omega)) return "ansatz_omega must be finite";
  for (int a = 0; a < d->dim; ++a) {
    if (!(std::isfinite(d->lo[a]) && std::isfinite(d->hi[a]) && d->lo[a] < d->hi[a]))
      return "domain bounds must be finite with lo < hi";
    if (d->n_points[a] < 2) return "n_points must be >= 2 on every axis";
  }
  if (d->n_levels < 1 || d->n_levels > ELMFB_MAX_LEVELS) return "n_levels out of range";
  if (!(std::isfinite(d->delta) && d->delta > 1.0 && d->delta < 7.0))
    return "delta must satisfy 1 < delta < 7";
  if (d->K < 1 || d->K > 256) return "K must be in 1..256";
  for (int l = 0; l < d->n_levels; ++l)
    for (int a = 0; a < d->dim; ++a)
      if (d->J[l][a] < 1 || d->J[l][a] > 4096) return "J out of range";
  if (d->store_prec != ELMFB_FP64 && d->store_prec != ELMFB_FP32 && d->store_prec != ELMFB_BF16 &&
      d->store_prec != ELMFB_FP16)
    return "unknown store precision";
  if (d->input_norm != ELMFB_INPUT_LOCAL && d->input_norm != ELMFB_INPUT_GLOBAL)
    return "unknown input_norm";
  if (!d->W_host != !d->b_host) return "W_host and b_host must both be given or both be NULL";
  if (!d->W_host) {
    for (int i = 0; i < 2; ++i)
      if (!(std::isfinite(d->w_range[i]) && std::isfinite(d->b_range[i])))
        return "w_range and b_range must be finite";
    if (d->w_range[0] > d->w_range[1] || d->b_range[0] > d->b_range[1])
      return "w_range and b_range must have lo <= hi";
  }
  return "";
}

// ---- counter-based draws of the random-feature parameters (SplitMix64, Steele, Lea and
// Flood 2014, in counter mode): value c of stream `seed` is the generator's finaliser of
// seed + (c + 1) gamma (mod 2^64); U(c) = lo + (hi - lo) u with u the top 53 bits times 2^-53,
// each operation rounded on its own.
#pragma STDC FP_CONTRACT OFF
uint64_t splitmix_at(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

double uniform_at(uint64_t seed, uint64_t c, double lo, double hi) {
  const double u = (double)(splitmix_at(seed, c) >> 11) * 0x1p-53;
  const double span = hi - lo;
  const double t = span * u;
  return lo + t;
}

int64_t full_params(const elmfb_problem_desc& d) {
  int64_t n = 0;
  for (int l = 0; l < d.n_levels; ++l) {
    int64_t s = 1;
    for (int a = 0; a < d.dim; ++a) s *= d.J[l][a];
    n += s;
  }
  return n * d.K;
}

// W [n][dim], b [n] for parameter q at counters 4q + a and 4q + 3
void draw_params(const elmfb_problem_desc& d, double* W, double* b) {
  const int64_t n = full_params(d);
  for (int64_t q = 0; q < n; ++q) {
    for (int a = 0; a < d.dim; ++a)
      W[q * d.dim + a] = uniform_at(d.seed, 4 * (uint64_t)q + (uint64_t)a, d.w_range[0], d.w_range[1]);
    b[q] = uniform_at(d.seed, 4 * (uint64_t)q + 3, d.b_range[0], d.b_range[1]);
  }
}

// Build every host table of the decomposition.
std::string plan_impl(elmfb_problem h) {
  const elmfb_problem_desc& d = h->desc;
  Geo& g = h->geo;
  std::memset(&g, 0, sizeof(g));
  g.dim = d.dim;
  g.nx = d.n_points[0];
  g.ny = d.dim == 2 ? d.n_points[1] : 1;
  g.n_levels = d.n_levels;
  g.K = d.K;
  g.n_bc = d.n_bc + d.n_bc_pts;
  g.domain = d.domain;
  g.bc_w = d.n_bc_pts > 0 ? d.bc_pts_weight : 0.0;
  for (int i = 0; i < 3; ++i) g.op_coef[i] = d.op_coef[i];
  h->bcs.n = d.n_bc;
  for (int i = 0; i < d.n_bc; ++i) {
    h->bcs.order[i] = d.bc_order[i];
    h->bcs.x[i] = d.bc_x[i];
    h->bcs.w[i] = d.bc_weight[i];
    h->bcs.val[i] = d.bc_value[i];
  }
  g.op = d.op;
  g.ansatz = d.ansatz;
  g.input_norm = d.input_norm;
  g.ansatz_omega = d.ansatz_omega;
  const int npts[2] = {g.nx, g.ny};
  double lo[2] = {d.lo[0], d.dim == 2 ? d.lo[1] : 0.0};
  double hi[2] = {d.hi[0], d.dim == 2 ? d.hi[1] : 1.0};
  for (int a = 0; a < 2; ++a) {
    g.lo[a] = lo[a];
    g.hi[a] = hi[a];
    g.step[a] = npts[a] > 1 ? (hi[a] - lo[a]) / (double)(npts[a] - 1) : 0.0;
  }
  g.n_rows = (int64_t)g.nx * g.ny;
  std::vector<double> xs[2];
  for (int a = 0; a < 2; ++a) {
    xs[a].resize(npts[a]);
    for (int m = 0; m < npts[a]; ++m) xs[a][m] = grid_x(lo[a], hi[a], npts[a], m);
  }
  // L-shaped domain: grid points with x > mid_x and y > mid_y are not collocation points
  const bool lshape = d.domain == ELMFB_DOMAIN_L;
  for (int a = 0; a < 2; ++a) g.lmid[a] = 0.5 * (lo[a] + hi[a]);
  g.n_int = g.n_rows;
  if (lshape) {
    int64_t cx = 0, cy = 0;
    for (int m = 0; m < npts[0]; ++m) cx += xs[0][m] > g.lmid[0];
    for (int m = 0; m < npts[1]; ++m) cy += xs[1][m] > g.lmid[1];
    g.n_int = g.n_rows - cx * cy;
  }
  const double sqn = std::sqrt((double)g.n_int);
  g.inv_scale = 1.0 / (sqn * (double)d.n_levels);
  g.inv_sqrt_n = 1.0 / sqn;
  g.inv_levels = 1.0 / (double)d.n_levels;

  // per level, per axis: centres, half-width, per-subdomain ranges, per-point cover ranges
  std::vector<int> m0s[kMaxLevels][2], m1s[kMaxLevels][2];
  h->cov.clear();
  int nb = 0;
  for (int l = 0; l < d.n_levels; ++l) {
    g.bbase[l] = nb;
    for (int a = 0; a < 2; ++a) {
      const int J = (a < d.dim) ? d.J[l][a] : 1;
      g.J[l][a] = J;
      const int n = npts[a];
      m0s[l][a].assign(J, 0);
      m1s[l][a].assign(J, 0);
      if (J == 1) {
        g.mid[l][a] = 0.5 * (lo[a] + hi[a]);
        g.sigma[l][a] = 0.5 * (hi[a] - lo[a]);
        g.cen_h[l][a] = 0.0;
        m0s[l][a][0] = 0;
        m1s[l][a][0] = n;
      } else {
        const double hc = (hi[a] - lo[a]) / (double)(J - 1);
        g.cen_h[l][a] = hc;
        const double prod = d.delta * hc;
        g.sigma[l][a] = prod / 2.0;
        const double sigma = g.sigma[l][a];
        for (int j = 0; j < J; ++j) {
          const double mu = centre_x(lo[a], hi[a], J, j);
          int first = -1, last = -2;
          for (int m = 0; m < n; ++m) {
            if (std::fabs(xs[a][m] - mu) < sigma) {
              if (first < 0) first = m;
              if (last >= 0 && last != m - 1) return "non-contiguous support";
              last = m;
            }
          }
          if (first < 0) { m0s[l][a][j] = 0; m1s[l][a][j] = 0; }
          else { m0s[l][a][j] = first; m1s[l][a][j] = last + 1; }
        }
      }
      // cover ranges per grid index
      g.cov_off[l][a] = (int32_t)h->cov.size();
      for (int m = 0; m < n; ++m) {
        int jlo = -1, jhi = -2;
        for (int j = 0; j < J; ++j) {
          if (m >= m0s[l][a][j] && m < m1s[l][a][j]) {
            if (jlo < 0) jlo = j;
            if (jhi >= 0 && jhi != j - 1) return "non-contiguous cover";
            jhi = j;
          }
        }
        if (jlo < 0) { jlo = 0; jhi = -1; }
        h->cov.push_back(jlo);
        h->cov.push_back(jhi);
      }
    }
    nb += g.J[l][0] * g.J[l][1];
  }
  // kept subdomains: all of them on a box; on an L-shaped domain those whose centre is not in
  // the removed quarter.  bmap[bmap_off[l] + jx*Jy + jy] = block index or -1; pidx = index of
  // the block among all subdomains of the full grids (its parameters in W_host, b_host).
  h->bmap.clear();
  h->block_pidx.clear();
  int nkept = 0, nfull = 0;
  for (int l = 0; l < d.n_levels; ++l) {
    g.bmap_off[l] = (int32_t)h->bmap.size();
    g.bbase[l] = nkept;
    for (int jx = 0; jx < g.J[l][0]; ++jx)
      for (int jy = 0; jy < g.J[l][1]; ++jy, ++nfull) {
        const bool drop = lshape && centre_x(lo[0], hi[0], g.J[l][0], jx) > g.lmid[0] &&
                          centre_x(lo[1], hi[1], g.J[l][1], jy) > g.lmid[1];
        h->bmap.push_back(drop ? -1 : nkept);
        if (!drop) {
          h->block_pidx.push_back(nfull);
          ++nkept;
        }
      }
  }
  h->n_sub_full = nfull;
  g.n_blocks = nkept;
  g.n_phi = (int64_t)nkept * d.K;
  // per-axis window sums of an L-shaped domain: 6 doubles per (level, axis, grid index)
  int32_t nls = 0;
  for (int l = 0; l < d.n_levels; ++l)
    for (int a = 0; a < 2; ++a) {
      g.lsum_off[l][a] = nls;
      if (lshape) nls += npts[a];
    }
  h->n_lsum = nls;

  // axis segments and the envelope table layout
  h->segs.clear();
  std::vector<int> segoff[kMaxLevels][2];
  int32_t tab = 0;
  for (int l = 0; l < d.n_levels; ++l)
    for (int a = 0; a < 2; ++a) {
      segoff[l][a].assign(g.J[l][a], 0);
      for (int j = 0; j < g.J[l][a]; ++j) {
        AxisSeg s{l, a, j, m0s[l][a][j], m1s[l][a][j], tab};
        segoff[l][a][j] = tab;
        tab += m1s[l][a][j] - m0s[l][a][j];
        h->segs.push_back(s);
      }
    }
  h->n_tab = tab;

  // blocks, tiles, chunks
  h->blocks.clear();
  h->tiles.clear();
  h->chunks.clear();
  h->chunk_start.clear();
  int64_t a_off = 0, p_off = 0, nnz = 0;
  for (int l = 0; l < d.n_levels; ++l)
    for (int jx = 0; jx < g.J[l][0]; ++jx)
      for (int jy = 0; jy < g.J[l][1]; ++jy) {
        if (h->bmap[g.bmap_off[l] + jx * g.J[l][1] + jy] < 0) continue;
        DevBlock B{};
        B.jx = jx;
        B.jy = jy;
        B.a_off = a_off;
        B.p_off = p_off;
        B.q0 = (int32_t)(h->blocks.size() * (size_t)d.K);
        B.ix0 = m0s[l][0][jx];
        B.nx = m1s[l][0][jx] - m0s[l][0][jx];
        B.iy0 = m0s[l][1][jy];
        B.ny = m1s[l][1][jy] - m0s[l][1][jy];
        const int64_t n = (int64_t)B.nx * B.ny;
        if (n > (int64_t)1 << 30) return "block too large";
        B.n = (int32_t)n;
        B.ld = (int32_t)((n + kRowAlign - 1) / kRowAlign * kRowAlign);
        B.tabx = segoff[l][0][jx];
        B.taby = segoff[l][1][jy];
        B.level = l;
        B.nk = d.K;
        const int b = (int)h->blocks.size();
        for (int64_t p0 = 0; p0 < n; p0 += kTile) h->tiles.push_back(Tile{b, (int32_t)p0});
        h->chunk_start.push_back((int32_t)h->chunks.size());
        for (int64_t p0 = 0; p0 < n; p0 += kChunkPts) h->chunks.push_back(Tile{b, (int32_t)p0});
        h->blocks.push_back(B);
        a_off += (int64_t)B.ld * d.K;
        nnz += n * d.K;
        p_off += n;
      }
  h->chunk_start.push_back((int32_t)h->chunks.size());
  h->nnz = nnz;
  h->n_store = a_off;
  h->n_block_points = p_off;

  // overlapping pairs (i <= j) over all levels: on level l the subdomains meeting a box are the
  // covering ranges of its first and last grid index (covering ranges are monotone)
  h->pairs_all.clear();
  h->diag_pair.assign(h->blocks.size(), -1);
  for (size_t i = 0; i < h->blocks.size(); ++i) {
    const DevBlock& Bi = h->blocks[i];
    if (Bi.n == 0) continue;
    const int ix1 = Bi.ix0 + Bi.nx, iy1 = Bi.iy0 + Bi.ny;
    for (int l = Bi.level; l < d.n_levels; ++l) {
      const int jx0 = h->cov[g.cov_off[l][0] + 2 * Bi.ix0];
      const int jx1 = h->cov[g.cov_off[l][0] + 2 * (ix1 - 1) + 1];
      const int jy0 = h->cov[g.cov_off[l][1] + 2 * Bi.iy0];
      const int jy1 = h->cov[g.cov_off[l][1] + 2 * (iy1 - 1) + 1];
      for (int jx = jx0; jx <= jx1; ++jx)
        for (int jy = jy0; jy <= jy1; ++jy) {
          const int j = h->bmap[g.bmap_off[l] + jx * g.J[l][1] + jy];
          if (j < (int)i) continue;   // discarded (-1) or already paired
          const DevBlock& Bj = h->blocks[j];
          if (Bj.n == 0) continue;
          const int ox0 = std::max(Bi.ix0, Bj.ix0), ox1 = std::min(ix1, Bj.ix0 + Bj.nx);
          const int oy0 = std::max(Bi.iy0, Bj.iy0), oy1 = std::min(iy1, Bj.iy0 + Bj.ny);
          if (ox1 <= ox0 || oy1 <= oy0) continue;
          GramPair pr{};
          pr.bi = (int32_t)i;
          pr.bj = j;
          pr.ix0 = ox0;
          pr.nx = ox1 - ox0;
          pr.iy0 = oy0;
          pr.ny = oy1 - oy0;
          if (j == (int)i) h->diag_pair[i] = (int64_t)h->pairs_all.size();
          h->pairs_all.push_back(pr);
        }
    }
  }
  return "";
}

int64_t footprint(elmfb_problem h) {
  const Geo& g = h->geo;
  int64_t b = 0;
  auto add = [&](int64_t n) { b += (n + 255) / 256 * 256; };
  add(h->n_store * 8);                                    // FP64 matrix
  if (h->lo_prec != ELMFB_FP64) add(h->n_store * elem_size(h->lo_prec));   // low-precision copy
  add(h->n_block_points * 8);                             // tpart
  add((int64_t)h->chunks.size() * g.K * 8);               // part
  add(4 * 2 * kRedBlocks * 8);                            // reductions
  add(4 * (g.n_rows + g.n_bc) * 8);                       // h, u, t, r
  add((int64_t)g.n_bc * g.n_phi * 8);                     // soft-constraint rows
  add((int64_t)g.n_bc * 3 * 8);                           // their points and values
  add((int64_t)h->bmap.size() * 4);                       // block map
  add(h->n_lsum * 6 * 8);                                 // per-axis window sums (L domain)
  add(7 * g.n_phi * 8);                                   // v, w, x, vt, xt, c
  add(g.n_phi * 2 * 8 + g.n_phi * 8);                     // W, b
  add(h->n_tab * 3 * 8);
  add((int64_t)h->blocks.size() * sizeof(DevBlock));
  add((int64_t)(h->tiles.size() + h->chunks.size()) * sizeof(Tile));
  add((int64_t)(h->chunk_start.size() + h->cov.size()) * 4);
  add((int64_t)h->segs.size() * sizeof(AxisSeg));
  add(sizeof(SolveState) + 64);
  add(64);                                                // flag
  add((int64_t)kHistCap * 2 * 8);                         // bidiagonal of the last LSQR run
  return b;
}

void release(elmfb_problem h) {
  for (auto& kv : h->graphs) hipGraphExecDestroy(kv.second);
  h->graphs.clear();
  for (void* p : h->allocs) hipFree(p);
  h->allocs.clear();
  if (h->ev_in) hipEventDestroy(h->ev_in);
  if (h->ev_out) hipEventDestroy(h->ev_out);
  if (h->stream) hipStreamDestroy(h->stream);
  h->ev_in = h->ev_out = nullptr;
  h->stream = nullptr;
}

}  // namespace

namespace elmfb {
std::string validate_desc(const elmfb_problem_desc* d) { return validate_impl(d); }
std::string plan_problem(elmfb_problem h) { return plan_impl(h); }
int64_t feature_param_count(const elmfb_problem_desc& d) { return full_params(d); }
void draw_feature_params(const elmfb_problem_desc& d, double* W, double* b) {
  draw_params(d, W, b);
}
}  // namespace elmfb

extern "C" {

elmfb_status elmfb_draw_features(const elmfb_problem_desc* desc, double* W_host, double* b_host) {
  if (!desc || !W_host || !b_host) return fail(nullptr, ELMFB_E_INVALID, "NULL argument");
  if (desc->dim != 1 && desc->dim != 2) return fail(nullptr, ELMFB_E_INVALID, "dim must be 1 or 2");
  if (desc->n_levels < 1 || desc->n_levels > ELMFB_MAX_LEVELS || desc->K < 1 || desc->K > 256)
    return fail(nullptr, ELMFB_E_INVALID, "bad levels or K");
  for (int l = 0; l < desc->n_levels; ++l)
    for (int a = 0; a < desc->dim; ++a)
      if (desc->J[l][a] < 1 || desc->J[l][a] > 4096) return fail(nullptr, ELMFB_E_INVALID, "J out of range");
  for (int i = 0; i < 2; ++i)
    if (!(std::isfinite(desc->w_range[i]) && std::isfinite(desc->b_range[i])))
      return fail(nullptr, ELMFB_E_INVALID, "w_range and b_range must be finite");
  if (desc->w_range[0] > desc->w_range[1] || desc->b_range[0] > desc->b_range[1])
    return fail(nullptr, ELMFB_E_INVALID, "w_range and b_range must have lo <= hi");
  draw_params(*desc, W_host, b_host);
  return ELMFB_OK;
}

elmfb_status elmfb_define_problem(const elmfb_problem_desc* desc_in, elmfb_problem* out) {
  if (!out) return fail(nullptr, ELMFB_E_INVALID, "out is NULL");
  *out = nullptr;
  const std::string v = validate_impl(desc_in);
  if (!v.empty()) return fail(nullptr, ELMFB_E_INVALID, v);
  // parameters drawn by the library when the caller passes none
  elmfb_problem_desc dd = *desc_in;
  std::vector<double> Wd, bd;
  if (!dd.W_host) {
    const int64_t np = full_params(dd);
    Wd.resize((size_t)(np * dd.dim));
    bd.resize((size_t)np);
    draw_params(dd, Wd.data(), bd.data());
    dd.W_host = Wd.data();
    dd.b_host = bd.data();
  }
  const elmfb_problem_desc* desc = &dd;
  elmfb_problem h = new (std::nothrow) elmfb_problem_s();
  if (!h) return fail(nullptr, ELMFB_E_NOMEM, "host allocation failed");
  h->desc = *desc;
  h->lo_prec = desc->store_prec;
  const std::string pe = plan_impl(h);
  if (!pe.empty()) {
    delete h;
    return fail(nullptr, ELMFB_E_INVALID, pe);
  }
  h->bytes_device = footprint(h);
  if (const char* cap = std::getenv("ELMFB_MEM_CAP")) {
    const long long c = std::atoll(cap);
    if (c > 0) h->mem_cap = c;
    if (c > 0 && h->bytes_device > c) {
      const std::string m = "device footprint " + std::to_string(h->bytes_device) +
                            " B exceeds ELMFB_MEM_CAP";
      delete h;
      return fail(nullptr, ELMFB_E_NOMEM, m);
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    delete h;
    return fail(nullptr, ELMFB_E_DEVICE, "no HIP device available");
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete h;
    return fail(nullptr, ELMFB_E_DEVICE, "cannot query the HIP device");
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    const std::string m = std::string("device is ") + prop.gcnArchName + ", need gfx950";
    delete h;
    return fail(nullptr, ELMFB_E_DEVICE, m);
  }
  if (hipError_t e = noalloc_init_device(); e != hipSuccess) {
    delete h;
    return fail(nullptr, ELMFB_E_DEVICE, std::string("scratch array address: ") +
                                             hipGetErrorString(e));
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && (size_t)h->bytes_device > free_b) {
    const std::string m = "device footprint " + std::to_string(h->bytes_device) +
                          " B exceeds free memory " + std::to_string(free_b) + " B";
    delete h;
    return fail(nullptr, ELMFB_E_NOMEM, m);
  }

  const Geo& g = h->geo;
#define ALLOC(p, bytes)                                                     \
  do {                                                                      \
    hipError_t e_ = dalloc(h, &(p), (bytes));                               \
    if (e_ != hipSuccess) {                                                 \
      release(h);                                                           \
      delete h;                                                             \
      return fail(nullptr, ELMFB_E_NOMEM, std::string("hipMalloc: ") +     \
                                              hipGetErrorString(e_));      \
    }                                                                       \
  } while (0)
  ALLOC(h->d_A, h->n_store * 8);
  if (h->lo_prec != ELMFB_FP64) ALLOC(h->d_A_lo, h->n_store * elem_size(h->lo_prec));
  ALLOC(h->d_tpart, h->n_block_points * 8);
  ALLOC(h->d_part, (int64_t)h->chunks.size() * g.K * 8);
  ALLOC(h->d_red, 4 * 2 * kRedBlocks * 8);
  ALLOC(h->d_h, (g.n_rows + g.n_bc) * 8);
  ALLOC(h->d_u, (g.n_rows + g.n_bc) * 8);
  ALLOC(h->d_t, (g.n_rows + g.n_bc) * 8);
  if (g.n_bc > 0) ALLOC(h->d_bc, (int64_t)g.n_bc * g.n_phi * 8);
  if (desc->n_bc_pts > 0) ALLOC(h->d_bcpts, (int64_t)desc->n_bc_pts * 3 * 8);
  ALLOC(h->d_bmap, (int64_t)h->bmap.size() * 4);
  if (h->n_lsum > 0) ALLOC(h->d_lsum, h->n_lsum * 6 * 8);
  h->geo.bmap = h->d_bmap;
  h->geo.lsum = h->d_lsum;
  h->geo.bcpts = h->d_bcpts;
  ALLOC(h->d_v, g.n_phi * 8);
  ALLOC(h->d_w, g.n_phi * 8);
  ALLOC(h->d_x, g.n_phi * 8);
  ALLOC(h->d_vt, g.n_phi * 8);
  ALLOC(h->d_xt, g.n_phi * 8);
  ALLOC(h->d_c, g.n_phi * 8);
  ALLOC(h->d_r, (g.n_rows + g.n_bc) * 8);
  ALLOC(h->d_W, g.n_phi * 2 * 8);
  ALLOC(h->d_b, g.n_phi * 8);
  ALLOC(h->d_tab, h->n_tab * 3 * 8);
  ALLOC(h->d_blocks, (int64_t)h->blocks.size() * sizeof(DevBlock));
  ALLOC(h->d_tiles, (int64_t)h->tiles.size() * sizeof(Tile));
  ALLOC(h->d_chunks, (int64_t)h->chunks.size() * sizeof(Tile));
  ALLOC(h->d_cstart, (int64_t)h->chunk_start.size() * 4);
  ALLOC(h->d_cov, (int64_t)h->cov.size() * 4);
  ALLOC(h->d_segs, (int64_t)h->segs.size() * sizeof(AxisSeg));
  ALLOC(h->d_state, sizeof(SolveState));
  ALLOC(h->d_scalar, 64);
  ALLOC(h->d_flag, 64);
  ALLOC(h->d_hist, (int64_t)kHistCap * 2 * 8);
#undef ALLOC

  // W padded to two columns; the parameters of kept block j are rows pidx_j K .. of W_host
  std::vector<double> W2((size_t)g.n_phi * 2, 0.0), b1((size_t)g.n_phi, 0.0);
  for (int j = 0; j < g.n_blocks; ++j)
    for (int k = 0; k < g.K; ++k) {
      const int64_t q = (int64_t)j * g.K + k;
      const int64_t src = (int64_t)h->block_pidx[j] * g.K + k;
      for (int a = 0; a < desc->dim; ++a) W2[2 * q + a] = desc->W_host[src * desc->dim + a];
      b1[q] = desc->b_host[src];
    }
  for (int64_t q = 0; q < (int64_t)h->n_sub_full * g.K * desc->dim; ++q)
    if (!std::isfinite(desc->W_host[q])) { elmfb_destroy(h); return fail(nullptr, ELMFB_E_NUMERIC, "W has non-finite values"); }
  for (int64_t q = 0; q < (int64_t)h->n_sub_full * g.K; ++q)
    if (!std::isfinite(desc->b_host[q])) { elmfb_destroy(h); return fail(nullptr, ELMFB_E_NUMERIC, "b has non-finite values"); }

#define H2D(dst, src, bytes)                                                          \
  do {                                                                                \
    hipError_t e_ = hipMemcpy((dst), (src), (size_t)(bytes), hipMemcpyHostToDevice);  \
    if (e_ != hipSuccess) {                                                           \
      elmfb_destroy(h);                                                               \
      return fail(nullptr, ELMFB_E_DEVICE, std::string("hipMemcpy: ") +              \
                                               hipGetErrorString(e_));               \
    }                                                                                 \
  } while (0)
  H2D(h->d_W, W2.data(), W2.size() * 8);
  H2D(h->d_b, b1.data(), g.n_phi * 8);
  H2D(h->d_bmap, h->bmap.data(), h->bmap.size() * 4);
  if (desc->n_bc_pts > 0) {
    // Dirichlet points [n][2] then their values [n]
    std::vector<double> bp((size_t)desc->n_bc_pts * 3);
    std::memcpy(bp.data(), desc->bc_pts_host, (size_t)desc->n_bc_pts * 2 * 8);
    std::memcpy(bp.data() + 2 * desc->n_bc_pts, desc->bc_pts_val_host, (size_t)desc->n_bc_pts * 8);
    H2D(h->d_bcpts, bp.data(), bp.size() * 8);
  }
  if (!h->blocks.empty()) H2D(h->d_blocks, h->blocks.data(), h->blocks.size() * sizeof(DevBlock));
  if (!h->tiles.empty()) H2D(h->d_tiles, h->tiles.data(), h->tiles.size() * sizeof(Tile));
  if (!h->chunks.empty()) H2D(h->d_chunks, h->chunks.data(), h->chunks.size() * sizeof(Tile));
  H2D(h->d_cstart, h->chunk_start.data(), h->chunk_start.size() * 4);
  if (!h->cov.empty()) H2D(h->d_cov, h->cov.data(), h->cov.size() * 4);
  if (!h->segs.empty()) H2D(h->d_segs, h->segs.data(), h->segs.size() * sizeof(AxisSeg));
#undef H2D
  // the row padding of the stored blocks is never assembled; the vector loads of the matrix
  // passes read it with zero weights, so it must hold finite values
  {
    hipError_t ez = hipMemset(h->d_A, 0, (size_t)h->n_store * 8);
    if (ez == hipSuccess && h->d_A_lo)
      ez = hipMemset(h->d_A_lo, 0, (size_t)(h->n_store * elem_size(h->lo_prec)));
    if (ez != hipSuccess) {
      elmfb_destroy(h);
      return fail(nullptr, ELMFB_E_DEVICE, std::string("hipMemset: ") + hipGetErrorString(ez));
    }
  }
  h->desc.W_host = nullptr;
  h->desc.b_host = nullptr;
  h->desc.bc_pts_host = nullptr;
  h->desc.bc_pts_val_host = nullptr;

  if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming) != hipSuccess) {
    elmfb_destroy(h);
    return fail(nullptr, ELMFB_E_DEVICE, "stream/event creation failed");
  }
  // envelope tables depend only on the geometry: build them once here
  hipError_t e = launch_axis_tables(g, h->d_segs, (int)h->segs.size(), h->d_cov, h->d_tab, h->stream);
  if (e == hipSuccess && h->n_lsum > 0) e = launch_axis_sums(g, h->d_cov, h->d_lsum, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    const std::string m = std::string("axis tables: ") + hipGetErrorString(e);
    elmfb_destroy(h);
    return fail(nullptr, ELMFB_E_DEVICE, m);
  }
  *out = h;
  return ELMFB_OK;
}

elmfb_status elmfb_query(elmfb_problem h, elmfb_sizes* out) {
  if (!h || !out) return fail(h, ELMFB_E_INVALID, "NULL argument");
  out->n_rows = h->geo.n_rows;
  out->n_phi = h->geo.n_phi;
  out->nnz = h->nnz;
  out->n_blocks = h->geo.n_blocks;
  out->n_block_points = h->n_block_points;
  out->bytes_device = h->bytes_device;
  out->n_pairs = (int64_t)h->pairs_all.size();
  out->n_bc = h->geo.n_bc;
  out->n_interior = h->geo.n_int;
  return ELMFB_OK;
}

elmfb_status elmfb_points(elmfb_problem h, double* xy_dev, void* stream) {
  if (!h || !xy_dev) return fail(h, ELMFB_E_INVALID, "NULL argument");
  HIP_OR_FAIL(h, launch_points(h->geo, xy_dev, (hipStream_t)stream));
  return ELMFB_OK;
}

elmfb_status elmfb_assemble(elmfb_problem h, const double* f_dev, int32_t n_rhs, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!h || !f_dev) return fail(h, ELMFB_E_INVALID, "NULL argument");
  if (n_rhs < 1 || n_rhs > 1024) return fail(h, ELMFB_E_INVALID, "n_rhs must be in 1..1024");
  hipStream_t s = (hipStream_t)stream;
  const Geo& g = h->geo;
  const int64_t nrt = g.n_rows + g.n_bc;
  if (n_rhs > 1 && (int64_t)n_rhs * nrt > h->hs_cap) {
    dfree(h, h->d_hs);
    h->d_hs = nullptr;
    h->hs_cap = 0;
    HIP_OR_FAIL(h, dalloc(h, &h->d_hs, (int64_t)n_rhs * nrt * 8));
    h->hs_cap = (int64_t)n_rhs * nrt;
  }
  h->bj_ready = false;   // factors and the folded matrix belong to the previous assembly
  h->folded64 = h->folded_lo = false;
  HIP_OR_FAIL(h, hipMemsetAsync(h->d_flag, 0, 4, s));
  HIP_OR_FAIL(h, launch_rhs(g, f_dev, h->d_h, h->d_flag, s));
  HIP_OR_FAIL(h, launch_assemble(g, h->lo_prec, h->d_blocks, h->d_tiles,
                                 (int64_t)h->tiles.size(), h->d_tab, h->d_W, h->d_b, h->d_A,
                                 h->d_A_lo, s));
  if (g.n_bc > 0 && g.dim == 1)
    HIP_OR_FAIL(h, launch_bc_assemble(g, h->bcs, h->d_blocks, h->d_W, h->d_b, h->d_bc, h->d_h,
                                      s));
  if (g.n_bc > 0 && g.dim == 2)
    HIP_OR_FAIL(h, launch_bc_assemble_pts(g, h->d_blocks, h->d_W, h->d_b, h->d_bc, h->d_h, s));
  if (n_rhs > 1) {
    // every right-hand side: its h_r = f_r/sqrt(N_I), then the constraint values of h (the same
    // for all of them); d_h keeps the first
    for (int r = 0; r < n_rhs; ++r) {
      double* dst = h->d_hs + (int64_t)r * nrt;
      if (r == 0) {
        HIP_OR_FAIL(h, hipMemcpyAsync(dst, h->d_h, (size_t)nrt * 8, hipMemcpyDeviceToDevice, s));
        continue;
      }
      HIP_OR_FAIL(h, launch_rhs(g, f_dev + (int64_t)r * g.n_rows, dst, h->d_flag, s));
      if (g.n_bc > 0)
        HIP_OR_FAIL(h, hipMemcpyAsync(dst + g.n_rows, h->d_h + g.n_rows, (size_t)g.n_bc * 8,
                                      hipMemcpyDeviceToDevice, s));
    }
  }
  int32_t bad = 0;
  HIP_OR_FAIL(h, hipMemcpyAsync(&bad, h->d_flag, 4, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(h, hipStreamSynchronize(s));
  h->n_rhs = n_rhs;
  h->ms_assemble =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (bad) {
    h->assembled = false;
    return fail(h, ELMFB_E_NUMERIC, "f holds non-finite values");
  }
  h->assembled = true;
  h->anorm_f = -1.0;
  h->bj_ready = false;
  h->gram_prec = -1;
  return ELMFB_OK;
}

elmfb_status elmfb_matvec(elmfb_problem h, const double* v_dev, double* y_dev, void* stream) {
  if (!h || !v_dev || !y_dev) return fail(h, ELMFB_E_INVALID, "NULL argument");
  if (!h->assembled) return fail(h, ELMFB_E_STATE, "matvec before assemble");
  hipStream_t s = (hipStream_t)stream;
  const Geo& g = h->geo;
  HIP_OR_FAIL(h, launch_mv_blocks(g, ELMFB_FP64, h->d_blocks, h->d_tiles, (int64_t)h->tiles.size(),
                                  h->d_A, v_dev, nullptr, h->d_tpart, nullptr, s));
  HIP_OR_FAIL(h, launch_gather_rows(g, h->d_blocks, h->d_cov, h->d_tpart, ROW_STORE, y_dev,
                                    nullptr, nullptr, h->d_red, rows_wg(g), s));
  if (g.n_bc > 0)
    HIP_OR_FAIL(h, launch_bc_rows(g, h->d_bc, v_dev, nullptr, ROW_STORE, y_dev, nullptr, nullptr,
                                  h->d_red + rows_wg(g), s));
  return ELMFB_OK;
}

elmfb_status elmfb_rmatvec(elmfb_problem h, const double* u_dev, double* x_dev, void* stream) {
  if (!h || !u_dev || !x_dev) return fail(h, ELMFB_E_INVALID, "NULL argument");
  if (!h->assembled) return fail(h, ELMFB_E_STATE, "rmatvec before assemble");
  hipStream_t s = (hipStream_t)stream;
  const Geo& g = h->geo;
  HIP_OR_FAIL(h, launch_rmv_chunks(g, ELMFB_FP64, h->d_blocks, h->d_chunks,
                                   (int64_t)h->chunks.size(), h->d_A, u_dev, nullptr, h->d_part,
                                   nullptr, s));
  HIP_OR_FAIL(h, launch_rmv_finish(g, h->d_cstart, h->d_part, COL_STORE, x_dev, nullptr,
                                   h->d_red, cols_wg(g), h->d_bc, u_dev, nullptr, s));
  return ELMFB_OK;
}

elmfb_status elmfb_copy_rhs(elmfb_problem h, double* h_dev, void* stream) {
  if (!h || !h_dev) return fail(h, ELMFB_E_INVALID, "NULL argument");
  if (!h->assembled) return fail(h, ELMFB_E_STATE, "copy_rhs before assemble");
  const int64_t nrt = h->geo.n_rows + h->geo.n_bc;
  if (h->n_rhs > 1)
    HIP_OR_FAIL(h, hipMemcpyAsync(h_dev, h->d_hs, (size_t)(h->n_rhs * nrt) * 8,
                                  hipMemcpyDeviceToDevice, (hipStream_t)stream));
  else
    HIP_OR_FAIL(h, hipMemcpyAsync(h_dev, h->d_h, (size_t)nrt * 8, hipMemcpyDeviceToDevice,
                                  (hipStream_t)stream));
  return ELMFB_OK;
}

elmfb_status elmfb_copy_bc(elmfb_problem h, double* dst_dev, void* stream) {
  if (!h || !dst_dev) return fail(h, ELMFB_E_INVALID, "NULL argument");
  if (!h->assembled) return fail(h, ELMFB_E_STATE, "copy_bc before assemble");
  if (h->geo.n_bc == 0) return ELMFB_OK;
  HIP_OR_FAIL(h, hipMemcpyAsync(dst_dev, h->d_bc, (size_t)h->geo.n_bc * h->geo.n_phi * 8,
                                hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return ELMFB_OK;
}

elmfb_status elmfb_copy_blocks(elmfb_problem h, int32_t prec, void* dst_dev, int64_t* table_host,
                               void* stream) {
  if (!h) return fail(h, ELMFB_E_INVALID, "NULL handle");
  if (table_host) {
    int64_t dense = 0;
    for (size_t b = 0; b < h->blocks.size(); ++b) {
      const DevBlock& B = h->blocks[b];
      int64_t* t = table_host + 8 * b;
      t[0] = B.level;
      t[1] = B.jx;
      t[2] = B.jy;
      t[3] = B.ix0;
      t[4] = B.nx;
      t[5] = B.iy0;
      t[6] = B.ny;
      t[7] = dense;
      dense += (int64_t)B.n * h->geo.K;
    }
  }
  if (dst_dev) {
    if (!h->assembled) return fail(h, ELMFB_E_STATE, "copy_blocks before assemble");
    const bool folded = (prec & ELMFB_COPY_FOLDED) != 0;
    prec &= ~ELMFB_COPY_FOLDED;
    const void* src = nullptr;
    if (folded) {
      if (prec == ELMFB_FP64 && h->bj_ready && h->folded64) src = h->d_Ahat;
      else if (prec == h->lo_prec && prec != ELMFB_FP64 && h->bj_ready && h->folded_lo)
        src = h->d_Ahat_lo;
      else return fail(h, ELMFB_E_STATE, "no folded copy in that precision");
    } else if (prec == ELMFB_FP64) {
      src = h->d_A;
    } else if (prec == h->lo_prec && h->d_A_lo) {
      src = h->d_A_lo;
    } else {
      return fail(h, ELMFB_E_STATE, "no stored copy in that precision");
    }
    // stored rows are padded to ld; the copy drops the padding
    const int64_t es = elem_size(prec);
    int64_t dense = 0;
    for (const DevBlock& B : h->blocks) {
      if (B.n == 0) continue;
      HIP_OR_FAIL(h, hipMemcpy2DAsync(static_cast<char*>(dst_dev) + dense * es, (size_t)(B.n * es),
                                      static_cast<const char*>(src) + B.a_off * es,
                                      (size_t)(B.ld * es), (size_t)(B.n * es), (size_t)h->geo.K,
                                      hipMemcpyDeviceToDevice, (hipStream_t)stream));
      dense += (int64_t)B.n * h->geo.K;
    }
  }
  return ELMFB_OK;
}


elmfb_status elmfb_evaluate(elmfb_problem h, const double* coef_dev, int32_t n_rhs,
                            const double* pts_dev, int64_t n_pts, double* u_dev, void* stream) {
  if (!h || n_pts < 0 || n_rhs < 1 || (n_pts > 0 && (!coef_dev || !pts_dev || !u_dev)))
    return fail(h, ELMFB_E_INVALID, "bad argument");
  for (int r = 0; r < n_rhs; ++r)
    HIP_OR_FAIL(h, launch_evaluate(h->geo, h->d_W, h->d_b, coef_dev + (int64_t)r * h->geo.n_phi,
                                   pts_dev, n_pts, u_dev + (int64_t)r * n_pts,
                                   (hipStream_t)stream));
  return ELMFB_OK;
}

elmfb_status elmfb_time_kernels(elmfb_problem h, int32_t prec, int32_t reps, double* ms_host,
                                void* stream) {
  if (!h || !ms_host || reps < 1) return fail(h, ELMFB_E_INVALID, "bad argument");
  if (!h->assembled) return fail(h, ELMFB_E_STATE, "time_kernels before assemble");
  const void* A = nullptr;
  if (prec == ELMFB_FP64) A = h->d_A;
  else if (prec == h->lo_prec && h->d_A_lo) A = h->d_A_lo;
  else return fail(h, ELMFB_E_STATE, "no stored copy in that precision");
  hipStream_t s = (hipStream_t)stream;
  const Geo& g = h->geo;
  // v = 1 (in d_x), u = 1 (in d_t)
  std::vector<double> ones((size_t)(g.n_rows > g.n_phi ? g.n_rows : g.n_phi), 1.0);
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_x, ones.data(), (size_t)g.n_phi * 8, hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_t, ones.data(), (size_t)g.n_rows * 8, hipMemcpyHostToDevice, s));
  // four timed groups: the two matrix-streaming passes, then the row gather that completes
  // y = M v and the column pass that completes x = M^T u (both with their norm partials, as in
  // an LSQR step)
  hipEvent_t ev[5];
  for (int i = 0; i < 5; ++i) HIP_OR_FAIL(h, hipEventCreate(&ev[i]));
  hipError_t e = hipEventRecord(ev[0], s);
  for (int i = 0; i < reps && e == hipSuccess; ++i)
    e = launch_mv_blocks(g, prec, h->d_blocks, h->d_tiles, (int64_t)h->tiles.size(), A, h->d_x,
                         nullptr, h->d_tpart, nullptr, s);
  if (e == hipSuccess) e = hipEventRecord(ev[1], s);
  for (int i = 0; i < reps && e == hipSuccess; ++i)
    e = launch_rmv_chunks(g, prec, h->d_blocks, h->d_chunks, (int64_t)h->chunks.size(), A,
                          h->d_t, nullptr, h->d_part, nullptr, s);
  if (e == hipSuccess) e = hipEventRecord(ev[2], s);
  for (int i = 0; i < reps && e == hipSuccess; ++i)
    e = launch_gather_rows(g, h->d_blocks, h->d_cov, h->d_tpart, ROW_STORE_SQ, h->d_r, nullptr,
                           nullptr, h->d_red, rows_wg(g), s);
  if (e == hipSuccess) e = hipEventRecord(ev[3], s);
  for (int i = 0; i < reps && e == hipSuccess; ++i)
    e = launch_rmv_finish(g, h->d_cstart, h->d_part, COL_STORE_SQ, h->d_xt, nullptr, h->d_red,
                          cols_wg(g), s);
  if (e == hipSuccess) e = hipEventRecord(ev[4], s);
  if (e == hipSuccess) e = hipEventSynchronize(ev[4]);
  float t[4] = {0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventElapsedTime(&t[i], ev[i], ev[i + 1]);
  for (int i = 0; i < 5; ++i) hipEventDestroy(ev[i]);
  HIP_OR_FAIL(h, e);
  for (int i = 0; i < 4; ++i) ms_host[i] = (double)t[i] / reps;
  return ELMFB_OK;
}

void elmfb_destroy(elmfb_problem h) {
  if (!h) return;
  if (h->stream) hipStreamSynchronize(h->stream);
  release(h);
  delete h;
}

const char* elmfb_last_error(elmfb_problem h) {
  if (h) return h->err.c_str();
  return g_thread_error.c_str();
}

}  // extern "C"
