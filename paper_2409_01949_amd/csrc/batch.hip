// Host runtime of batches: many independent problems, each with up to 8 right-hand sides, whose
// assembly and Krylov iterations run as single launches over the whole batch (k_batch.hip).
// Each instance is planned like a single problem (same geometry code), then the tables are
// concatenated with global offsets.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "handle.h"

static thread_local std::string g_batch_error;

struct elmfb_batch_s {
  int n = 0, R = 1, lo_prec = ELMFB_FP64;
  std::string err;
  std::vector<Geo> geos;
  std::vector<InstInfo> insts;
  std::vector<int64_t> nrows, nphis;
  std::vector<DevBlock> blocks;
  std::vector<Tile> tiles, ftiles;
  std::vector<int32_t> cov;
  std::vector<BSeg> segs;
  std::vector<RowTile> rtiles;
  std::vector<ColTile> ctiles;
  std::vector<int64_t> foff, goff;   // per block: packed-factor and square Gram offsets
  int64_t n_rows = 0, n_phi = 0, nnz = 0, n_bp = 0, n_tab = 0, n_fac = 0, n_gsq = 0, bytes = 0;
  int64_t n_store = 0;               // stored elements per matrix copy, row padding included
  int tp[4] = {32, 32, 32, 32};      // points per LDS stage of A^T U, per matrix precision
  int fa[4] = {8, 8, 8, 8};          // features loaded ahead per lane in A V, per precision
  int rpt = 1;                       // rows per thread of the row gather
  bool tuned[4] = {false, false, false, false};
  bool lo_unsafe = false;            // FP16 fold over an identity-fallback block: not used

  std::vector<void*> allocs;
  Geo* d_geos = nullptr;
  InstInfo* d_insts = nullptr;
  int64_t *d_nrows = nullptr, *d_nphis = nullptr;
  DevBlock* d_blocks = nullptr;
  Tile* d_tiles = nullptr;
  int32_t* d_cov = nullptr;
  BSeg* d_segs = nullptr;
  RowTile* d_rtiles = nullptr;
  ColTile* d_ctiles = nullptr;
  int64_t *d_foff = nullptr, *d_goff = nullptr;
  double *d_tab = nullptr, *d_W = nullptr, *d_b = nullptr, *d_A = nullptr;
  void* d_A_lo = nullptr;
  double *d_h = nullptr, *d_u = nullptr, *d_v = nullptr, *d_w = nullptr, *d_x = nullptr,
         *d_c = nullptr;
  double* d_tpart = nullptr;
  int64_t tpart_bp = 0;        // block points d_tpart holds (the subdomain or patch boxes)
  double *d_red_r = nullptr, *d_red_b = nullptr, *d_red_c = nullptr, *d_red_h = nullptr;
  double *d_x0 = nullptr, *d_h0 = nullptr;   // warm start and h - M x0 (allocated on first use)
  SolveState* d_state = nullptr;
  BtOuter* d_outer = nullptr;
  int32_t *d_flag = nullptr, *d_count = nullptr;
  double* d_rc = nullptr;      // block-Jacobi inverse factors R_b^{-1} (column-packed)
  double* d_Ahat = nullptr;    // preconditioned matrix M_b R_b^{-1} (FP64)
  Tile* d_ftiles = nullptr;    // 64-point runs of the blocks (forming M R^{-1})
  std::vector<ColSlice> slices;    // one per subdomain block (the M^T U pass)
  std::vector<GramTask> tasks;     // one per subdomain block (the diagonal Gram blocks)
  ColSlice* d_slices = nullptr;
  GramTask* d_tasks = nullptr;
  int kmax = 1;                    // largest K

  // Patches of the block-Jacobi preconditioner: P^d neighbouring subdomains of a level as one
  // block (patch > 1).  Their tables are planned for one P at a time (patch_planned); the folded
  // matrix M R^{-1} of the patches, FP64 and store_prec, lives in their own block layout, and y
  // (the coefficients of M R^{-1}) in the patch column order: column q of that order is column
  // pperm[q] of x.
  int patch = 1;                   // P of the factors held
  int patch_planned = 0;
  std::vector<Geo> pgeos;
  std::vector<InstInfo> pinsts;
  std::vector<DevBlock> pblocks;
  std::vector<int32_t> pcov, pmem, pmoff, pperm;
  std::vector<ColSlice> pslices;
  std::vector<Tile> pftiles, pruns, pmvruns;
  std::vector<GramTask> ptasks;
  std::vector<int64_t> pfoff, pgoff;
  std::vector<int64_t> pchunk_blk, pchunk_task;   // factor chunks: first block and first task
  int pkmax = 1;
  int64_t pn_store = 0, pn_bp = 0, pn_fac = 0, pn_scratch = 0, pn_dense = 0;
  Geo* d_pgeos = nullptr;
  InstInfo* d_pinsts = nullptr;
  DevBlock* d_pblocks = nullptr;
  int32_t *d_pcov = nullptr, *d_pmem = nullptr, *d_pmoff = nullptr, *d_pperm = nullptr;
  ColSlice* d_pslices = nullptr;
  Tile *d_pftiles = nullptr, *d_pruns = nullptr, *d_pmvruns = nullptr;
  GramTask* d_ptasks = nullptr;
  int64_t *d_pfoff = nullptr, *d_pgoff = nullptr;
  double *d_pAhat = nullptr, *d_prc = nullptr;
  void* d_plo = nullptr;
  bool assembled = false, bj_ready = false;
  bool lo_hat = false;         // the low-precision copy holds M R^{-1} (else M)
  bool coords_y = false;       // solve in/out coefficients are y = R x (block-Jacobi coordinates)
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::map<int64_t, hipGraphExec_t> graphs;
};

namespace {

elmfb_status bfail(elmfb_batch b, elmfb_status code, const std::string& msg) {
  if (b) b->err = msg;
  g_batch_error = msg;
  return code;
}

#define BHIP(b, expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return bfail((b), ELMFB_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
hipError_t balloc(elmfb_batch b, T** p, int64_t bytes) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, (size_t)(bytes > 0 ? bytes : 16));
  if (e != hipSuccess) return e;
  b->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return hipSuccess;
}

void bfree(elmfb_batch b, void* p) {
  if (!p) return;
  for (size_t i = 0; i < b->allocs.size(); ++i) {
    if (b->allocs[i] == p) {
      hipFree(p);
      b->allocs.erase(b->allocs.begin() + (long)i);
      return;
    }
  }
}

void brelease(elmfb_batch b) {
  for (auto& kv : b->graphs) hipGraphExecDestroy(kv.second);
  b->graphs.clear();
  for (void* p : b->allocs) hipFree(p);
  b->allocs.clear();
  if (b->ev_in) hipEventDestroy(b->ev_in);
  if (b->ev_out) hipEventDestroy(b->ev_out);
  if (b->stream) hipStreamDestroy(b->stream);
  b->ev_in = b->ev_out = nullptr;
  b->stream = nullptr;
}

// Workgroups of a launch go to the 8 XCDs in turn (workgroup w to XCD w mod 8), and each XCD has
// its own L2.  The 64-point runs of one block all read the block's packed factor, so they are
// ordered to land on one XCD: whole blocks are dealt to the XCD with the fewest runs so far, and
// the runs are interleaved by XCD, with empty runs (blk = -1) where an XCD's list is shorter.
constexpr int kXcds = 8;

std::vector<Tile> xcd_grouped(const std::vector<Tile>& runs) {
  std::vector<std::vector<Tile>> q(kXcds);
  for (size_t a = 0; a < runs.size();) {
    size_t b = a;
    while (b < runs.size() && runs[b].blk == runs[a].blk) ++b;
    size_t x = 0;
    for (size_t y = 1; y < q.size(); ++y)
      if (q[y].size() < q[x].size()) x = y;
    q[x].insert(q[x].end(), runs.begin() + a, runs.begin() + b);
    a = b;
  }
  size_t len = 0;
  for (const auto& v : q) len = std::max(len, v.size());
  std::vector<Tile> out;
  out.reserve(len * kXcds);
  for (size_t r = 0; r < len; ++r)
    for (int x = 0; x < kXcds; ++x) out.push_back(r < q[x].size() ? q[x][r] : Tile{-1, 0});
  return out;
}

std::string plan_batch(elmfb_batch B, const elmfb_problem_desc* descs) {
  int64_t row_off = 0, col_off = 0, a_off = 0, p_off = 0, f_off = 0, g_off = 0, nnz = 0;
  int32_t blk_off = 0, tab_off = 0, cov_off = 0;
  for (int i = 0; i < B->n; ++i) {
    elmfb_problem_s hp;
    hp.desc = descs[i];
    hp.lo_prec = descs[i].store_prec;
    const std::string e = plan_problem(&hp);
    if (!e.empty()) return "instance " + std::to_string(i) + ": " + e;
    Geo g = hp.geo;
    for (int l = 0; l < g.n_levels; ++l) {
      g.bbase[l] += blk_off;
      g.cov_off[l][0] += cov_off;
      g.cov_off[l][1] += cov_off;
    }
    B->geos.push_back(g);
    InstInfo I{};
    I.row_off = row_off;
    I.col_off = col_off;
    I.rt0 = (int32_t)B->rtiles.size();
    for (int64_t r0 = 0; r0 < g.n_rows; r0 += 256) B->rtiles.push_back(RowTile{i, (int32_t)(row_off + r0)});
    I.rt1 = (int32_t)B->rtiles.size();
    I.ct0 = (int32_t)B->ctiles.size();
    for (int64_t q0 = 0; q0 < g.n_phi; q0 += 256) B->ctiles.push_back(ColTile{i, (int32_t)(col_off + q0)});
    I.ct1 = (int32_t)B->ctiles.size();
    I.b0 = blk_off;
    I.b1 = blk_off + (int32_t)hp.blocks.size();
    B->insts.push_back(I);
    B->nrows.push_back(g.n_rows);
    B->nphis.push_back(g.n_phi);
    const int64_t K = g.K;
    for (size_t b = 0; b < hp.blocks.size(); ++b) {
      DevBlock D = hp.blocks[b];
      D.a_off += a_off;
      D.p_off += p_off;
      D.q0 += (int32_t)col_off;
      D.tabx += tab_off;
      D.taby += tab_off;
      D.inst = i;
      B->blocks.push_back(D);
      for (int p0 = 0; p0 < D.n; p0 += 64) B->ftiles.push_back(Tile{blk_off + (int32_t)b, p0});
      B->foff.push_back(f_off);
      B->goff.push_back(g_off);
      B->slices.push_back(ColSlice{blk_off + (int32_t)b, 0});
      B->tasks.push_back(GramTask{blk_off + (int32_t)b, 0, 0});
      f_off += K * (K + 1) / 2;
      g_off += K * K;
    }
    B->kmax = std::max(B->kmax, (int)K);
    for (const Tile& t : hp.tiles) B->tiles.push_back(Tile{t.blk + blk_off, t.p0});
    for (const AxisSeg& s : hp.segs) {
      AxisSeg s2 = s;
      s2.tab_off += tab_off;
      B->segs.push_back(BSeg{s2, i, 0});
    }
    B->cov.insert(B->cov.end(), hp.cov.begin(), hp.cov.end());
    row_off += g.n_rows;
    col_off += g.n_phi;
    a_off += hp.n_store;
    nnz += hp.nnz;
    p_off += hp.n_block_points;
    blk_off += (int32_t)hp.blocks.size();
    tab_off += (int32_t)hp.n_tab;
    cov_off += (int32_t)hp.cov.size();
    if (row_off > ((int64_t)1 << 31) || col_off > ((int64_t)1 << 31)) return "batch too large";
  }
  B->ftiles = xcd_grouped(B->ftiles);
  B->n_rows = row_off;
  B->n_phi = col_off;
  B->nnz = nnz;
  B->n_store = a_off;
  B->n_bp = p_off;
  B->n_tab = tab_off;
  B->n_fac = f_off;
  B->n_gsq = g_off;
  return "";
}

// Device bytes of the factors and folded matrices held (the subdomain or the patch ones).
int64_t factor_bytes(elmfb_batch B) {
  const int64_t es_lo = B->lo_prec == ELMFB_FP64 ? 0 : elem_size(B->lo_prec);
  int64_t b = 0;
  if (B->d_rc) b += B->n_fac * 8;
  if (B->d_Ahat) b += B->n_store * 8;
  if (B->d_prc) b += B->pn_fac * 8;
  if (B->d_pAhat) b += B->pn_store * 8;
  if (B->d_plo) b += B->pn_store * es_lo;
  return b;
}

// Scratch for the Gram blocks and factors of the patches, per chunk of patches (two nk x nk
// matrices per patch): the chunks are formed so that each needs at most this many doubles.
constexpr int64_t kPatchScratch = (int64_t)1 << 28;   // 2 GiB of doubles per matrix set

// Patch tables for P: per instance and level, patches of P consecutive subdomains along each
// axis (the last along an axis keeps what is left), in x-major order; a patch block covers the
// bounding box of its members' boxes (their union, as neighbouring supports overlap), holds their
// columns member by member (members in x-major order) and is stored like a subdomain block,
// [nk][ld] feature-major.  A grid index is covered by the patches of the subdomains covering it.
std::string plan_patches(elmfb_batch B, int P) {
  B->pgeos.clear(); B->pinsts.clear(); B->pblocks.clear(); B->pcov.clear(); B->pmem.clear();
  B->pmoff.clear(); B->pperm.assign((size_t)B->n_phi, -1); B->pslices.clear();
  B->pftiles.clear(); B->pruns.clear(); B->pmvruns.clear(); B->ptasks.clear(); B->pfoff.clear();
  B->pgoff.clear();
  B->pchunk_blk.clear(); B->pchunk_task.clear();
  int64_t a_off = 0, p_off = 0, f_off = 0, dense = 0;
  int kmax = 1;
  for (int i = 0; i < B->n; ++i) {
    const Geo& g = B->geos[i];
    const InstInfo& I = B->insts[i];
    const int K = g.K;
    Geo pg = g;
    InstInfo pi = I;
    pi.b0 = (int32_t)B->pslices.size();
    int64_t col = I.col_off;
    int nb_i = 0;
    for (int l = 0; l < g.n_levels; ++l) {
      const int Jx = g.J[l][0], Jy = g.J[l][1];
      const int PJx = (Jx + P - 1) / P, PJy = (Jy + P - 1) / P;
      pg.J[l][0] = PJx;
      pg.J[l][1] = PJy;
      pg.bbase[l] = (int32_t)B->pblocks.size();
      for (int a = 0; a < 2; ++a) {
        const int np = a == 0 ? g.nx : g.ny;
        pg.cov_off[l][a] = (int32_t)B->pcov.size();
        for (int m = 0; m < np; ++m) {
          const int jlo = B->cov[g.cov_off[l][a] + 2 * m], jhi = B->cov[g.cov_off[l][a] + 2 * m + 1];
          B->pcov.push_back(jhi >= jlo ? jlo / P : 0);
          B->pcov.push_back(jhi >= jlo ? jhi / P : -1);
        }
      }
      for (int px = 0; px < PJx; ++px)
        for (int py = 0; py < PJy; ++py) {
          DevBlock D{};
          int x0 = 1 << 30, x1 = -1, y0 = 1 << 30, y1 = -1, nm = 0;
          B->pmoff.push_back((int32_t)B->pmem.size());
          for (int jx = P * px; jx < std::min(P * px + P, Jx); ++jx)
            for (int jy = P * py; jy < std::min(P * py + P, Jy); ++jy) {
              const int mb = g.bbase[l] + jx * Jy + jy;
              const DevBlock& M = B->blocks[mb];
              B->pmem.push_back(mb);
              for (int k = 0; k < K; ++k) B->pperm[col + (int64_t)nm * K + k] = M.q0 + k;
              ++nm;
              if (M.n == 0) continue;
              x0 = std::min(x0, M.ix0); x1 = std::max(x1, M.ix0 + M.nx);
              y0 = std::min(y0, M.iy0); y1 = std::max(y1, M.iy0 + M.ny);
            }
          if (x1 < 0) { x0 = x1 = y0 = y1 = 0; }
          D.nk = nm * K;
          if (D.nk > kPatchMaxK)
            return "a patch holds more than 512 columns: take a smaller patch size";
          D.ix0 = x0; D.nx = x1 - x0; D.iy0 = y0; D.ny = y1 - y0;
          D.n = D.nx * D.ny;
          D.ld = (D.n + kRowAlign - 1) / kRowAlign * kRowAlign;
          D.a_off = a_off;
          D.p_off = p_off;
          D.q0 = (int32_t)col;
          D.level = l;
          D.inst = i;
          D.jx = px;
          D.jy = py;
          const int b = (int)B->pblocks.size();
          B->pblocks.push_back(D);
          for (int k0 = 0; k0 < D.nk; k0 += kBatchMaxK) B->pslices.push_back(ColSlice{b, k0});
          for (int p0 = 0; p0 < D.ld; p0 += 256) B->pruns.push_back(Tile{b, p0});
          for (int i0 = 0; i0 < D.nk; i0 += kBatchMaxK)
            for (int j0 = i0; j0 < D.nk; j0 += kBatchMaxK) B->ptasks.push_back(GramTask{b, i0, j0});
          B->pfoff.push_back(f_off);
          f_off += (int64_t)D.nk * (D.nk + 1) / 2;
          a_off += (int64_t)D.nk * D.ld;
          p_off += D.n;
          dense += (int64_t)D.nk * D.n;
          col += D.nk;
          kmax = std::max(kmax, D.nk);
          ++nb_i;
        }
    }
    pg.n_blocks = nb_i;
    pi.b1 = (int32_t)B->pslices.size();
    B->pgeos.push_back(pg);
    B->pinsts.push_back(pi);
  }
  // fold runs, dealt to the XCDs by block; factor chunks with their scratch offsets
  const int run = fold_run_points(kmax);
  std::vector<Tile> ft;
  for (size_t b = 0; b < B->pblocks.size(); ++b)
    for (int p0 = 0; p0 < B->pblocks[b].n; p0 += run) ft.push_back(Tile{(int32_t)b, p0});
  B->pftiles = xcd_grouped(ft);
  std::vector<Tile> mr;
  for (size_t b = 0; b < B->pblocks.size(); ++b)
    for (int p0 = 0; p0 < B->pblocks[b].n; p0 += 256) mr.push_back(Tile{(int32_t)b, p0});
  B->pmvruns = xcd_grouped(mr);
  int64_t g_off = 0, scratch = 0;
  size_t t = 0;
  for (size_t b = 0; b < B->pblocks.size(); ++b) {
    const int64_t sq = (int64_t)B->pblocks[b].nk * B->pblocks[b].nk;
    if (b == 0 || g_off + sq > kPatchScratch) {
      B->pchunk_blk.push_back((int64_t)b);
      while (t < B->ptasks.size() && B->ptasks[t].blk < (int32_t)b) ++t;
      B->pchunk_task.push_back((int64_t)t);
      g_off = 0;
    }
    B->pgoff.push_back(g_off);
    g_off += sq;
    scratch = std::max(scratch, g_off);
  }
  B->pchunk_blk.push_back((int64_t)B->pblocks.size());
  B->pchunk_task.push_back((int64_t)B->ptasks.size());
  B->pkmax = kmax;
  B->pn_store = a_off;
  B->pn_bp = p_off;
  B->pn_fac = f_off;
  B->pn_scratch = scratch;
  B->pn_dense = dense;
  return "";
}

// The block structure a pass runs on: the subdomain blocks of the assembly, or the patch blocks
// of the block-Jacobi preconditioner.
struct BtLayout {
  const Geo* geos;
  const InstInfo* insts;
  const DevBlock* blocks;
  int64_t nb;
  const Tile* mv_runs;   // point runs of the M V pass (NULL: one workgroup per block)
  int64_t n_mv;          // its grid: runs, or blocks
  const int32_t* cov;
  const ColSlice* slices;
  int64_t ns;
  int kmax;
  int64_t n_bp;
};

BtLayout sub_layout(elmfb_batch B) {
  return BtLayout{B->d_geos, B->d_insts, B->d_blocks, (int64_t)B->blocks.size(), nullptr,
                  (int64_t)B->blocks.size(), B->d_cov, B->d_slices, (int64_t)B->slices.size(),
                  B->kmax, B->n_bp};
}

BtLayout patch_layout(elmfb_batch B) {
  return BtLayout{B->d_pgeos, B->d_pinsts, B->d_pblocks, (int64_t)B->pblocks.size(),
                  B->d_pmvruns, (int64_t)B->pmvruns.size(), B->d_pcov, B->d_pslices,
                  (int64_t)B->pslices.size(), B->pkmax, B->pn_bp};
}

// Preconditioned passes run on the folded matrix, in the patch layout when the factors are of
// patches; everything else on the subdomain blocks.
BtLayout layout_of(elmfb_batch B, bool bj) {
  return bj && B->patch > 1 ? patch_layout(B) : sub_layout(B);
}

int prec_index(int prec) {
  return prec == ELMFB_FP32 ? 1 : (prec == ELMFB_BF16 ? 2 : (prec == ELMFB_FP16 ? 3 : 0));
}

// The matrix the Krylov steps run on: M, or with block-Jacobi the folded M R^{-1}; FP64 or the
// low-precision copy.
const void* matrix_of(elmfb_batch B, int prec, bool bj) {
  const bool pt = bj && B->patch > 1;
  if (prec == ELMFB_FP64)
    return bj ? (pt ? (const void*)B->d_pAhat : (const void*)B->d_Ahat) : (const void*)B->d_A;
  return pt ? (const void*)B->d_plo : (const void*)B->d_A_lo;
}

// Factors, their offsets and the column order of the preconditioned coefficients.
const double* factors_of(elmfb_batch B) { return B->patch > 1 ? B->d_prc : B->d_rc; }
const int64_t* foff_of(elmfb_batch B) { return B->patch > 1 ? B->d_pfoff : B->d_foff; }
const int32_t* perm_of(elmfb_batch B) { return B->patch > 1 ? B->d_pperm : nullptr; }

// The matrix copy of precision prec that tuning and timing run on, with its layout: the folded
// patch matrices while patch factors are held (the solves run on them), else the stored copy of
// M (for P = 1 its low-precision buffer holds M R^{-1} after preconditioning).
struct TimedTarget {
  BtLayout L;
  const void* A;
};
TimedTarget timed_target(elmfb_batch B, int prec) {
  if (B->patch > 1 && B->bj_ready) return TimedTarget{patch_layout(B), matrix_of(B, prec, true)};
  return TimedTarget{sub_layout(B), matrix_of(B, prec, false)};
}

// One LSQR step for every (instance, rhs) on the matrix of precision `prec` (M, or M R^{-1} with
// block-Jacobi): u = A v sv - alpha su u, beta; v = A^T u su - beta sv v, alpha; rotation;
// x, w update; stop tests.
hipError_t bt_iteration(elmfb_batch B, int prec, bool bj, hipStream_t s) {
  const int n = B->n, R = B->R;
  const BtLayout L = layout_of(B, bj);
  const void* A = matrix_of(B, prec, bj);
  hipError_t e;
  if ((e = launch_bt_mvb(prec, L.blocks, L.mv_runs, L.n_mv, L.kmax, A, B->d_v, R, B->d_state,
                         B->d_tpart, s, B->fa[prec_index(prec)])))
    return e;
  if ((e = launch_bt_gather(L.geos, L.insts, L.blocks, L.cov, B->d_rtiles,
                            (int64_t)B->rtiles.size(), B->d_tpart, ROW_LSQR_U, R, B->d_u, nullptr,
                            B->d_state, B->d_red_r, s, B->rpt)))
    return e;
  if ((e = launch_bt_lsqr_beta(B->d_state, L.insts, n, R, B->d_red_r, s))) return e;
  if ((e = launch_bt_rmvb(prec, B->tp[prec_index(prec)], L.geos, L.insts, L.blocks, L.slices, L.ns,
                          A, B->d_u, R, B->d_state, COL_LSQR_V, B->d_v, B->d_red_c, s)))
    return e;
  if ((e = launch_bt_lsqr_alpha(B->d_state, L.insts, n, R, B->d_red_c, s))) return e;
  if ((e = launch_bt_update(B->d_geos, L.insts, B->d_ctiles, (int64_t)B->ctiles.size(), R,
                            B->d_x, B->d_w, B->d_v, B->d_state, B->d_red_b, s)))
    return e;
  return launch_bt_lsqr_stop(B->d_state, L.insts, n, R, B->d_red_b, s);
}

// LSQR start from the rows already in d_u (u = rhs) with their squared-norm partials in
// d_red_r: beta, v = A^T u / beta, alpha, w = v / alpha, x = 0.  red_b: partials of the norm
// the stop tests are relative to (default: ||u||).
hipError_t bt_lsqr_start(elmfb_batch B, int prec, bool bj, double atol, double btol, int iter_lim,
                         const BtOuter* ot, double inner_rel, hipStream_t s,
                         const double* red_b = nullptr) {
  const int n = B->n, R = B->R;
  const BtLayout L = layout_of(B, bj);
  hipError_t e;
  if ((e = launch_bt_lsqr_init(B->d_state, L.insts, n, R, red_b ? red_b : B->d_red_r,
                               B->d_red_r, atol, btol, iter_lim, ot, inner_rel, s)))
    return e;
  if ((e = launch_bt_rmvb(prec, B->tp[prec_index(prec)], L.geos, L.insts, L.blocks, L.slices, L.ns,
                          matrix_of(B, prec, bj), B->d_u, R, B->d_state, COL_STORE_SQ, B->d_v,
                          B->d_red_c, s)))
    return e;
  if ((e = launch_bt_lsqr_init_alpha(B->d_state, L.insts, n, R, B->d_red_c, s))) return e;
  if ((e = hipMemsetAsync(B->d_x, 0, (size_t)(B->n_phi * R * 8), s))) return e;
  if ((e = hipMemsetAsync(B->d_w, 0, (size_t)(B->n_phi * R * 8), s))) return e;
  // with t1 = t2 = 0 (fresh state) the update leaves x = 0 and sets w = v sv
  return launch_bt_update(B->d_geos, L.insts, B->d_ctiles, (int64_t)B->ctiles.size(), R,
                          B->d_x, B->d_w, B->d_v, B->d_state, B->d_red_b, s);
}

// u = b - A c with the FP64 matrix A (M, or M R^{-1} with block-Jacobi and c in preconditioned
// coordinates), squared-norm partials in d_red_r; c = NULL means c = 0; b = NULL means h.
hipError_t bt_residual(elmfb_batch B, const double* c, bool bj, hipStream_t s,
                       const double* b = nullptr) {
  const int R = B->R;
  const BtLayout L = layout_of(B, bj);
  hipError_t e;
  if (c) {
    if ((e = launch_bt_mvb(ELMFB_FP64, L.blocks, L.mv_runs, L.n_mv, L.kmax,
                           matrix_of(B, ELMFB_FP64, bj), c, R, nullptr, B->d_tpart, s,
                           B->fa[0])))
      return e;
  } else if ((e = hipMemsetAsync(B->d_tpart, 0, (size_t)(L.n_bp * R * 8), s))) {
    return e;
  }
  return launch_bt_gather(L.geos, L.insts, L.blocks, L.cov, B->d_rtiles,
                          (int64_t)B->rtiles.size(), B->d_tpart, ROW_RESID, R, B->d_u,
                          b ? b : B->d_h, nullptr, B->d_red_r, s, B->rpt);
}

// Run LSQR steps until every pair has stopped: replays of a captured graph of `chunk` steps (or
// eager launches), the host reading the number of running pairs after each.
elmfb_status bt_run(elmfb_batch B, int prec, bool bj, int chunk, bool use_graph, hipStream_t s) {
  const int nR = B->n * B->R;
  int32_t active = 1;
  BHIP(B, launch_bt_count_active(B->d_state, nR, B->d_count, s));
  BHIP(B, hipMemcpyAsync(&active, B->d_count, 4, hipMemcpyDeviceToHost, s));
  BHIP(B, hipStreamSynchronize(s));
  while (active > 0) {
    if (use_graph) {
      // graphs of at most kGraphMaxSteps steps, replayed until `chunk` steps are enqueued
      for (int left = chunk; left > 0;) {
        const int m = left > kGraphMaxSteps ? kGraphMaxSteps : left;
        // the captured kernels depend on the tuned shapes as well
        const int64_t key = ((int64_t)m << 24) | ((int64_t)B->rpt << 20) |
                            ((int64_t)B->fa[prec_index(prec)] << 15) |
                            ((int64_t)(bj ? B->patch : 0) << 10) | (prec << 8) |
                            (bj ? 128 : 0) | B->tp[prec_index(prec)];
        auto it = B->graphs.find(key);
        hipGraphExec_t exec = nullptr;
        if (it != B->graphs.end()) {
          exec = it->second;
        } else {
          hipGraph_t graph = nullptr;
          BHIP(B, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
          hipError_t e2 = hipSuccess;
          for (int i = 0; i < m && e2 == hipSuccess; ++i) e2 = bt_iteration(B, prec, bj, s);
          hipError_t e3 = hipStreamEndCapture(s, &graph);
          if (e2 != hipSuccess || e3 != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            BHIP(B, e2 != hipSuccess ? e2 : e3);
          }
          hipError_t e4 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
          hipGraphDestroy(graph);
          BHIP(B, e4);
          B->graphs[key] = exec;
        }
        BHIP(B, hipGraphLaunch(exec, s));
        left -= m;
      }
    } else {
      for (int i = 0; i < chunk; ++i) BHIP(B, bt_iteration(B, prec, bj, s));
    }
    BHIP(B, launch_bt_count_active(B->d_state, nR, B->d_count, s));
    BHIP(B, hipMemcpyAsync(&active, B->d_count, 4, hipMemcpyDeviceToHost, s));
    BHIP(B, hipStreamSynchronize(s));
  }
  return ELMFB_OK;
}

}  // namespace

extern "C" {

elmfb_status elmfb_define_batch(const elmfb_problem_desc* descs, int32_t n, int32_t n_rhs,
                                elmfb_batch* out) {
  if (!out || !descs) return bfail(nullptr, ELMFB_E_INVALID, "NULL argument");
  *out = nullptr;
  if (n < 1) return bfail(nullptr, ELMFB_E_INVALID, "n must be >= 1");
  if (n_rhs < 1 || n_rhs > kMaxRhs) return bfail(nullptr, ELMFB_E_INVALID, "n_rhs must be in 1..8");
  for (int i = 0; i < n; ++i) {
    const std::string v = validate_desc(&descs[i]);
    if (!v.empty()) return bfail(nullptr, ELMFB_E_INVALID, "instance " + std::to_string(i) + ": " + v);
    if (descs[i].K > kBatchMaxK) return bfail(nullptr, ELMFB_E_INVALID, "batched instances need K <= 128");
    if (descs[i].n_bc != 0 || descs[i].n_bc_pts != 0 || descs[i].op == ELMFB_OP_OSCILLATOR ||
        descs[i].op == ELMFB_OP_HELMHOLTZ || descs[i].domain != ELMFB_DOMAIN_BOX)
      return bfail(nullptr, ELMFB_E_UNSUPPORTED,
                   "batched instances: box domains only, no soft-constraint rows, no oscillator "
                   "or Helmholtz operator");
    if (descs[i].store_prec != descs[0].store_prec)
      return bfail(nullptr, ELMFB_E_INVALID, "all instances need the same store_prec");
  }
  elmfb_batch B = new (std::nothrow) elmfb_batch_s();
  if (!B) return bfail(nullptr, ELMFB_E_NOMEM, "host allocation failed");
  B->n = n;
  B->R = n_rhs;
  B->lo_prec = descs[0].store_prec;
  const std::string pe = plan_batch(B, descs);
  if (!pe.empty()) {
    delete B;
    return bfail(nullptr, ELMFB_E_INVALID, pe);
  }
  const int R = n_rhs;
  const int64_t es_lo = B->lo_prec == ELMFB_FP64 ? 0 : elem_size(B->lo_prec);
  const int64_t nblk = (int64_t)B->blocks.size();
  int64_t bytes = B->n_store * (8 + es_lo) + B->n_bp * R * 8 + B->n_rows * R * 8 * 2 +
                  B->n_phi * R * 8 * 4 + B->n_phi * 24 + B->n_tab * 24 +
                  (int64_t)(B->rtiles.size() * 3 + B->ctiles.size() + nblk) * kMaxRhs * 8 +
                  nblk * ((int64_t)sizeof(DevBlock) + 16 + (int64_t)sizeof(ColSlice) +
                          (int64_t)sizeof(GramTask)) +
                  (int64_t)(B->tiles.size() + B->ftiles.size()) * sizeof(Tile) +
                  (int64_t)n * R * ((int64_t)sizeof(SolveState) + (int64_t)sizeof(BtOuter));
  B->bytes = bytes;
  if (const char* cap = std::getenv("ELMFB_MEM_CAP")) {
    const long long c = std::atoll(cap);
    if (c > 0 && bytes > c) {
      delete B;
      return bfail(nullptr, ELMFB_E_NOMEM, "batch footprint exceeds ELMFB_MEM_CAP");
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    delete B;
    return bfail(nullptr, ELMFB_E_DEVICE, "no HIP device available");
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && (size_t)bytes > free_b) {
    delete B;
    return bfail(nullptr, ELMFB_E_NOMEM, "batch footprint exceeds free device memory");
  }
#define BALLOC(p, nbytes)                                                          \
  do {                                                                             \
    hipError_t e_ = balloc(B, &(p), (nbytes));                                     \
    if (e_ != hipSuccess) {                                                        \
      brelease(B);                                                                 \
      delete B;                                                                    \
      return bfail(nullptr, ELMFB_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e_)); \
    }                                                                              \
  } while (0)
  BALLOC(B->d_geos, n * (int64_t)sizeof(Geo));
  BALLOC(B->d_insts, n * (int64_t)sizeof(InstInfo));
  BALLOC(B->d_nrows, n * 8);
  BALLOC(B->d_nphis, n * 8);
  BALLOC(B->d_blocks, nblk * (int64_t)sizeof(DevBlock));
  BALLOC(B->d_foff, nblk * 8);
  BALLOC(B->d_goff, nblk * 8);
  BALLOC(B->d_slices, nblk * (int64_t)sizeof(ColSlice));
  BALLOC(B->d_tasks, nblk * (int64_t)sizeof(GramTask));
  BALLOC(B->d_tiles, (int64_t)B->tiles.size() * sizeof(Tile));
  BALLOC(B->d_cov, (int64_t)B->cov.size() * 4);
  BALLOC(B->d_segs, (int64_t)B->segs.size() * sizeof(BSeg));
  BALLOC(B->d_rtiles, (int64_t)B->rtiles.size() * sizeof(RowTile));
  BALLOC(B->d_ctiles, (int64_t)B->ctiles.size() * sizeof(ColTile));
  BALLOC(B->d_tab, B->n_tab * 24);
  BALLOC(B->d_W, B->n_phi * 16);
  BALLOC(B->d_b, B->n_phi * 8);
  BALLOC(B->d_A, B->n_store * 8);
  if (es_lo) BALLOC(B->d_A_lo, B->n_store * es_lo);
  BALLOC(B->d_h, B->n_rows * R * 8);
  BALLOC(B->d_u, B->n_rows * R * 8);
  BALLOC(B->d_v, B->n_phi * R * 8);
  BALLOC(B->d_w, B->n_phi * R * 8);
  BALLOC(B->d_x, B->n_phi * R * 8);
  BALLOC(B->d_c, B->n_phi * R * 8);
  BALLOC(B->d_ftiles, (int64_t)B->ftiles.size() * sizeof(Tile));
  BALLOC(B->d_tpart, B->n_bp * R * 8);
  B->tpart_bp = B->n_bp;
  BALLOC(B->d_red_r, (int64_t)B->rtiles.size() * kMaxRhs * 8);
  BALLOC(B->d_red_b, (int64_t)B->ctiles.size() * kMaxRhs * 8);
  BALLOC(B->d_red_c, nblk * kMaxRhs * 8);
  BALLOC(B->d_red_h, (int64_t)B->rtiles.size() * kMaxRhs * 8);
  BALLOC(B->d_state, (int64_t)n * R * sizeof(SolveState));
  BALLOC(B->d_outer, (int64_t)n * R * sizeof(BtOuter));
  BALLOC(B->d_flag, 64);
  BALLOC(B->d_count, 64);
#undef BALLOC
  // features, W padded to two columns, instance by instance
  std::vector<double> W2((size_t)B->n_phi * 2, 0.0), bb((size_t)B->n_phi, 0.0);
  std::vector<double> Wd, bd;   // parameters drawn by the library for instances without them
  for (int i = 0; i < n; ++i) {
    const elmfb_problem_desc& d = descs[i];
    const double* Wi = d.W_host;
    const double* bi = d.b_host;
    if (!Wi) {
      const int64_t np = feature_param_count(d);
      Wd.assign((size_t)(np * d.dim), 0.0);
      bd.assign((size_t)np, 0.0);
      draw_feature_params(d, Wd.data(), bd.data());
      Wi = Wd.data();
      bi = bd.data();
    }
    const int64_t c0 = B->insts[i].col_off;
    for (int64_t q = 0; q < B->nphis[i]; ++q) {
      for (int a = 0; a < d.dim; ++a) W2[2 * (c0 + q) + a] = Wi[q * d.dim + a];
      bb[c0 + q] = bi[q];
    }
  }
  hipError_t e = hipSuccess;
  auto up = [&](void* dst, const void* src, size_t bytes_) {
    if (e == hipSuccess && bytes_ > 0) e = hipMemcpy(dst, src, bytes_, hipMemcpyHostToDevice);
  };
  up(B->d_geos, B->geos.data(), B->geos.size() * sizeof(Geo));
  up(B->d_insts, B->insts.data(), B->insts.size() * sizeof(InstInfo));
  up(B->d_nrows, B->nrows.data(), B->nrows.size() * 8);
  up(B->d_nphis, B->nphis.data(), B->nphis.size() * 8);
  up(B->d_blocks, B->blocks.data(), B->blocks.size() * sizeof(DevBlock));
  up(B->d_foff, B->foff.data(), B->foff.size() * 8);
  up(B->d_goff, B->goff.data(), B->goff.size() * 8);
  up(B->d_slices, B->slices.data(), B->slices.size() * sizeof(ColSlice));
  up(B->d_tasks, B->tasks.data(), B->tasks.size() * sizeof(GramTask));
  up(B->d_tiles, B->tiles.data(), B->tiles.size() * sizeof(Tile));
  up(B->d_ftiles, B->ftiles.data(), B->ftiles.size() * sizeof(Tile));
  up(B->d_cov, B->cov.data(), B->cov.size() * 4);
  up(B->d_segs, B->segs.data(), B->segs.size() * sizeof(BSeg));
  up(B->d_rtiles, B->rtiles.data(), B->rtiles.size() * sizeof(RowTile));
  up(B->d_ctiles, B->ctiles.data(), B->ctiles.size() * sizeof(ColTile));
  up(B->d_W, W2.data(), W2.size() * 8);
  up(B->d_b, bb.data(), bb.size() * 8);
  // the row padding of the stored blocks is never assembled; the matrix passes may read it with
  // zero weights, so it must hold finite values
  if (e == hipSuccess) e = hipMemset(B->d_A, 0, (size_t)B->n_store * 8);
  if (e == hipSuccess && B->d_A_lo) e = hipMemset(B->d_A_lo, 0, (size_t)(B->n_store * es_lo));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming);
  if (e == hipSuccess)
    e = launch_bt_tables(B->d_geos, B->d_segs, (int)B->segs.size(), B->d_cov, B->d_tab, B->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
  if (e != hipSuccess) {
    const std::string m = std::string("batch setup: ") + hipGetErrorString(e);
    brelease(B);
    delete B;
    return bfail(nullptr, ELMFB_E_DEVICE, m);
  }
  *out = B;
  return ELMFB_OK;
}

elmfb_status elmfb_batch_query(elmfb_batch B, int64_t* offsets_host, elmfb_sizes* totals_host) {
  if (!B) return bfail(B, ELMFB_E_INVALID, "NULL batch");
  if (offsets_host) {
    for (int i = 0; i < B->n; ++i) {
      offsets_host[2 * i] = B->insts[i].row_off;
      offsets_host[2 * i + 1] = B->insts[i].col_off;
    }
    offsets_host[2 * B->n] = B->n_rows;
    offsets_host[2 * B->n + 1] = B->n_phi;
  }
  if (totals_host) {
    totals_host->n_rows = B->n_rows;
    totals_host->n_phi = B->n_phi;
    totals_host->nnz = B->nnz;
    totals_host->n_blocks = (int64_t)B->blocks.size();
    totals_host->n_block_points = B->n_bp;
    totals_host->bytes_device = B->bytes;
    totals_host->n_pairs = 0;
    totals_host->n_bc = 0;
    totals_host->n_interior = B->n_rows;
  }
  return ELMFB_OK;
}

elmfb_status elmfb_batch_query_instances(elmfb_batch B, elmfb_sizes* out) {
  if (!B || !out) return bfail(B, ELMFB_E_INVALID, "NULL argument");
  for (int i = 0; i < B->n; ++i) {
    elmfb_sizes& z = out[i];
    z = elmfb_sizes{};
    z.n_rows = B->nrows[i];
    z.n_phi = B->nphis[i];
    z.n_interior = B->nrows[i];
  }
  // stored entries, blocks and block points per instance from the block table
  int64_t stored = 0;
  for (const DevBlock& b : B->blocks) {
    elmfb_sizes& z = out[b.inst];
    z.nnz += (int64_t)b.n * B->geos[b.inst].K;
    z.n_blocks += 1;
    z.n_block_points += b.n;
    stored += (int64_t)b.ld * B->geos[b.inst].K;
  }
  // the instance's share of the device footprint, by its share of the stored entries
  for (int i = 0; i < B->n; ++i) {
    int64_t mine = 0;
    for (int64_t j = B->insts[i].b0; j < B->insts[i].b1; ++j)
      mine += (int64_t)B->blocks[j].ld * B->geos[i].K;
    out[i].bytes_device = stored > 0 ? (int64_t)((double)B->bytes * mine / stored) : 0;
  }
  return ELMFB_OK;
}

elmfb_status elmfb_batch_copy_blocks(elmfb_batch B, int32_t prec, void* dst_dev,
                                     int64_t* table_host, void* stream) {
  if (!B) return bfail(B, ELMFB_E_INVALID, "NULL batch");
  const bool folded = (prec & ELMFB_COPY_FOLDED) != 0;
  prec &= ~ELMFB_COPY_FOLDED;
  // folded copies of patch factors are stored in the patch blocks
  const bool pt = folded && B->patch > 1 && B->bj_ready;
  const std::vector<DevBlock>& blocks = pt ? B->pblocks : B->blocks;
  if (table_host) {
    int64_t dense = 0;
    for (size_t i = 0; i < blocks.size(); ++i) {
      const DevBlock& d = blocks[i];
      int64_t* t = table_host + 8 * i;
      t[0] = d.inst;
      t[1] = d.level;
      t[2] = d.ix0;
      t[3] = d.nx;
      t[4] = d.iy0;
      t[5] = d.ny;
      t[6] = d.nk;
      t[7] = dense;
      dense += (int64_t)d.n * d.nk;
    }
  }
  if (dst_dev) {
    if (!B->assembled) return bfail(B, ELMFB_E_STATE, "copy_blocks before assemble");
    const void* src = nullptr;
    if (prec == ELMFB_FP64) {
      src = folded ? (B->bj_ready ? matrix_of(B, ELMFB_FP64, true) : nullptr) : (const void*)B->d_A;
    } else if (prec == B->lo_prec && B->d_A_lo) {
      // the low-precision buffer holds M until elmfb_batch_precondition, then M R^{-1} (per
      // subdomain); the folded copy of patch factors has its own buffer
      if (pt) src = B->d_plo;
      else src = folded == B->lo_hat ? B->d_A_lo : nullptr;
    }
    if (!src) return bfail(B, ELMFB_E_STATE, "no stored copy of that kind and precision");
    // stored rows are padded to ld; the copy drops the padding
    const int64_t es = elem_size(prec);
    int64_t dense = 0;
    for (const DevBlock& d : blocks) {
      if (d.n == 0) continue;
      BHIP(B, hipMemcpy2DAsync(static_cast<char*>(dst_dev) + dense * es, (size_t)(d.n * es),
                               static_cast<const char*>(src) + d.a_off * es, (size_t)(d.ld * es),
                               (size_t)(d.n * es), (size_t)d.nk, hipMemcpyDeviceToDevice,
                               (hipStream_t)stream));
      dense += (int64_t)d.n * d.nk;
    }
  }
  return ELMFB_OK;
}

elmfb_status elmfb_batch_assemble(elmfb_batch B, const double* f_dev, void* stream) {
  if (!B || !f_dev) return bfail(B, ELMFB_E_INVALID, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  BHIP(B, hipMemsetAsync(B->d_flag, 0, 4, s));
  BHIP(B, launch_bt_rhs(B->d_geos, B->d_insts, B->d_rtiles, (int64_t)B->rtiles.size(), B->R,
                        f_dev, B->d_h, B->d_flag, s));
  B->bj_ready = false;
  B->lo_hat = false;
  B->lo_unsafe = false;
  BHIP(B, launch_bt_assemble(B->lo_prec, B->d_geos, B->d_blocks, B->d_tiles,
                             (int64_t)B->tiles.size(), B->d_tab, B->d_W, B->d_b, B->d_A,
                             B->d_A_lo, s));
  int32_t bad = 0;
  BHIP(B, hipMemcpyAsync(&bad, B->d_flag, 4, hipMemcpyDeviceToHost, s));
  BHIP(B, hipStreamSynchronize(s));
  if (bad) {
    B->assembled = false;
    return bfail(B, ELMFB_E_NUMERIC, "f holds non-finite values");
  }
  B->assembled = true;
  return ELMFB_OK;
}

elmfb_status elmfb_batch_matvec(elmfb_batch B, const double* v_dev, double* y_dev, void* stream) {
  if (!B || !v_dev || !y_dev) return bfail(B, ELMFB_E_INVALID, "NULL argument");
  if (!B->assembled) return bfail(B, ELMFB_E_STATE, "matvec before assemble");
  hipStream_t s = (hipStream_t)stream;
  const int R = B->R;
  BHIP(B, launch_bt_pack(B->d_insts, B->d_nphis, B->n, R, B->n_phi, v_dev, B->d_w, 1, 1, s));
  BHIP(B, launch_bt_mvb(ELMFB_FP64, B->d_blocks, nullptr, (int64_t)B->blocks.size(), B->kmax,
                        B->d_A, B->d_w, R, nullptr, B->d_tpart, s, B->fa[0]));
  BHIP(B, launch_bt_gather(B->d_geos, B->d_insts, B->d_blocks, B->d_cov, B->d_rtiles,
                           (int64_t)B->rtiles.size(), B->d_tpart, ROW_STORE, R, B->d_u, nullptr,
                           nullptr, B->d_red_r, s, B->rpt));
  BHIP(B, launch_bt_pack(B->d_insts, B->d_nrows, B->n, R, B->n_rows, B->d_u, y_dev, 0, 0, s));
  return ELMFB_OK;
}

elmfb_status elmfb_batch_rmatvec(elmfb_batch B, const double* u_dev, double* x_dev, void* stream) {
  if (!B || !u_dev || !x_dev) return bfail(B, ELMFB_E_INVALID, "NULL argument");
  if (!B->assembled) return bfail(B, ELMFB_E_STATE, "rmatvec before assemble");
  hipStream_t s = (hipStream_t)stream;
  const int R = B->R;
  BHIP(B, launch_bt_pack(B->d_insts, B->d_nrows, B->n, R, B->n_rows, u_dev, B->d_u, 1, 0, s));
  BHIP(B, launch_bt_rmvb(ELMFB_FP64, B->tp[0], B->d_geos, B->d_insts, B->d_blocks, B->d_slices,
                         (int64_t)B->slices.size(), B->d_A, B->d_u, R, nullptr, COL_STORE, B->d_w,
                         B->d_red_c, s));
  BHIP(B, launch_bt_pack(B->d_insts, B->d_nphis, B->n, R, B->n_phi, B->d_w, x_dev, 0, 1, s));
  return ELMFB_OK;
}

elmfb_status elmfb_batch_precondition(elmfb_batch B, double shift, int32_t* n_fallback_host,
                                      void* stream) {
  return elmfb_batch_precondition_patches(B, shift, 1, n_fallback_host, stream);
}

elmfb_status elmfb_batch_precondition_patches(elmfb_batch B, double shift, int32_t patch,
                                              int32_t* n_fallback_host, void* stream) {
  if (!B) return bfail(B, ELMFB_E_INVALID, "NULL batch");
  if (!B->assembled) return bfail(B, ELMFB_E_STATE, "precondition before assemble");
  if (!(shift > 0.0) || !(shift < 1.0)) return bfail(B, ELMFB_E_INVALID, "shift must be in (0, 1)");
  if (patch < 1 || patch > 4) return bfail(B, ELMFB_E_INVALID, "patch must be in 1..4");
  if (patch > 1 && B->coords_y)
    return bfail(B, ELMFB_E_UNSUPPORTED, "block-Jacobi coordinates are per subdomain (patch 1)");
  // the widest patch, checked before any table or factor held is touched
  for (const Geo& g : B->geos)
    for (int l = 0; l < g.n_levels; ++l)
      if ((int64_t)std::min(patch, (int)g.J[l][0]) * std::min(patch, (int)g.J[l][1]) * g.K >
          kPatchMaxK)
        return bfail(B, ELMFB_E_INVALID,
                     "a patch holds more than 512 columns: take a smaller patch size");
  hipStream_t s = (hipStream_t)stream;
  auto release = [&](auto*& p) { bfree(B, p); p = nullptr; };
  if (patch > 1 && B->patch_planned != patch) {
    B->patch_planned = 0;
    const std::string pe = plan_patches(B, patch);   // cannot fail after the check above
    if (!pe.empty()) return bfail(B, ELMFB_E_INVALID, pe);
  }
  B->bj_ready = false;
  // device bytes held for factors and folded copies: settled on every exit, error returns
  // included (storage may be released or allocated before a later step fails)
  struct FactorBytes {
    elmfb_batch b;
    int64_t before;
    ~FactorBytes() { b->bytes += factor_bytes(b) - before; }
  } factor_guard{B, factor_bytes(B)};
  // the factors of one patch size at a time: release the other kind's storage
  if (patch == 1) {
    release(B->d_pAhat); release(B->d_prc); release(B->d_plo);
  } else {
    release(B->d_Ahat); release(B->d_rc);
  }
  for (auto& kv : B->graphs) hipGraphExecDestroy(kv.second);
  B->graphs.clear();
  int32_t nfail = 0;
  hipError_t e = hipMemsetAsync(B->d_flag, 0, 4, s);
  if (patch == 1) {
    const int64_t nb = (int64_t)B->blocks.size();
    if (!B->d_rc) {
      hipError_t e1 = balloc(B, &B->d_rc, B->n_fac * 8);
      hipError_t e2 = e1 == hipSuccess ? balloc(B, &B->d_Ahat, B->n_store * 8) : e1;
      if (e2 == hipSuccess) e2 = hipMemsetAsync(B->d_Ahat, 0, (size_t)B->n_store * 8, s);  // padding
      if (e2 != hipSuccess) {
        release(B->d_rc);
        release(B->d_Ahat);
        return bfail(B, ELMFB_E_NOMEM, std::string("factor storage: ") + hipGetErrorString(e2));
      }
    }
    double* G = nullptr;
    hipError_t e1 = balloc(B, &G, B->n_gsq * 8);
    if (e1 != hipSuccess)
      return bfail(B, ELMFB_E_NOMEM, std::string("Gram scratch: ") + hipGetErrorString(e1));
    if (e == hipSuccess)
      e = launch_bt_gram_diag(B->d_blocks, B->d_tasks, nb, false, B->d_A, B->d_goff, G, s);
    if (e == hipSuccess)
      e = launch_bt_bj_factor(B->d_blocks, 0, nb, G, B->d_goff, B->d_foff, B->kmax, shift, B->d_rc,
                              B->d_flag, s);
    // M R^{-1} in FP64, and its rounded copy in place of the low-precision M
    if (e == hipSuccess)
      e = launch_bt_fold(B->lo_prec, false, B->kmax, B->d_blocks, B->d_ftiles,
                         (int64_t)B->ftiles.size(), B->d_A, B->d_rc, B->d_foff, B->d_Ahat,
                         B->d_A_lo, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&nfail, B->d_flag, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    bfree(B, G);
    BHIP(B, e);
    B->lo_hat = B->lo_prec != ELMFB_FP64;
  } else {
    if (B->patch_planned != patch) {
      // device tables (replacing those of another patch size)
      release(B->d_pgeos); release(B->d_pinsts); release(B->d_pblocks); release(B->d_pcov);
      release(B->d_pmem); release(B->d_pmoff); release(B->d_pperm); release(B->d_pslices);
      release(B->d_pftiles); release(B->d_pruns); release(B->d_pmvruns); release(B->d_ptasks);
      release(B->d_pfoff);
      release(B->d_pgoff);
      hipError_t ea = hipSuccess;
      auto put = [&](auto*& dst, const auto& v) {
        using T = typename std::remove_reference<decltype(v)>::type::value_type;
        if (ea != hipSuccess) return;
        ea = balloc(B, &dst, (int64_t)(v.size() * sizeof(T)));
        if (ea == hipSuccess && !v.empty())
          ea = hipMemcpy(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
      };
      put(B->d_pgeos, B->pgeos); put(B->d_pinsts, B->pinsts); put(B->d_pblocks, B->pblocks);
      put(B->d_pcov, B->pcov); put(B->d_pmem, B->pmem); put(B->d_pmoff, B->pmoff);
      put(B->d_pperm, B->pperm); put(B->d_pslices, B->pslices); put(B->d_pftiles, B->pftiles);
      put(B->d_pruns, B->pruns); put(B->d_pmvruns, B->pmvruns); put(B->d_ptasks, B->ptasks);
      put(B->d_pfoff, B->pfoff);
      put(B->d_pgoff, B->pgoff);
      // the per-block-point partials of M V must hold the patch boxes as well (the larger
      // buffer replaces the old one only once it is allocated)
      if (ea == hipSuccess && B->pn_bp > B->tpart_bp) {
        double* t = nullptr;
        ea = balloc(B, &t, B->pn_bp * B->R * 8);
        if (ea == hipSuccess) {
          release(B->d_tpart);
          B->d_tpart = t;
          B->bytes += (B->pn_bp - B->tpart_bp) * B->R * 8;
          B->tpart_bp = B->pn_bp;
        }
      }
      release(B->d_pAhat); release(B->d_prc); release(B->d_plo);
      if (ea != hipSuccess) return bfail(B, ELMFB_E_NOMEM, std::string("patch tables: ") + hipGetErrorString(ea));
      B->patch_planned = patch;
    }
    const int64_t es_lo = B->lo_prec == ELMFB_FP64 ? 0 : elem_size(B->lo_prec);
    if (!B->d_pAhat) {
      hipError_t e1 = balloc(B, &B->d_pAhat, B->pn_store * 8);
      if (e1 == hipSuccess) e1 = balloc(B, &B->d_prc, B->pn_fac * 8);
      if (e1 == hipSuccess && es_lo) e1 = balloc(B, &B->d_plo, B->pn_store * es_lo);
      // row padding of the low-precision copy: never written by the fold, read with zero weights
      if (e1 == hipSuccess && es_lo) e1 = hipMemsetAsync(B->d_plo, 0, (size_t)(B->pn_store * es_lo), s);
      if (e1 != hipSuccess) {
        release(B->d_pAhat); release(B->d_prc); release(B->d_plo);
        return bfail(B, ELMFB_E_NOMEM, std::string("patch storage: ") + hipGetErrorString(e1));
      }
    }
    double *G = nullptr, *Wk = nullptr;
    hipError_t e1 = balloc(B, &G, B->pn_scratch * 8);
    if (e1 == hipSuccess && B->pkmax > kBatchMaxK) e1 = balloc(B, &Wk, B->pn_scratch * 8);
    if (e1 != hipSuccess) {
      bfree(B, G);
      return bfail(B, ELMFB_E_NOMEM, std::string("patch Gram scratch: ") + hipGetErrorString(e1));
    }
    // patches of M in FP64, then per chunk their Gram blocks and factors, then M R^{-1} in place
    if (e == hipSuccess)
      e = launch_bt_expand(B->d_geos, B->d_pblocks, B->d_pruns, (int64_t)B->pruns.size(),
                           B->d_blocks, B->d_pmem, B->d_pmoff, B->d_A, B->d_pAhat, s);
    for (size_t c = 0; c + 1 < B->pchunk_blk.size() && e == hipSuccess; ++c) {
      const int64_t b0 = B->pchunk_blk[c], b1 = B->pchunk_blk[c + 1];
      const int64_t t0 = B->pchunk_task[c], t1 = B->pchunk_task[c + 1];
      e = launch_bt_gram_diag(B->d_pblocks, B->d_ptasks + t0, t1 - t0, B->pkmax > kBatchMaxK,
                              B->d_pAhat, B->d_pgoff, G, s);
      if (e == hipSuccess) {
        if (B->pkmax <= kBatchMaxK)
          e = launch_bt_bj_factor(B->d_pblocks, (int)b0, b1 - b0, G, B->d_pgoff, B->d_pfoff,
                                  B->pkmax, shift, B->d_prc, B->d_flag, s);
        else
          e = launch_bt_bj_factor_blocked(B->d_pblocks, (int)b0, b1 - b0, G, Wk, B->d_pgoff,
                                          B->d_pfoff, shift, B->d_prc, B->d_flag, s);
      }
    }
    if (e == hipSuccess)
      e = launch_bt_fold(B->lo_prec, false, B->pkmax, B->d_pblocks, B->d_pftiles,
                         (int64_t)B->pftiles.size(), B->d_pAhat, B->d_prc, B->d_pfoff, B->d_pAhat,
                         B->d_plo, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&nfail, B->d_flag, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    bfree(B, G);
    bfree(B, Wk);
    BHIP(B, e);
    B->lo_hat = false;   // the low-precision copy of M itself is untouched
  }
  if (n_fallback_host) *n_fallback_host = nfail;
  B->patch = patch;
  B->bj_ready = true;
  // an identity fallback leaves that block's columns unscaled; their FP16 rounding may overflow
  B->lo_unsafe = B->lo_prec == ELMFB_FP16 && nfail > 0;
  return ELMFB_OK;
}

elmfb_status elmfb_batch_patch_info(elmfb_batch B, int32_t* patch_host, int64_t* n_blocks_host,
                                    int64_t* n_entries_host, int32_t* perm_host) {
  if (!B) return bfail(B, ELMFB_E_INVALID, "NULL batch");
  const bool pt = B->patch > 1 && B->patch_planned == B->patch;
  if (patch_host) *patch_host = B->patch;
  if (n_blocks_host) *n_blocks_host = pt ? (int64_t)B->pblocks.size() : (int64_t)B->blocks.size();
  if (n_entries_host) *n_entries_host = pt ? B->pn_dense : B->nnz;
  if (perm_host) {
    for (int64_t q = 0; q < B->n_phi; ++q) perm_host[q] = pt ? B->pperm[q] : (int32_t)q;
  }
  return ELMFB_OK;
}

elmfb_status elmfb_batch_autotune(elmfb_batch B, int32_t prec, int32_t reps, double* ms_host,
                                  int32_t* chosen_host, void* stream) {
  if (!B) return bfail(B, ELMFB_E_INVALID, "NULL batch");
  if (!B->assembled) return bfail(B, ELMFB_E_STATE, "autotune before assemble");
  if (prec != ELMFB_FP64 && prec != B->lo_prec)
    return bfail(B, ELMFB_E_INVALID, "no stored matrix copy of that precision");
  if (reps < 1 || reps > 1000) return bfail(B, ELMFB_E_INVALID, "reps must be in 1..1000");
  hipStream_t s = (hipStream_t)stream;
  const int R = B->R;
  const TimedTarget T = timed_target(B, prec);
  const BtLayout& L = T.L;
  const void* A = T.A;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  BHIP(B, hipEventCreate(&t0));
  BHIP(B, hipEventCreate(&t1));
  // u = 1 on every row and right-hand side (timing input only)
  std::vector<double> ones((size_t)B->n_rows * R, 1.0);
  hipError_t e = hipMemcpyAsync(B->d_u, ones.data(), ones.size() * 8, hipMemcpyHostToDevice, s);
  double best = 1e300;
  int best_tp = 32;
  for (int c = 0; c < 3 && e == hipSuccess; ++c) {
    const int tp = kBtTileChoices[c];
    double ms = -1.0;
    if (!(prec == ELMFB_FP64 && tp == 64)) {
      e = launch_bt_rmvb(prec, tp, L.geos, L.insts, L.blocks, L.slices, L.ns, A, B->d_u, R,
                         nullptr, COL_STORE, B->d_w, B->d_red_c, s);
      if (e == hipSuccess) e = hipEventRecord(t0, s);
      for (int r = 0; r < reps && e == hipSuccess; ++r)
        e = launch_bt_rmvb(prec, tp, L.geos, L.insts, L.blocks, L.slices, L.ns, A, B->d_u, R,
                           nullptr, COL_STORE, B->d_w, B->d_red_c, s);
      if (e == hipSuccess) e = hipEventRecord(t1, s);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float f = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&f, t0, t1);
      ms = (double)f / reps;
      if (e == hipSuccess && ms < best) {
        best = ms;
        best_tp = tp;
      }
    }
    if (ms_host) ms_host[c] = ms;
  }
  hipEventDestroy(t0);
  hipEventDestroy(t1);
  BHIP(B, e);
  B->tp[prec_index(prec)] = best_tp;
  B->tuned[prec_index(prec)] = true;
  if (chosen_host) *chosen_host = best_tp;
  return ELMFB_OK;
}

elmfb_status elmfb_batch_time_kernels(elmfb_batch B, int32_t prec, int32_t reps, double* ms_host,
                                      void* stream) {
  if (!B || !ms_host) return bfail(B, ELMFB_E_INVALID, "NULL argument");
  if (!B->assembled) return bfail(B, ELMFB_E_STATE, "time_kernels before assemble");
  if (prec != ELMFB_FP64 && prec != B->lo_prec)
    return bfail(B, ELMFB_E_INVALID, "no stored matrix copy of that precision");
  if (reps < 1 || reps > 1000) return bfail(B, ELMFB_E_INVALID, "reps must be in 1..1000");
  hipStream_t s = (hipStream_t)stream;
  const int R = B->R;
  const TimedTarget T = timed_target(B, prec);
  const BtLayout& L = T.L;
  const void* A = T.A;
  // V = 1 and U = 1 on every column, row and right-hand side (timing inputs only); the row
  // gather writes its rows into the row-sized work vector U, which the M^T U timing then reads
  std::vector<double> ones((size_t)std::max(B->n_rows, B->n_phi) * R, 1.0);
  BHIP(B, hipMemcpyAsync(B->d_v, ones.data(), (size_t)B->n_phi * R * 8, hipMemcpyHostToDevice, s));
  BHIP(B, hipMemcpyAsync(B->d_u, ones.data(), (size_t)B->n_rows * R * 8, hipMemcpyHostToDevice, s));
  hipEvent_t ev[4];
  for (int i = 0; i < 4; ++i) BHIP(B, hipEventCreate(&ev[i]));
  hipError_t e = hipEventRecord(ev[0], s);
  for (int r = 0; r < reps && e == hipSuccess; ++r)
    e = launch_bt_mvb(prec, L.blocks, L.mv_runs, L.n_mv, L.kmax, A, B->d_v, R, nullptr,
                      B->d_tpart, s, B->fa[prec_index(prec)]);
  if (e == hipSuccess) e = hipEventRecord(ev[1], s);
  for (int r = 0; r < reps && e == hipSuccess; ++r)
    e = launch_bt_gather(L.geos, L.insts, L.blocks, L.cov, B->d_rtiles, (int64_t)B->rtiles.size(),
                         B->d_tpart, ROW_STORE_SQ, R, B->d_u, nullptr, nullptr, B->d_red_r, s,
                         B->rpt);
  if (e == hipSuccess) e = hipEventRecord(ev[2], s);
  for (int r = 0; r < reps && e == hipSuccess; ++r)
    e = launch_bt_rmvb(prec, B->tp[prec_index(prec)], L.geos, L.insts, L.blocks, L.slices, L.ns, A,
                       B->d_u, R, nullptr, COL_STORE_SQ, B->d_w, B->d_red_c, s);
  if (e == hipSuccess) e = hipEventRecord(ev[3], s);
  if (e == hipSuccess) e = hipEventSynchronize(ev[3]);
  float t[3] = {0.f, 0.f, 0.f};
  for (int i = 0; i < 3 && e == hipSuccess; ++i) e = hipEventElapsedTime(&t[i], ev[i], ev[i + 1]);
  for (int i = 0; i < 4; ++i) hipEventDestroy(ev[i]);
  BHIP(B, e);
  for (int i = 0; i < 3; ++i) ms_host[i] = (double)t[i] / reps;
  return ELMFB_OK;
}

namespace {

// Shapes chosen by elmfb_batch_tune, kept for the process and keyed by (operator, precision,
// largest K in 16s, stored entries in powers of two, right-hand sides, patch size of the factors
// whose folded matrix is timed): a later batch of the same class takes them without timing.
struct ShapeKey {
  int op, prec, kclass, sclass, rhs, patch;
  bool operator<(const ShapeKey& o) const {
    if (patch != o.patch) return patch < o.patch;
    if (op != o.op) return op < o.op;
    if (prec != o.prec) return prec < o.prec;
    if (kclass != o.kclass) return kclass < o.kclass;
    if (sclass != o.sclass) return sclass < o.sclass;
    return rhs < o.rhs;
  }
};
std::mutex g_shape_mu;
std::map<ShapeKey, elmfb_batch_shape> g_shapes;

ShapeKey shape_key(elmfb_batch B, int prec) {
  int kmax = 0;
  for (const Geo& g : B->geos) kmax = std::max(kmax, (int)g.K);
  int sc = 0;
  for (int64_t n = B->nnz; n > 1; n >>= 1) ++sc;
  const int pt = B->patch > 1 && B->bj_ready ? B->patch : 1;
  return ShapeKey{B->geos.empty() ? 0 : B->geos[0].op, prec, (kmax + 15) / 16, sc, B->R, pt};
}

bool valid_shape(int prec, const elmfb_batch_shape& sh) {
  const bool tile = sh.rmvb_tile == 16 || sh.rmvb_tile == 32 ||
                    (sh.rmvb_tile == 64 && prec != ELMFB_FP64);
  return tile && (sh.mvb_ahead == 4 || sh.mvb_ahead == 8 || sh.mvb_ahead == 16) &&
         (sh.gather_rows == 1 || sh.gather_rows == 2);
}

}  // namespace

elmfb_status elmfb_batch_tune(elmfb_batch B, int32_t prec, int32_t reps, int32_t use_cache,
                              elmfb_batch_shape* out, void* stream) {
  if (!B) return bfail(B, ELMFB_E_INVALID, "NULL batch");
  if (!B->assembled) return bfail(B, ELMFB_E_STATE, "tune before assemble");
  if (prec != ELMFB_FP64 && prec != B->lo_prec)
    return bfail(B, ELMFB_E_INVALID, "no stored matrix copy of that precision");
  if (reps < 1 || reps > 1000) return bfail(B, ELMFB_E_INVALID, "reps must be in 1..1000");
  const ShapeKey key = shape_key(B, prec);
  elmfb_batch_shape sh{};
  for (int i = 0; i < 3; ++i) sh.ms_rmvb[i] = sh.ms_mvb[i] = -1.0;
  sh.ms_gather[0] = sh.ms_gather[1] = -1.0;
  if (use_cache) {
    std::lock_guard<std::mutex> lock(g_shape_mu);
    auto it = g_shapes.find(key);
    if (it != g_shapes.end()) {
      sh = it->second;
      sh.from_cache = 1;
    }
  }
  if (!sh.from_cache) {
    hipStream_t s = (hipStream_t)stream;
    const int R = B->R;
    const TimedTarget T = timed_target(B, prec);
    const BtLayout& L = T.L;
    const void* A = T.A;
    std::vector<double> ones((size_t)std::max(B->n_rows, B->n_phi) * R, 1.0);
    BHIP(B, hipMemcpyAsync(B->d_v, ones.data(), (size_t)B->n_phi * R * 8, hipMemcpyHostToDevice, s));
    BHIP(B, hipMemcpyAsync(B->d_u, ones.data(), (size_t)B->n_rows * R * 8, hipMemcpyHostToDevice, s));
    hipEvent_t t0 = nullptr, t1 = nullptr;
    BHIP(B, hipEventCreate(&t0));
    BHIP(B, hipEventCreate(&t1));
    hipError_t e = hipSuccess;
    // one warm-up launch, then `reps` timed launches of a candidate
    auto timed = [&](auto&& launch) -> double {
      if (e == hipSuccess) e = launch();
      if (e == hipSuccess) e = hipEventRecord(t0, s);
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
      if (e == hipSuccess) e = hipEventRecord(t1, s);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float f = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&f, t0, t1);
      return e == hipSuccess ? (double)f / reps : -1.0;
    };
    const int tiles[3] = {16, 32, 64}, aheads[3] = {4, 8, 16};
    double best = 1e300;
    for (int c = 0; c < 3; ++c) {
      if (prec == ELMFB_FP64 && tiles[c] == 64) continue;
      sh.ms_rmvb[c] = timed([&] {
        return launch_bt_rmvb(prec, tiles[c], L.geos, L.insts, L.blocks, L.slices, L.ns, A,
                              B->d_u, R, nullptr, COL_STORE, B->d_w, B->d_red_c, s);
      });
      if (sh.ms_rmvb[c] >= 0 && sh.ms_rmvb[c] < best) { best = sh.ms_rmvb[c]; sh.rmvb_tile = tiles[c]; }
    }
    best = 1e300;
    for (int c = 0; c < 3; ++c) {
      sh.ms_mvb[c] = timed([&] {
        return launch_bt_mvb(prec, L.blocks, L.mv_runs, L.n_mv, L.kmax, A, B->d_v, R, nullptr,
                             B->d_tpart, s, aheads[c]);
      });
      if (sh.ms_mvb[c] >= 0 && sh.ms_mvb[c] < best) { best = sh.ms_mvb[c]; sh.mvb_ahead = aheads[c]; }
    }
    best = 1e300;
    for (int c = 0; c < 2; ++c) {
      sh.ms_gather[c] = timed([&] {
        return launch_bt_gather(L.geos, L.insts, L.blocks, L.cov, B->d_rtiles,
                                (int64_t)B->rtiles.size(), B->d_tpart, ROW_STORE_SQ, R, B->d_u,
                                nullptr, nullptr, B->d_red_r, s, c + 1);
      });
      if (sh.ms_gather[c] >= 0 && sh.ms_gather[c] < best) { best = sh.ms_gather[c]; sh.gather_rows = c + 1; }
    }
    hipEventDestroy(t0);
    hipEventDestroy(t1);
    BHIP(B, e);
    std::lock_guard<std::mutex> lock(g_shape_mu);
    g_shapes[key] = sh;
  }
  const int pi = prec_index(prec);
  B->tp[pi] = sh.rmvb_tile;
  B->fa[pi] = sh.mvb_ahead;
  B->rpt = sh.gather_rows;
  B->tuned[pi] = true;
  if (out) *out = sh;
  return ELMFB_OK;
}

elmfb_status elmfb_batch_set_shape(elmfb_batch B, int32_t prec, const elmfb_batch_shape* shape) {
  if (!B || !shape) return bfail(B, ELMFB_E_INVALID, "NULL argument");
  if (prec != ELMFB_FP64 && prec != ELMFB_FP32 && prec != ELMFB_BF16 && prec != ELMFB_FP16)
    return bfail(B, ELMFB_E_INVALID, "bad precision");
  if (!valid_shape(prec, *shape))
    return bfail(B, ELMFB_E_INVALID,
                 "tile 16/32/64 (not 64 in FP64), ahead 4/8/16 and gather rows 1/2 required");
  const int pi = prec_index(prec);
  B->tp[pi] = shape->rmvb_tile;
  B->fa[pi] = shape->mvb_ahead;
  B->rpt = shape->gather_rows;
  return ELMFB_OK;
}

elmfb_status elmfb_batch_set_tile(elmfb_batch B, int32_t prec, int32_t tile) {
  if (!B) return bfail(B, ELMFB_E_INVALID, "NULL batch");
  if (prec != ELMFB_FP64 && prec != ELMFB_FP32 && prec != ELMFB_BF16 && prec != ELMFB_FP16)
    return bfail(B, ELMFB_E_INVALID, "bad precision");
  if (!(tile == 16 || tile == 32 || (tile == 64 && prec != ELMFB_FP64)))
    return bfail(B, ELMFB_E_INVALID, "tile must be 16, 32 or (not FP64) 64");
  B->tp[prec_index(prec)] = tile;
  return ELMFB_OK;
}

elmfb_status elmfb_batch_set_coords(elmfb_batch B, int32_t preconditioned) {
  if (!B) return bfail(B, ELMFB_E_INVALID, "NULL batch");
  if (preconditioned && B->patch > 1)
    return bfail(B, ELMFB_E_UNSUPPORTED, "block-Jacobi coordinates are per subdomain (patch 1)");
  B->coords_y = preconditioned != 0;
  return ELMFB_OK;
}

elmfb_status elmfb_batch_from_coords(elmfb_batch B, const double* y_dev, double* x_dev,
                                     void* stream) {
  if (!B || !y_dev || !x_dev) return bfail(B, ELMFB_E_INVALID, "NULL argument");
  if (!B->bj_ready) return bfail(B, ELMFB_E_STATE, "no block-Jacobi factors");
  if (B->patch > 1)
    return bfail(B, ELMFB_E_UNSUPPORTED, "block-Jacobi coordinates are per subdomain (patch 1)");
  hipStream_t s = (hipStream_t)stream;
  const int R = B->R;
  BHIP(B, launch_bt_pack(B->d_insts, B->d_nphis, B->n, R, B->n_phi, y_dev, B->d_w, 1, 1, s));
  BHIP(B, launch_bt_bj_recover(B->d_blocks, (int64_t)B->blocks.size(), B->d_rc, B->d_foff,
                               nullptr, R, B->d_w, nullptr, B->d_v, s));
  BHIP(B, launch_bt_pack(B->d_insts, B->d_nphis, B->n, R, B->n_phi, B->d_v, x_dev, 0, 1, s));
  return ELMFB_OK;
}

elmfb_status elmfb_batch_solve(elmfb_batch B, const elmfb_solve_opts* opts, double* coef_dev,
                               elmfb_solve_info* info, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!B || !opts || !coef_dev) return bfail(B, ELMFB_E_INVALID, "NULL argument");
  if (!B->assembled) return bfail(B, ELMFB_E_STATE, "solve before assemble");
  const bool mixed = opts->method == ELMFB_MIXED_IR;
  if (opts->method != ELMFB_LSQR && !mixed)
    return bfail(B, ELMFB_E_UNSUPPORTED, "batches solve with LSQR or MIXED_IR");
  if (opts->n_check)
    return bfail(B, ELMFB_E_UNSUPPORTED, "batched solves take no check points");
  if (B->coords_y && !opts->precond)
    return bfail(B, ELMFB_E_STATE, "block-Jacobi coordinates need a preconditioned solve");
  if (opts->precond && !B->bj_ready)
    return bfail(B, ELMFB_E_STATE, "precond requested before elmfb_batch_precondition");
  if (mixed && B->lo_prec == ELMFB_FP64)
    return bfail(B, ELMFB_E_INVALID, "MIXED_IR needs a store_prec copy (FP32, BF16 or FP16)");
  if (mixed && B->lo_prec == ELMFB_FP16 && (!opts->precond || B->lo_unsafe))
    return bfail(B, ELMFB_E_UNSUPPORTED,
                 "FP16 inner solves run on the folded copy of M R^-1: precondition (no identity "
                 "fallback) and set precond");
  if (mixed && !opts->precond && B->lo_hat)
    return bfail(B, ELMFB_E_STATE,
                 "the low-precision copy holds the preconditioned matrix: assemble again for "
                 "unpreconditioned refinement");
  if (opts->iter_lim < 0 || opts->check_every < 1 || opts->check_every > 100000 ||
      !(opts->atol >= 0.0) || !(opts->btol >= 0.0) ||
      (mixed && (opts->inner_iters < 1 || opts->outer_lim < 0)))
    return bfail(B, ELMFB_E_INVALID, "bad solve options");
  const int n = B->n, R = B->R;
  const bool bj = opts->precond != 0;
  const BtLayout L = layout_of(B, bj);
  const bool warm = opts->x0_dev != nullptr;
  if (warm && !B->d_x0) {
    hipError_t e1 = balloc(B, &B->d_x0, B->n_phi * R * 8);
    hipError_t e2 = e1 == hipSuccess ? balloc(B, &B->d_h0, B->n_rows * R * 8) : e1;
    if (e2 != hipSuccess) {
      bfree(B, B->d_x0);
      B->d_x0 = nullptr;
      return bfail(B, ELMFB_E_NOMEM, std::string("warm-start storage: ") + hipGetErrorString(e2));
    }
    B->bytes += (B->n_phi + B->n_rows) * R * 8;
  }
  hipStream_t caller = (hipStream_t)stream;
  hipStream_t s = B->stream;
  BHIP(B, hipEventRecord(B->ev_in, caller));
  BHIP(B, hipStreamWaitEvent(s, B->ev_in, 0));
  // ||h|| partials (d_red_h); with a warm start the solve runs on h0 = h - M x0 (FP64 M)
  BHIP(B, bt_residual(B, nullptr, false, s));
  BHIP(B, hipMemcpyAsync(B->d_red_h, B->d_red_r, B->rtiles.size() * kMaxRhs * 8,
                         hipMemcpyDeviceToDevice, s));
  const double* rhs = B->d_h;
  if (warm) {
    BHIP(B, launch_bt_pack(B->d_insts, B->d_nphis, n, R, B->n_phi, opts->x0_dev, B->d_x0, 1, 1, s));
    BHIP(B, bt_residual(B, B->d_x0, B->coords_y, s));   // h - M x0, or h - (M R^{-1}) y0
    BHIP(B, hipMemcpyAsync(B->d_h0, B->d_u, (size_t)(B->n_rows * R * 8), hipMemcpyDeviceToDevice,
                           s));
    rhs = B->d_h0;
  }
  if (!mixed) {
    // u holds the right-hand side (h, or h - M x0) and d_red_r its partials
    BHIP(B, bt_lsqr_start(B, ELMFB_FP64, bj, opts->atol, opts->btol, opts->iter_lim, nullptr, 0.0,
                          s, B->d_red_h));
    const elmfb_status st = bt_run(B, ELMFB_FP64, bj, opts->check_every, opts->use_graph != 0, s);
    if (st != ELMFB_OK) return st;
    if (bj && !B->coords_y)
      BHIP(B, launch_bt_bj_recover(L.blocks, L.nb, factors_of(B), foff_of(B), perm_of(B), R,
                                   B->d_x, warm ? B->d_x0 : nullptr, B->d_c, s));
    else if (warm)
      BHIP(B, launch_bt_recover_plain(B->n_phi * R, B->d_x, B->d_x0, B->d_c, s));
    else
      BHIP(B, hipMemcpyAsync(B->d_c, B->d_x, (size_t)(B->n_phi * R * 8), hipMemcpyDeviceToDevice, s));
  } else {
    // FP64 refinement: r = rhs - A c, inner LSQR on the stored low-precision copy, c += d
    const int lo = B->lo_prec;
    BHIP(B, launch_bt_outer_check(B->d_outer, B->d_state, L.insts, n, R, B->d_red_h, nullptr,
                                  0.0, 1, opts->btol, opts->outer_lim, s));
    if (warm)   // the residual of x0 (in d_red_r) may already meet the target
      BHIP(B, launch_bt_outer_check(B->d_outer, B->d_state, L.insts, n, R, B->d_red_r,
                                    nullptr, 0.0, 2, opts->btol, opts->outer_lim, s));
    BHIP(B, hipMemsetAsync(B->d_c, 0, (size_t)(B->n_phi * R * 8), s));
    for (;;) {
      int32_t active = 0;
      BHIP(B, launch_bt_count_outer(B->d_outer, n * R, B->d_count, s));
      BHIP(B, hipMemcpyAsync(&active, B->d_count, 4, hipMemcpyDeviceToHost, s));
      BHIP(B, hipStreamSynchronize(s));
      if (active == 0) break;
      BHIP(B, bt_lsqr_start(B, lo, bj, 0.0, 0.0, opts->inner_iters, B->d_outer, 0.5, s));
      const elmfb_status st = bt_run(B, lo, bj, opts->check_every, opts->use_graph != 0, s);
      if (st != ELMFB_OK) return st;
      // c += d (c in preconditioned coordinates with block-Jacobi)
      BHIP(B, launch_bt_axpy(B->n_phi * R, B->d_x, B->d_c, s));
      BHIP(B, bt_residual(B, B->d_c, bj, s, rhs));
      const double* red_a = nullptr;
      if (opts->atol > 0.0) {   // ||A^T r|| per block with the FP64 matrix (v is free here)
        BHIP(B, launch_bt_rmvb(ELMFB_FP64, B->tp[0], L.geos, L.insts, L.blocks, L.slices, L.ns,
                               matrix_of(B, ELMFB_FP64, bj), B->d_u, R, nullptr, COL_STORE_SQ,
                               B->d_v, B->d_red_c, s));
        red_a = B->d_red_c;
      }
      BHIP(B, launch_bt_outer_check(B->d_outer, B->d_state, L.insts, n, R, B->d_red_r, red_a,
                                    opts->atol, 0, opts->btol, opts->outer_lim, s));
    }
  }
  const double* fin = B->d_c;
  if (mixed) {   // coefficients x = x0 + R^{-1} c (or x0 + c; y = y0 + c in block-Jacobi coordinates)
    if (bj && !B->coords_y)
      BHIP(B, launch_bt_bj_recover(L.blocks, L.nb, factors_of(B), foff_of(B), perm_of(B), R,
                                   B->d_c, warm ? B->d_x0 : nullptr, B->d_x, s));
    else
      BHIP(B, launch_bt_recover_plain(B->n_phi * R, B->d_c, warm ? B->d_x0 : nullptr, B->d_x, s));
    fin = B->d_x;
  }
  BHIP(B, launch_bt_pack(B->d_insts, B->d_nphis, n, R, B->n_phi, fin, coef_dev, 0, 1, s));
  BHIP(B, hipEventRecord(B->ev_out, s));
  BHIP(B, hipStreamWaitEvent(caller, B->ev_out, 0));
  if (info) {
    std::vector<SolveState> st((size_t)n * R);
    std::vector<BtOuter> ot(mixed ? (size_t)n * R : 0);
    BHIP(B, hipMemcpyAsync(st.data(), B->d_state, st.size() * sizeof(SolveState),
                           hipMemcpyDeviceToHost, s));
    if (mixed)
      BHIP(B, hipMemcpyAsync(ot.data(), B->d_outer, ot.size() * sizeof(BtOuter),
                             hipMemcpyDeviceToHost, s));
    BHIP(B, hipStreamSynchronize(s));
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (size_t k = 0; k < st.size(); ++k) {
      info[k] = elmfb_solve_info{};
      info[k].istop = mixed ? ot[k].istop : st[k].istop;
      info[k].iters = mixed ? ot[k].iters : st[k].itn;
      info[k].outer_iters = mixed ? ot[k].outer : 0;
      info[k].rnorm = mixed ? ot[k].rnorm : st[k].rnorm;
      info[k].arnorm = st[k].arnorm;
      info[k].anorm = st[k].anorm;
      info[k].xnorm = st[k].xnorm;
      info[k].rel_l2 = -1.0;
      info[k].ms_solve = ms;
    }
  }
  return ELMFB_OK;
}

void elmfb_batch_destroy(elmfb_batch B) {
  if (!B) return;
  if (B->stream) hipStreamSynchronize(B->stream);
  brelease(B);
  delete B;
}

const char* elmfb_batch_last_error(elmfb_batch B) {
  if (B) return B->err.c_str();
  return g_batch_error.c_str();
}

}  // extern "C"
