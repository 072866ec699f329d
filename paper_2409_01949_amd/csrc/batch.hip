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
#include <string>
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
  std::vector<Tile> tiles, chunks;
  std::vector<int32_t> cstart, cov;
  std::vector<BSeg> segs;
  std::vector<RowTile> rtiles;
  std::vector<ColTile> ctiles;
  int64_t n_rows = 0, n_phi = 0, nnz = 0, n_bp = 0, n_tab = 0, bytes = 0;

  std::vector<void*> allocs;
  Geo* d_geos = nullptr;
  InstInfo* d_insts = nullptr;
  int64_t *d_nrows = nullptr, *d_nphis = nullptr;
  DevBlock* d_blocks = nullptr;
  Tile *d_tiles = nullptr, *d_chunks = nullptr;
  int32_t *d_cstart = nullptr, *d_cov = nullptr;
  BSeg* d_segs = nullptr;
  RowTile* d_rtiles = nullptr;
  ColTile* d_ctiles = nullptr;
  double *d_tab = nullptr, *d_W = nullptr, *d_b = nullptr, *d_A = nullptr;
  void* d_A_lo = nullptr;
  double *d_h = nullptr, *d_u = nullptr, *d_v = nullptr, *d_w = nullptr, *d_x = nullptr;
  double *d_tpart = nullptr, *d_part = nullptr;
  double *d_red_r = nullptr, *d_red_r2 = nullptr, *d_red_c = nullptr, *d_red_c2 = nullptr;
  SolveState* d_state = nullptr;
  int32_t *d_flag = nullptr, *d_count = nullptr;
  bool assembled = false;
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::map<int, hipGraphExec_t> graphs;
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

std::string plan_batch(elmfb_batch B, const elmfb_problem_desc* descs) {
  int64_t row_off = 0, col_off = 0, a_off = 0, p_off = 0;
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
    B->insts.push_back(I);
    B->nrows.push_back(g.n_rows);
    B->nphis.push_back(g.n_phi);
    for (size_t b = 0; b < hp.blocks.size(); ++b) {
      DevBlock D = hp.blocks[b];
      D.a_off += a_off;
      D.p_off += p_off;
      D.q0 += (int32_t)col_off;
      D.tabx += tab_off;
      D.taby += tab_off;
      D.inst = i;
      const int gb = blk_off + (int)b;
      B->cstart.push_back((int32_t)B->chunks.size());
      for (int64_t p0 = 0; p0 < D.n; p0 += kBChunkPts) B->chunks.push_back(Tile{gb, (int32_t)p0});
      B->blocks.push_back(D);
    }
    for (const Tile& t : hp.tiles) B->tiles.push_back(Tile{t.blk + blk_off, t.p0});
    for (const AxisSeg& s : hp.segs) {
      AxisSeg s2 = s;
      s2.tab_off += tab_off;
      B->segs.push_back(BSeg{s2, i, 0});
    }
    B->cov.insert(B->cov.end(), hp.cov.begin(), hp.cov.end());
    row_off += g.n_rows;
    col_off += g.n_phi;
    a_off += hp.nnz;
    p_off += hp.n_block_points;
    blk_off += (int32_t)hp.blocks.size();
    tab_off += (int32_t)hp.n_tab;
    cov_off += (int32_t)hp.cov.size();
    if (row_off > ((int64_t)1 << 31) || col_off > ((int64_t)1 << 31)) return "batch too large";
  }
  B->cstart.push_back((int32_t)B->chunks.size());
  B->n_rows = row_off;
  B->n_phi = col_off;
  B->nnz = a_off;
  B->n_bp = p_off;
  B->n_tab = tab_off;
  return "";
}

hipError_t bt_iteration(elmfb_batch B, hipStream_t s) {
  const int n = B->n, R = B->R;
  hipError_t e;
  if ((e = launch_bt_mv(ELMFB_FP64, B->d_geos, B->d_blocks, B->d_tiles, (int64_t)B->tiles.size(),
                        B->d_A, B->d_v, R, B->d_state, B->d_tpart, s)))
    return e;
  if ((e = launch_bt_gather(B->d_geos, B->d_insts, B->d_blocks, B->d_cov, B->d_rtiles,
                            (int64_t)B->rtiles.size(), B->d_tpart, ROW_LSQR_U, R, B->d_u, nullptr,
                            B->d_state, B->d_red_r, s)))
    return e;
  if ((e = launch_bt_lsqr_beta(B->d_state, B->d_insts, n, R, B->d_red_r, s))) return e;
  if ((e = launch_bt_rmv(ELMFB_FP64, B->d_geos, B->d_insts, B->d_blocks, B->d_chunks,
                         (int64_t)B->chunks.size(), B->d_A, B->d_u, R, B->d_state, B->d_part, s)))
    return e;
  if ((e = launch_bt_finish(B->d_geos, B->d_insts, B->d_ctiles, (int64_t)B->ctiles.size(),
                            B->d_cstart, B->d_part, COL_LSQR_V, R, B->d_v, B->d_state, B->d_red_c,
                            s)))
    return e;
  if ((e = launch_bt_lsqr_alpha(B->d_state, B->d_insts, n, R, B->d_red_c, s))) return e;
  if ((e = launch_bt_update(B->d_geos, B->d_insts, B->d_ctiles, (int64_t)B->ctiles.size(), R,
                            B->d_x, B->d_w, B->d_v, B->d_state, B->d_red_c2, s)))
    return e;
  return launch_bt_lsqr_stop(B->d_state, B->d_insts, n, R, B->d_red_c2, s);
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
  const int64_t es_lo = B->lo_prec == ELMFB_FP32 ? 4 : (B->lo_prec == ELMFB_BF16 ? 2 : 0);
  int64_t bytes = B->nnz * (8 + es_lo) + B->n_bp * R * 8 +
                  (int64_t)B->chunks.size() * kBatchMaxK * R * 8 + B->n_rows * R * 8 * 2 +
                  B->n_phi * R * 8 * 3 + B->n_phi * 24 + B->n_tab * 24 +
                  (int64_t)(B->rtiles.size() + B->ctiles.size()) * 2 * kMaxRhs * 8 +
                  (int64_t)B->blocks.size() * sizeof(DevBlock) +
                  (int64_t)(B->tiles.size() + B->chunks.size()) * sizeof(Tile);
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
  BALLOC(B->d_blocks, (int64_t)B->blocks.size() * sizeof(DevBlock));
  BALLOC(B->d_tiles, (int64_t)B->tiles.size() * sizeof(Tile));
  BALLOC(B->d_chunks, (int64_t)B->chunks.size() * sizeof(Tile));
  BALLOC(B->d_cstart, (int64_t)B->cstart.size() * 4);
  BALLOC(B->d_cov, (int64_t)B->cov.size() * 4);
  BALLOC(B->d_segs, (int64_t)B->segs.size() * sizeof(BSeg));
  BALLOC(B->d_rtiles, (int64_t)B->rtiles.size() * sizeof(RowTile));
  BALLOC(B->d_ctiles, (int64_t)B->ctiles.size() * sizeof(ColTile));
  BALLOC(B->d_tab, B->n_tab * 24);
  BALLOC(B->d_W, B->n_phi * 16);
  BALLOC(B->d_b, B->n_phi * 8);
  BALLOC(B->d_A, B->nnz * 8);
  if (es_lo) BALLOC(B->d_A_lo, B->nnz * es_lo);
  BALLOC(B->d_h, B->n_rows * R * 8);
  BALLOC(B->d_u, B->n_rows * R * 8);
  BALLOC(B->d_v, B->n_phi * R * 8);
  BALLOC(B->d_w, B->n_phi * R * 8);
  BALLOC(B->d_x, B->n_phi * R * 8);
  BALLOC(B->d_tpart, B->n_bp * R * 8);
  BALLOC(B->d_part, (int64_t)B->chunks.size() * kBatchMaxK * R * 8);
  BALLOC(B->d_red_r, (int64_t)B->rtiles.size() * kMaxRhs * 8);
  BALLOC(B->d_red_r2, (int64_t)B->rtiles.size() * kMaxRhs * 8);
  BALLOC(B->d_red_c, (int64_t)B->ctiles.size() * kMaxRhs * 8);
  BALLOC(B->d_red_c2, (int64_t)B->ctiles.size() * kMaxRhs * 8);
  BALLOC(B->d_state, (int64_t)n * R * sizeof(SolveState));
  BALLOC(B->d_flag, 64);
  BALLOC(B->d_count, 64);
#undef BALLOC
  // features, W padded to two columns, instance by instance
  std::vector<double> W2((size_t)B->n_phi * 2, 0.0), bb((size_t)B->n_phi, 0.0);
  for (int i = 0; i < n; ++i) {
    const elmfb_problem_desc& d = descs[i];
    const int64_t c0 = B->insts[i].col_off;
    for (int64_t q = 0; q < B->nphis[i]; ++q) {
      for (int a = 0; a < d.dim; ++a) W2[2 * (c0 + q) + a] = d.W_host[q * d.dim + a];
      bb[c0 + q] = d.b_host[q];
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
  up(B->d_tiles, B->tiles.data(), B->tiles.size() * sizeof(Tile));
  up(B->d_chunks, B->chunks.data(), B->chunks.size() * sizeof(Tile));
  up(B->d_cstart, B->cstart.data(), B->cstart.size() * 4);
  up(B->d_cov, B->cov.data(), B->cov.size() * 4);
  up(B->d_segs, B->segs.data(), B->segs.size() * sizeof(BSeg));
  up(B->d_rtiles, B->rtiles.data(), B->rtiles.size() * sizeof(RowTile));
  up(B->d_ctiles, B->ctiles.data(), B->ctiles.size() * sizeof(ColTile));
  up(B->d_W, W2.data(), W2.size() * 8);
  up(B->d_b, bb.data(), bb.size() * 8);
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
  }
  return ELMFB_OK;
}

elmfb_status elmfb_batch_assemble(elmfb_batch B, const double* f_dev, void* stream) {
  if (!B || !f_dev) return bfail(B, ELMFB_E_INVALID, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  BHIP(B, hipMemsetAsync(B->d_flag, 0, 4, s));
  BHIP(B, launch_bt_rhs(B->d_geos, B->d_insts, B->d_rtiles, (int64_t)B->rtiles.size(), B->R,
                        f_dev, B->d_h, B->d_flag, s));
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
  BHIP(B, launch_bt_mv(ELMFB_FP64, B->d_geos, B->d_blocks, B->d_tiles, (int64_t)B->tiles.size(),
                       B->d_A, B->d_w, R, nullptr, B->d_tpart, s));
  BHIP(B, launch_bt_gather(B->d_geos, B->d_insts, B->d_blocks, B->d_cov, B->d_rtiles,
                           (int64_t)B->rtiles.size(), B->d_tpart, ROW_STORE, R, B->d_u, nullptr,
                           nullptr, B->d_red_r, s));
  BHIP(B, launch_bt_pack(B->d_insts, B->d_nrows, B->n, R, B->n_rows, B->d_u, y_dev, 0, 0, s));
  return ELMFB_OK;
}

elmfb_status elmfb_batch_rmatvec(elmfb_batch B, const double* u_dev, double* x_dev, void* stream) {
  if (!B || !u_dev || !x_dev) return bfail(B, ELMFB_E_INVALID, "NULL argument");
  if (!B->assembled) return bfail(B, ELMFB_E_STATE, "rmatvec before assemble");
  hipStream_t s = (hipStream_t)stream;
  const int R = B->R;
  BHIP(B, launch_bt_pack(B->d_insts, B->d_nrows, B->n, R, B->n_rows, u_dev, B->d_u, 1, 0, s));
  BHIP(B, launch_bt_rmv(ELMFB_FP64, B->d_geos, B->d_insts, B->d_blocks, B->d_chunks,
                        (int64_t)B->chunks.size(), B->d_A, B->d_u, R, nullptr, B->d_part, s));
  BHIP(B, launch_bt_finish(B->d_geos, B->d_insts, B->d_ctiles, (int64_t)B->ctiles.size(),
                           B->d_cstart, B->d_part, COL_STORE, R, B->d_w, nullptr, B->d_red_c, s));
  BHIP(B, launch_bt_pack(B->d_insts, B->d_nphis, B->n, R, B->n_phi, B->d_w, x_dev, 0, 1, s));
  return ELMFB_OK;
}

elmfb_status elmfb_batch_solve(elmfb_batch B, const elmfb_solve_opts* opts, double* coef_dev,
                               elmfb_solve_info* info, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!B || !opts || !coef_dev) return bfail(B, ELMFB_E_INVALID, "NULL argument");
  if (!B->assembled) return bfail(B, ELMFB_E_STATE, "solve before assemble");
  if (opts->method != ELMFB_LSQR || opts->precond)
    return bfail(B, ELMFB_E_UNSUPPORTED, "batches solve with unpreconditioned LSQR");
  if (opts->x0_dev || opts->n_check)
    return bfail(B, ELMFB_E_UNSUPPORTED, "batched solves take no warm start or check points");
  if (opts->iter_lim < 0 || opts->check_every < 1 || opts->check_every > 100000 ||
      !(opts->atol >= 0.0) || !(opts->btol >= 0.0))
    return bfail(B, ELMFB_E_INVALID, "bad solve options");
  const int n = B->n, R = B->R;
  hipStream_t caller = (hipStream_t)stream;
  hipStream_t s = B->stream;
  BHIP(B, hipEventRecord(B->ev_in, caller));
  BHIP(B, hipStreamWaitEvent(s, B->ev_in, 0));
  // u = h, beta; v = A^T u / beta, alpha; w = v / alpha, x = 0
  // row partials of ||h||^2 (= ||u||^2 at the start): computed by a ROW_RESID pass with t = 0
  BHIP(B, hipMemsetAsync(B->d_tpart, 0, (size_t)(B->n_bp * R * 8), s));
  BHIP(B, launch_bt_gather(B->d_geos, B->d_insts, B->d_blocks, B->d_cov, B->d_rtiles,
                           (int64_t)B->rtiles.size(), B->d_tpart, ROW_RESID, R, B->d_u, B->d_h,
                           nullptr, B->d_red_r, s));
  BHIP(B, launch_bt_lsqr_init(B->d_state, B->d_insts, n, R, B->d_red_r, B->d_red_r, opts->atol,
                              opts->btol, opts->iter_lim, s));
  BHIP(B, launch_bt_rmv(ELMFB_FP64, B->d_geos, B->d_insts, B->d_blocks, B->d_chunks,
                        (int64_t)B->chunks.size(), B->d_A, B->d_u, R, B->d_state, B->d_part, s));
  BHIP(B, launch_bt_finish(B->d_geos, B->d_insts, B->d_ctiles, (int64_t)B->ctiles.size(),
                           B->d_cstart, B->d_part, COL_STORE_SQ, R, B->d_v, nullptr, B->d_red_c,
                           s));
  BHIP(B, launch_bt_lsqr_init_alpha(B->d_state, B->d_insts, n, R, B->d_red_c, s));
  // w = v / alpha (one update step with t1 = 0, t2 = 0 gives w = v sv)
  BHIP(B, hipMemsetAsync(B->d_x, 0, (size_t)(B->n_phi * R * 8), s));
  BHIP(B, hipMemsetAsync(B->d_w, 0, (size_t)(B->n_phi * R * 8), s));
  BHIP(B, launch_bt_update(B->d_geos, B->d_insts, B->d_ctiles, (int64_t)B->ctiles.size(), R,
                           B->d_x, B->d_w, B->d_v, B->d_state, B->d_red_c2, s));
  int32_t active = 1;
  BHIP(B, launch_bt_count_active(B->d_state, n * R, B->d_count, s));
  BHIP(B, hipMemcpyAsync(&active, B->d_count, 4, hipMemcpyDeviceToHost, s));
  BHIP(B, hipStreamSynchronize(s));
  const int chunk = opts->check_every;
  while (active > 0) {
    if (opts->use_graph) {
      auto it = B->graphs.find(chunk);
      hipGraphExec_t exec = nullptr;
      if (it != B->graphs.end()) {
        exec = it->second;
      } else {
        hipGraph_t graph = nullptr;
        BHIP(B, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e2 = hipSuccess;
        for (int i = 0; i < chunk && e2 == hipSuccess; ++i) e2 = bt_iteration(B, s);
        hipError_t e3 = hipStreamEndCapture(s, &graph);
        if (e2 != hipSuccess || e3 != hipSuccess) {
          if (graph) hipGraphDestroy(graph);
          BHIP(B, e2 != hipSuccess ? e2 : e3);
        }
        hipError_t e4 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        BHIP(B, e4);
        B->graphs[chunk] = exec;
      }
      BHIP(B, hipGraphLaunch(exec, s));
    } else {
      for (int i = 0; i < chunk; ++i) BHIP(B, bt_iteration(B, s));
    }
    BHIP(B, launch_bt_count_active(B->d_state, n * R, B->d_count, s));
    BHIP(B, hipMemcpyAsync(&active, B->d_count, 4, hipMemcpyDeviceToHost, s));
    BHIP(B, hipStreamSynchronize(s));
  }
  BHIP(B, launch_bt_pack(B->d_insts, B->d_nphis, n, R, B->n_phi, B->d_x, coef_dev, 0, 1, s));
  BHIP(B, hipEventRecord(B->ev_out, s));
  BHIP(B, hipStreamWaitEvent(caller, B->ev_out, 0));
  if (info) {
    std::vector<SolveState> st((size_t)n * R);
    BHIP(B, hipMemcpyAsync(st.data(), B->d_state, st.size() * sizeof(SolveState),
                           hipMemcpyDeviceToHost, s));
    BHIP(B, hipStreamSynchronize(s));
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (size_t k = 0; k < st.size(); ++k) {
      info[k] = elmfb_solve_info{};
      info[k].istop = st[k].istop;
      info[k].iters = st[k].itn;
      info[k].rnorm = st[k].rnorm;
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
