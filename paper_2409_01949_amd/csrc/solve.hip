// Solve drivers behind the C ABI: LSQR / CGLS on the block-sparse matrix with device-resident
// recurrences captured in hipGraphs, right block-Jacobi preconditioning, FP64 iterative
// refinement around low-precision inner LSQR, Gram blocks and the preconditioner factors.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "handle.h"

namespace {

// The matrix copy, right-hand side and preconditioning of one Krylov run.  With block-Jacobi
// (bj) the iterate is the correction in preconditioned coordinates; `apply` says whether R^{-1}
// is applied in every step (else A is the folded M R^{-1}).  A_x is the FP64 matrix M, for the
// residual of a warm start.
struct KCtx {
  const void* A;
  int prec;
  const double* rhs;
  bool bj;
  bool apply;
  const double* A_x;
};

double* red_slot(elmfb_problem h, int i) { return h->d_red + (int64_t)2 * kRedBlocks * i; }

// norm partials the soft-constraint rows add after the row gather's
int bc_parts(const Geo& g) { return g.n_bc > 0 ? bc_row_wgs(g) : 0; }

const double* state_field(elmfb_problem h, size_t off) {
  return reinterpret_cast<const double*>(reinterpret_cast<const char*>(h->d_state) + off);
}

// The one-workgroup LSQR takes the system when its vectors fit in LDS and its matrix is small
// enough to re-read from one CU's caches every step; ELMFB_PERSISTENT=0 turns it off.
bool one_workgroup_fits(elmfb_problem h) {
  if (const char* e = std::getenv("ELMFB_PERSISTENT"))
    if (e[0] == '0' && e[1] == 0) return false;
  // the one-workgroup kernel finds covering blocks arithmetically on a full tensor grid of
  // subdomains and keeps its handful of constraint rows in LDS
  if (h->geo.domain != ELMFB_DOMAIN_BOX || h->geo.n_bc > ELMFB_MAX_BC) return false;
  return persistent_lds_bytes(h->geo, h->n_block_points, h->n_store, false) <= kPersistMaxLds &&
         h->n_store <= kPersistMaxEntries;
}

hipError_t lsqr_iteration(elmfb_problem h, const KCtx& c, hipStream_t s) {
  const Geo& g = h->geo;
  SolveState* st = h->d_state;
  double *red1 = red_slot(h, 0), *red2 = red_slot(h, 1), *red3 = red_slot(h, 2);
  const int rw = rows_wg(g), cw = cols_wg(g);
  const int64_t nt = (int64_t)h->tiles.size(), nc = (int64_t)h->chunks.size();
  hipError_t e;
  // u = A v / alpha - ... (v scaled by 1/alpha as it is read)
  if (c.apply) {
    if ((e = launch_bj_apply(g, h->d_rinvT, h->d_v, state_field(h, offsetof(SolveState, sv)),
                             h->d_vt, st, s)))
      return e;
    if ((e = launch_mv_blocks(g, c.prec, h->d_blocks, h->d_tiles, nt, c.A, h->d_vt, nullptr,
                              h->d_tpart, st, s)))
      return e;
  } else {
    if ((e = launch_mv_blocks(g, c.prec, h->d_blocks, h->d_tiles, nt, c.A, h->d_v,
                              state_field(h, offsetof(SolveState, sv)), h->d_tpart, st, s)))
      return e;
  }
  if ((e = launch_gather_rows(g, h->d_blocks, h->d_cov, h->d_tpart, ROW_LSQR_U, h->d_u, nullptr,
                              st, red1, rw, s)))
    return e;
  // soft-constraint rows: their u entries and one more norm partial
  if ((e = launch_bc_rows(g, h->d_bc, c.apply ? h->d_vt : h->d_v,
                          c.apply ? nullptr : state_field(h, offsetof(SolveState, sv)), ROW_LSQR_U,
                          h->d_u, nullptr, st, red1 + rw, s)))
    return e;
  if ((e = launch_lsqr_beta(st, red1, rw + bc_parts(g), h->d_hist, s))) return e;
  if ((e = launch_rmv_chunks(g, c.prec, h->d_blocks, h->d_chunks, nc, c.A, h->d_u,
                             state_field(h, offsetof(SolveState, su)), h->d_part, st, s)))
    return e;
  int na = cw;
  if (c.apply) {
    if ((e = launch_rmv_finish(g, h->d_cstart, h->d_part, COL_STORE, h->d_xt, st, red2, cw, s)))
      return e;
    if ((e = launch_bj_apply_t(g, h->d_rinv, h->d_xt, COL_LSQR_V, h->d_v, st, red2, s))) return e;
    na = bj_wg(g);
  } else {
    if ((e = launch_rmv_finish(g, h->d_cstart, h->d_part, COL_LSQR_V, h->d_v, st, red2, cw,
                               h->d_bc, h->d_u, state_field(h, offsetof(SolveState, su)), s)))
      return e;
  }
  if ((e = launch_lsqr_alpha(st, red2, na, h->d_hist, s))) return e;
  if ((e = launch_lsqr_update(g, h->d_x, h->d_w, h->d_v, st, red3, cw, s))) return e;
  return launch_lsqr_stop(st, red3, cw, s);
}

hipError_t cgls_iteration(elmfb_problem h, const KCtx& c, hipStream_t s) {
  const Geo& g = h->geo;
  SolveState* st = h->d_state;
  double *red1 = red_slot(h, 0), *red2 = red_slot(h, 1), *red3 = red_slot(h, 2);
  const int rw = rows_wg(g), cw = cols_wg(g);
  hipError_t e;
  if ((e = launch_mv_blocks(g, c.prec, h->d_blocks, h->d_tiles, (int64_t)h->tiles.size(), c.A,
                            h->d_w, nullptr, h->d_tpart, st, s)))
    return e;
  if ((e = launch_gather_rows(g, h->d_blocks, h->d_cov, h->d_tpart, ROW_STORE_SQ, h->d_t, nullptr,
                              st, red1, rw, s)))
    return e;
  if ((e = launch_bc_rows(g, h->d_bc, h->d_w, nullptr, ROW_STORE_SQ, h->d_t, nullptr, st,
                          red1 + rw, s)))
    return e;
  if ((e = launch_cgls_step_a(st, red1, rw + bc_parts(g), s))) return e;
  if ((e = launch_cgls_update_x(g, h->d_x, h->d_w, st, s))) return e;
  if ((e = launch_cgls_update_r(g, h->d_u, h->d_t, st, red2, rw, s))) return e;
  if ((e = launch_rmv_chunks(g, c.prec, h->d_blocks, h->d_chunks, (int64_t)h->chunks.size(), c.A,
                             h->d_u, nullptr, h->d_part, st, s)))
    return e;
  if ((e = launch_rmv_finish(g, h->d_cstart, h->d_part, COL_STORE_SQ, h->d_v, st, red3, cw,
                             h->d_bc, h->d_u, nullptr, s)))
    return e;
  if ((e = launch_cgls_step_b(st, red2, rw, red3, cw, s))) return e;
  return launch_cgls_update_p(g, h->d_w, h->d_v, st, s);
}

// u (LSQR) or r (CGLS) = rhs - A x0, the first bidiagonalisation step, x = x0 (LSQR without
// preconditioning) or 0 (preconditioned LSQR solves for the correction y, x = x0 + R^{-1} y).
hipError_t solve_init(elmfb_problem h, const KCtx& c, int method, const double* x0,
                      hipStream_t s) {
  const Geo& g = h->geo;
  double *red1 = red_slot(h, 0), *red2 = red_slot(h, 1), *red3 = red_slot(h, 2);
  const int rw = rows_wg(g), cw = cols_wg(g);
  const int64_t nrt = g.n_rows + g.n_bc;   // collocation rows, then the soft-constraint rows
  int n2 = rw;
  hipError_t e;
  if (x0) {   // x0 is in the coordinates of M
    if ((e = launch_mv_blocks(g, ELMFB_FP64, h->d_blocks, h->d_tiles, (int64_t)h->tiles.size(),
                              c.A_x, x0, nullptr, h->d_tpart, nullptr, s)))
      return e;
    if ((e = launch_gather_rows(g, h->d_blocks, h->d_cov, h->d_tpart, ROW_RESID, h->d_u, c.rhs,
                                nullptr, red2, rw, s)))
      return e;
    if ((e = launch_bc_rows(g, h->d_bc, x0, nullptr, ROW_RESID, h->d_u, c.rhs, nullptr,
                            red2 + rw, s)))
      return e;
    n2 = rw + bc_parts(g);
  } else {
    if ((e = launch_copy(c.rhs, h->d_u, nrt, s))) return e;
    if ((e = launch_sumsq(h->d_u, nrt, red2, rw, s))) return e;
  }
  if ((e = launch_sumsq(c.rhs, nrt, red1, rw, s))) return e;
  if (method == ELMFB_LSQR) {
    if ((e = launch_lsqr_init(h->d_state, red1, rw, red2, n2, s))) return e;
    if ((e = launch_rmv_chunks(g, c.prec, h->d_blocks, h->d_chunks, (int64_t)h->chunks.size(), c.A,
                               h->d_u, state_field(h, offsetof(SolveState, su)), h->d_part,
                               nullptr, s)))
      return e;
    int na = cw;
    if (c.apply) {
      if ((e = launch_rmv_finish(g, h->d_cstart, h->d_part, COL_STORE, h->d_xt, nullptr, red3, cw,
                                 s)))
        return e;
      if ((e = launch_bj_apply_t(g, h->d_rinv, h->d_xt, COL_STORE_SQ, h->d_v, nullptr, red3, s)))
        return e;
      na = bj_wg(g);
    } else {
      if ((e = launch_rmv_finish(g, h->d_cstart, h->d_part, COL_STORE_SQ, h->d_v, nullptr, red3,
                                 cw, h->d_bc, h->d_u, state_field(h, offsetof(SolveState, su)),
                                 s)))
        return e;
    }
    if ((e = launch_lsqr_init_alpha(h->d_state, red3, na, h->d_hist, s))) return e;
    return launch_init_xw(g, c.bj ? nullptr : x0, h->d_x, h->d_w, h->d_v, h->d_state, s);
  }
  // CGLS: s = A^T r, p = s, x = x0
  if ((e = launch_rmv_chunks(g, c.prec, h->d_blocks, h->d_chunks, (int64_t)h->chunks.size(), c.A,
                             h->d_u, nullptr, h->d_part, nullptr, s)))
    return e;
  if ((e = launch_rmv_finish(g, h->d_cstart, h->d_part, COL_STORE_SQ, h->d_v, nullptr, red3, cw,
                             h->d_bc, h->d_u, nullptr, s)))
    return e;
  if ((e = launch_cgls_init(h->d_state, red1, rw, red2, n2, red3, cw, h->anorm_f, s))) return e;
  if ((e = launch_copy(h->d_v, h->d_w, g.n_phi, s))) return e;
  if (x0) return launch_copy(x0, h->d_x, g.n_phi, s);
  return hipMemsetAsync(h->d_x, 0, (size_t)g.n_phi * 8, s);
}

// Workgroups (and p . y partials) of the second pass of y = G p: 4 lanes per coefficient.
int gmv_wg(const Geo& g) {
  const int64_t nb = (4 * g.n_phi + 255) / 256;
  return (int)(nb < kRedBlocks ? nb : kRedBlocks);
}

// y = G p on the stored Gram blocks (all pairs), gmv_wg p . y partials into red.
hipError_t gram_mv(elmfb_problem h, const double* p, double* y, const SolveState* st, double* red,
                   hipStream_t s) {
  return launch_gram_mv(h->geo, h->gram_prec, h->d_gcg_pairs, h->gram_npairs, h->d_G,
                        h->d_gcg_rowptr, h->d_gcg_idx, p, h->d_gcg_part, y, st, red,
                        gmv_wg(h->geo), s);
}

// z = (R^T R)^{-1} r = R^{-1} R^{-T} r per block (block-Jacobi of the normal equations).
hipError_t gcg_precond(elmfb_problem h, const double* r, double* z, const SolveState* st,
                       hipStream_t s) {
  hipError_t e = launch_bj_apply_t(h->geo, h->d_rinv, r, COL_STORE, h->d_gcg_tmp, st, nullptr, s);
  if (e != hipSuccess) return e;
  return launch_bj_apply(h->geo, h->d_rinvT, h->d_gcg_tmp, nullptr, z, st, s);
}

// One CG step on G a = g.  a = d_x, r = d_v, p = d_w, q = d_vt, z = d_xt (c.bj) or r.
hipError_t gcg_iteration(elmfb_problem h, const KCtx& c, hipStream_t s) {
  const Geo& g = h->geo;
  SolveState* st = h->d_state;
  double *red1 = red_slot(h, 0), *red2 = red_slot(h, 1), *red3 = red_slot(h, 2);
  const int cw = cols_wg(g);
  hipError_t e;
  if ((e = gram_mv(h, h->d_w, h->d_vt, st, red1, s))) return e;
  if ((e = launch_gcg_alpha(st, red1, gmv_wg(g), s))) return e;
  if ((e = launch_gcg_update(g, h->d_x, h->d_v, h->d_w, h->d_vt, st, red2, cw, s))) return e;
  const double* z = h->d_v;
  if (c.bj) {
    if ((e = gcg_precond(h, h->d_v, h->d_xt, st, s))) return e;
    if ((e = launch_dot(h->d_v, h->d_xt, g.n_phi, st, red3, cw, s))) return e;
    z = h->d_xt;
  }
  if ((e = launch_gcg_beta(st, red2, cw, c.bj ? red3 : nullptr, cw, s))) return e;
  return launch_gcg_pupdate(g, h->d_w, z, st, 0, s);
}

// Start CG on G a = M^T rhs (rhs = c.rhs over the rows), from x0 or zero.
hipError_t gcg_start(elmfb_problem h, const KCtx& c, const double* x0, hipStream_t s) {
  const Geo& g = h->geo;
  double *red1 = red_slot(h, 0), *red2 = red_slot(h, 1), *red3 = red_slot(h, 2);
  const int cw = cols_wg(g);
  hipError_t e;
  // r = g = M^T rhs (FP64 products), ||g||^2 partials in red1
  if ((e = launch_rmv_chunks(g, ELMFB_FP64, h->d_blocks, h->d_chunks, (int64_t)h->chunks.size(),
                             h->d_A, c.rhs, nullptr, h->d_part, nullptr, s)))
    return e;
  if ((e = launch_rmv_finish(g, h->d_cstart, h->d_part, COL_STORE_SQ, h->d_v, nullptr, red1, cw,
                             s)))
    return e;
  if (x0) {
    if ((e = launch_copy(x0, h->d_x, g.n_phi, s))) return e;
    if ((e = gram_mv(h, h->d_x, h->d_vt, nullptr, red2, s))) return e;
    if ((e = launch_axpy(-1.0, h->d_vt, h->d_v, g.n_phi, s))) return e;
  } else {
    if ((e = hipMemsetAsync(h->d_x, 0, (size_t)g.n_phi * 8, s))) return e;
  }
  if ((e = launch_dot(h->d_v, h->d_v, g.n_phi, nullptr, red2, cw, s))) return e;
  const double* z = h->d_v;
  if (c.bj) {
    if ((e = gcg_precond(h, h->d_v, h->d_xt, nullptr, s))) return e;
    if ((e = launch_dot(h->d_v, h->d_xt, g.n_phi, nullptr, red3, cw, s))) return e;
    z = h->d_xt;
  }
  if ((e = launch_gcg_init(h->d_state, red1, cw, red2, cw, c.bj ? red3 : nullptr, cw, s))) return e;
  return launch_gcg_pupdate(g, h->d_w, z, h->d_state, 1, s);
}

// Device tables of the stored Gram pairs for CG, rebuilt after every elmfb_gram call.
elmfb_status gcg_prepare(elmfb_problem h) {
  if (h->gcg_gen == h->gram_gen) return ELMFB_OK;
  const Geo& g = h->geo;
  const int64_t np = h->gram_npairs;
  std::vector<std::vector<int32_t>> rows(g.n_blocks);
  for (int64_t p = 0; p < np; ++p) {
    const GramPair& P = h->gram_pairs_host[p];
    rows[P.bi].push_back((int32_t)(2 * p));
    if (P.bi != P.bj) rows[P.bj].push_back((int32_t)(2 * p + 1));
  }
  std::vector<int32_t> row_ptr(g.n_blocks + 1, 0), idx;
  for (int b = 0; b < g.n_blocks; ++b) {
    row_ptr[b] = (int32_t)idx.size();
    idx.insert(idx.end(), rows[b].begin(), rows[b].end());
  }
  row_ptr[g.n_blocks] = (int32_t)idx.size();
  dfree(h, h->d_gcg_pairs);
  dfree(h, h->d_gcg_rowptr);
  dfree(h, h->d_gcg_idx);
  dfree(h, h->d_gcg_part);
  h->d_gcg_pairs = nullptr;
  h->d_gcg_rowptr = h->d_gcg_idx = nullptr;
  h->d_gcg_part = nullptr;
  h->gcg_gen = -1;
  HIP_OR_FAIL(h, dalloc(h, &h->d_gcg_pairs, np * (int64_t)sizeof(GramPair)));
  HIP_OR_FAIL(h, dalloc(h, &h->d_gcg_rowptr, (int64_t)row_ptr.size() * 4));
  HIP_OR_FAIL(h, dalloc(h, &h->d_gcg_idx, (int64_t)idx.size() * 4 + 4));
  HIP_OR_FAIL(h, dalloc(h, &h->d_gcg_part, 2 * np * g.K * 8));
  if (!h->d_gcg_tmp) HIP_OR_FAIL(h, dalloc(h, &h->d_gcg_tmp, g.n_phi * 8));
  if (np > 0)
    HIP_OR_FAIL(h, hipMemcpy(h->d_gcg_pairs, h->gram_pairs_host.data(), np * sizeof(GramPair),
                             hipMemcpyHostToDevice));
  HIP_OR_FAIL(h, hipMemcpy(h->d_gcg_rowptr, row_ptr.data(), row_ptr.size() * 4,
                           hipMemcpyHostToDevice));
  if (!idx.empty())
    HIP_OR_FAIL(h, hipMemcpy(h->d_gcg_idx, idx.data(), idx.size() * 4, hipMemcpyHostToDevice));
  h->gcg_gen = h->gram_gen;
  return ELMFB_OK;
}

hipError_t enqueue_iterations(elmfb_problem h, const KCtx& c, int method, int n, hipStream_t s) {
  for (int i = 0; i < n; ++i) {
    hipError_t e = method == ELMFB_LSQR        ? lsqr_iteration(h, c, s)
                   : method == ELMFB_NORMAL_CG ? gcg_iteration(h, c, s)
                                               : cgls_iteration(h, c, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t get_graph(elmfb_problem h, const KCtx& c, int method, int n, hipGraphExec_t* out) {
  const std::vector<int64_t> key = {method, n, (int64_t)c.A, c.prec, (int64_t)c.rhs, c.bj,
                                    c.apply, method == ELMFB_NORMAL_CG ? h->gram_gen : 0};
  auto it = h->graphs.find(key);
  if (it != h->graphs.end()) {
    *out = it->second;
    return hipSuccess;
  }
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t e2 = enqueue_iterations(h, c, method, n, h->stream);
  e = hipStreamEndCapture(h->stream, &graph);
  if (e2 != hipSuccess) {
    if (graph) hipGraphDestroy(graph);
    return e2;
  }
  if (e != hipSuccess) return e;
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) return e;
  h->graphs[key] = exec;
  *out = exec;
  return hipSuccess;
}

hipError_t run_iterations(elmfb_problem h, const KCtx& c, int method, int n, bool graph,
                          hipStream_t s) {
  if (!graph) return enqueue_iterations(h, c, method, n, s);
  while (n > 0) {
    const int m = n > kGraphMaxSteps ? kGraphMaxSteps : n;
    hipGraphExec_t exec = nullptr;
    hipError_t e = get_graph(h, c, method, m, &exec);
    if (e == hipSuccess) e = hipGraphLaunch(exec, s);
    if (e != hipSuccess) return e;
    n -= m;
  }
  return hipSuccess;
}

// Evaluate the current solution at the check points and update the rel-L2 stop state.
hipError_t check_solution(elmfb_problem h, const elmfb_solve_opts* o, const double* x,
                          hipStream_t s) {
  hipError_t e = launch_evaluate(h->geo, h->d_W, h->d_b, x, o->check_pts_dev, o->n_check,
                                 h->d_eval, s);
  if (e != hipSuccess) return e;
  int nw = (int)((o->n_check + 255) / 256);
  if (nw > kRedBlocks) nw = kRedBlocks;
  return launch_check_rel_l2(h->d_eval, o->check_ref_dev, o->n_check, h->d_state, red_slot(h, 3),
                             nw, s);
}

// Plan the chunks of a set of Gram pairs, upload the tables, run the Gram kernel into G.
elmfb_status run_gram(elmfb_problem h, int prec, std::vector<GramPair>& pairs, void* G,
                      hipStream_t s) {
  const Geo& g = h->geo;
  const int64_t KK = (int64_t)g.K * g.K;
  std::vector<GramChunk> chunks;
  std::vector<int32_t> multi;
  int64_t p_off = 0;
  for (size_t p = 0; p < pairs.size(); ++p) {
    GramPair& pr = pairs[p];
    const int64_t ns = (int64_t)pr.nx * pr.ny;
    pr.g_off = (int64_t)p * KK;
    pr.c0 = (int32_t)chunks.size();
    pr.nchunks = (int32_t)((ns + kGramChunk - 1) / kGramChunk);
    pr.p_off = 0;
    if (pr.nchunks > 1) {
      pr.p_off = p_off;
      p_off += pr.nchunks;
      multi.push_back((int32_t)p);
    }
    for (int64_t s0 = 0; s0 < ns; s0 += kGramChunk) chunks.push_back(GramChunk{(int32_t)p, (int32_t)s0});
  }
  const int64_t acc_es = prec == ELMFB_FP64 ? 8 : 4;
  auto grow = [&](void** buf, int64_t* cap, int64_t need) -> hipError_t {
    if (need <= *cap) return hipSuccess;
    dfree(h, *buf);
    *buf = nullptr;
    *cap = 0;
    hipError_t e = dalloc_bytes(h, buf, need);
    if (e == hipSuccess) *cap = need;
    return e;
  };
  HIP_OR_FAIL(h, grow((void**)&h->d_gpairs, &h->gpairs_cap, (int64_t)pairs.size() * sizeof(GramPair)));
  HIP_OR_FAIL(h, grow((void**)&h->d_gchunks, &h->gchunks_cap, (int64_t)chunks.size() * sizeof(GramChunk)));
  HIP_OR_FAIL(h, grow((void**)&h->d_gmulti, &h->gmulti_cap, (int64_t)multi.size() * 4 + 4));
  HIP_OR_FAIL(h, grow(&h->d_gpart, &h->gpart_bytes, p_off * KK * acc_es));
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_gpairs, pairs.data(), pairs.size() * sizeof(GramPair),
                                hipMemcpyHostToDevice, s));
  if (!chunks.empty())
    HIP_OR_FAIL(h, hipMemcpyAsync(h->d_gchunks, chunks.data(), chunks.size() * sizeof(GramChunk),
                                  hipMemcpyHostToDevice, s));
  if (!multi.empty())
    HIP_OR_FAIL(h, hipMemcpyAsync(h->d_gmulti, multi.data(), multi.size() * 4,
                                  hipMemcpyHostToDevice, s));
  const void* A = prec == ELMFB_FP64 ? (const void*)h->d_A : h->d_A_lo;
  HIP_OR_FAIL(h, launch_gram(g, prec, h->d_blocks, h->d_gpairs, h->d_gchunks,
                             (int64_t)chunks.size(), h->d_gmulti, (int64_t)multi.size(), A, G,
                             h->d_gpart, s));
  h->gram_nchunks = (int64_t)chunks.size();
  h->gram_nmulti = (int64_t)multi.size();
  // the host tables above must outlive the asynchronous copies
  HIP_OR_FAIL(h, hipStreamSynchronize(s));
  return ELMFB_OK;
}

// Eigenvalues below x of the symmetric tridiagonal matrix with zero diagonal and off-diagonal
// e (Sturm count: the negative pivots of the LDL^T factorisation of T - x I).  For the
// Golub-Kahan matrix of a (k+1) x k bidiagonal B its eigenvalues are 0 and +-sigma_i(B), and
// bisection on it finds small singular values to high relative accuracy (Demmel and Kahan 1990).
int64_t tgk_count(const std::vector<double>& e, double x) {
  const double tiny = std::numeric_limits<double>::min();
  int64_t c = 0;
  double d = -x;
  for (size_t i = 0;; ++i) {
    if (d < 0.0) ++c;
    if (i == e.size()) break;
    if (d == 0.0) d = -tiny;
    d = -x - e[i] * (e[i] / d);
  }
  return c;
}

}  // namespace

extern "C" {

elmfb_status elmfb_bidiag_sigma(const double* ab_host, int32_t k, double* sigma_max_host,
                                double* sigma_min_host) {
  if (!ab_host || k < 1 || !sigma_max_host || !sigma_min_host)
    return fail(nullptr, ELMFB_E_INVALID, "bad argument");
  // off-diagonal of the Golub-Kahan matrix of B_k: alpha_1, beta_2, alpha_2, ..., alpha_k, beta_{k+1}
  std::vector<double> e((size_t)2 * k);
  double emax = 0.0;
  for (int i = 0; i < k; ++i) {
    e[2 * i] = ab_host[2 * i];
    e[2 * i + 1] = ab_host[2 * (i + 1) + 1];
    emax = std::max(emax, std::max(std::fabs(e[2 * i]), std::fabs(e[2 * i + 1])));
  }
  if (!(emax > 0.0) || !std::isfinite(emax))
    return fail(nullptr, ELMFB_E_NUMERIC, "degenerate bidiagonal");
  const int64_t n_all = 2 * (int64_t)k + 1;
  // largest eigenvalue: all 2k+1 lie below x
  double lo = 0.0, hi = 2.0 * emax;
  for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (tgk_count(e, mid) >= n_all) hi = mid;
    else lo = mid;
  }
  const double smax = hi;
  // smallest singular value: the (k+2)-th smallest eigenvalue (k negative ones and a zero below
  // it), by bisection on a logarithmic scale down to 1e-300 of sigma_max
  lo = smax * 1e-300;
  hi = smax;
  for (int it = 0; it < 400 && hi > lo * (1.0 + 1e-14); ++it) {
    const double mid = std::sqrt(lo * hi);
    if (tgk_count(e, mid) >= (int64_t)k + 2) hi = mid;
    else lo = mid;
  }
  *sigma_max_host = smax;
  *sigma_min_host = hi;
  return ELMFB_OK;
}

elmfb_status elmfb_condition_estimate(elmfb_problem h, double* sigma_max_host,
                                      double* sigma_min_host, int32_t* k_host) {
  if (!h || !sigma_max_host || !sigma_min_host) return fail(h, ELMFB_E_INVALID, "bad argument");
  const int k = std::min(h->hist_k, kHistCap - 1);
  if (k < 1) return fail(h, ELMFB_E_STATE, "the last solve recorded no LSQR step");
  std::vector<double> hist((size_t)2 * (k + 1));
  HIP_OR_FAIL(h, hipMemcpy(hist.data(), h->d_hist, hist.size() * 8, hipMemcpyDeviceToHost));
  const elmfb_status es = elmfb_bidiag_sigma(hist.data(), k, sigma_max_host, sigma_min_host);
  if (es != ELMFB_OK) return fail(h, es, "degenerate bidiagonal");
  if (k_host) *k_host = k;
  return ELMFB_OK;
}


elmfb_status elmfb_gram(elmfb_problem h, int32_t prec, int32_t which, void* stream) {
  if (!h) return fail(h, ELMFB_E_INVALID, "NULL handle");
  if (!h->assembled) return fail(h, ELMFB_E_STATE, "gram before assemble");
  if (h->geo.n_bc > 0)
    return fail(h, ELMFB_E_UNSUPPORTED, "Gram blocks of a system with soft-constraint rows");
  if (which != 0 && which != 1) return fail(h, ELMFB_E_INVALID, "which must be 0 or 1");
  if (prec != ELMFB_FP64 && !(prec == h->lo_prec && h->d_A_lo))
    return fail(h, ELMFB_E_STATE, "no stored matrix copy in that precision");
  std::vector<GramPair> pairs;
  if (which == 1) {
    pairs = h->pairs_all;
  } else {
    for (int64_t idx : h->diag_pair)
      if (idx >= 0) pairs.push_back(h->pairs_all[idx]);
  }
  const int64_t KK = (int64_t)h->geo.K * h->geo.K;
  const int64_t need = (int64_t)pairs.size() * KK * (prec == ELMFB_FP64 ? 8 : 4);
  if (need > h->G_bytes) {
    dfree(h, h->d_G);
    h->d_G = nullptr;
    h->G_bytes = 0;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && (size_t)need > free_b)
      return fail(h, ELMFB_E_NOMEM, "Gram blocks do not fit in free device memory");
    HIP_OR_FAIL(h, dalloc_bytes(h, &h->d_G, need));
    h->G_bytes = need;
  }
  hipStream_t s = (hipStream_t)stream;
  elmfb_status st = run_gram(h, prec, pairs, h->d_G, s);
  if (st != ELMFB_OK) return st;
  h->gram_prec = prec;
  h->gram_which = which;
  h->gram_gen += 1;
  // CG loops captured on the previous Gram blocks are keyed to the old generation and never
  // replayed again: release them once the stream has drained
  bool synced = false;
  for (auto it = h->graphs.begin(); it != h->graphs.end();) {
    if (it->first[0] == ELMFB_NORMAL_CG) {
      if (!synced) {
        HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
        synced = true;
      }
      hipGraphExecDestroy(it->second);
      it = h->graphs.erase(it);
    } else {
      ++it;
    }
  }
  h->gram_npairs = (int64_t)pairs.size();
  h->gram_pairs_host = pairs;
  return ELMFB_OK;
}

elmfb_status elmfb_time_gram(elmfb_problem h, int32_t prec, int32_t which, int32_t reps,
                             double* ms_host, double* flops_host, void* stream) {
  if (!h || !ms_host || reps < 1) return fail(h, ELMFB_E_INVALID, "bad argument");
  const elmfb_status st = elmfb_gram(h, prec, which, stream);
  if (st != ELMFB_OK) return st;
  const Geo& g = h->geo;
  if (flops_host) {
    double shared = 0.0;
    for (const GramPair& P : h->gram_pairs_host) shared += (double)P.nx * P.ny;
    *flops_host = 2.0 * g.K * g.K * shared;
  }
  hipStream_t s = (hipStream_t)stream;
  const void* A = prec == ELMFB_FP64 ? (const void*)h->d_A : h->d_A_lo;
  hipEvent_t e0, e1;
  HIP_OR_FAIL(h, hipEventCreate(&e0));
  HIP_OR_FAIL(h, hipEventCreate(&e1));
  // the tables of the call above are still on the device; relaunch the same computation
  hipError_t e = hipEventRecord(e0, s);
  for (int i = 0; i < reps && e == hipSuccess; ++i)
    e = launch_gram(g, prec, h->d_blocks, h->d_gpairs, h->d_gchunks, h->gram_nchunks,
                    h->d_gmulti, h->gram_nmulti, A, h->d_G, h->d_gpart, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  HIP_OR_FAIL(h, e);
  *ms_host = (double)t / reps;
  return ELMFB_OK;
}

elmfb_status elmfb_copy_gram(elmfb_problem h, void* dst_dev, int64_t* pairs_host,
                             int64_t* n_pairs_host, void* stream) {
  if (!h) return fail(h, ELMFB_E_INVALID, "NULL handle");
  if (h->gram_prec < 0) return fail(h, ELMFB_E_STATE, "no Gram blocks computed");
  if (n_pairs_host) *n_pairs_host = h->gram_npairs;
  if (pairs_host)
    for (int64_t p = 0; p < h->gram_npairs; ++p) {
      pairs_host[3 * p] = h->gram_pairs_host[p].bi;
      pairs_host[3 * p + 1] = h->gram_pairs_host[p].bj;
      pairs_host[3 * p + 2] = h->gram_pairs_host[p].g_off;
    }
  if (dst_dev) {
    const int64_t KK = (int64_t)h->geo.K * h->geo.K;
    HIP_OR_FAIL(h, hipMemcpyAsync(dst_dev, h->d_G,
                                  (size_t)(h->gram_npairs * KK * (h->gram_prec == ELMFB_FP64 ? 8 : 4)),
                                  hipMemcpyDeviceToDevice, (hipStream_t)stream));
  }
  return ELMFB_OK;
}

elmfb_status elmfb_precondition(elmfb_problem h, double shift, int32_t* n_fallback, void* stream) {
  if (!h) return fail(h, ELMFB_E_INVALID, "NULL handle");
  if (!h->assembled) return fail(h, ELMFB_E_STATE, "precondition before assemble");
  if (h->geo.n_bc > 0)
    return fail(h, ELMFB_E_UNSUPPORTED, "block-Jacobi for a system with soft-constraint rows");
  if (!(shift > 0.0) || !std::isfinite(shift)) return fail(h, ELMFB_E_INVALID, "shift must be > 0");
  const Geo& g = h->geo;
  const int64_t KK = (int64_t)g.K * g.K;
  hipStream_t s = (hipStream_t)stream;
  if (!h->d_bj_work) {
    HIP_OR_FAIL(h, dalloc(h, &h->d_bj_work, g.n_blocks * KK * 8 * 2));   // diagonal Gram + R
    HIP_OR_FAIL(h, dalloc(h, &h->d_rinv, g.n_blocks * KK * 8));
    HIP_OR_FAIL(h, dalloc(h, &h->d_rinvT, g.n_blocks * KK * 8));
    HIP_OR_FAIL(h, dalloc(h, &h->d_diag_off, g.n_blocks * 8));
  }
  double* gdiag = h->d_bj_work;
  double* rwork = h->d_bj_work + g.n_blocks * KK;
  // FP64 diagonal Gram blocks, one slot per block (empty blocks stay zero)
  std::vector<GramPair> pairs;
  std::vector<int64_t> offs(g.n_blocks, 0);
  for (int b = 0; b < g.n_blocks; ++b) offs[b] = (int64_t)b * KK;
  HIP_OR_FAIL(h, hipMemsetAsync(gdiag, 0, (size_t)(g.n_blocks * KK * 8), s));
  std::vector<int> owner;
  for (int b = 0; b < g.n_blocks; ++b)
    if (h->diag_pair[b] >= 0) {
      pairs.push_back(h->pairs_all[h->diag_pair[b]]);
      owner.push_back(b);
    }
  // run_gram places pair p at p*K*K; map through a compact buffer when blocks are empty
  const bool dense_map = (int)pairs.size() == g.n_blocks;
  double* target = gdiag;
  if (!dense_map) {
    void* tmp = nullptr;
    HIP_OR_FAIL(h, dalloc_bytes(h, &tmp, (int64_t)pairs.size() * KK * 8));
    target = (double*)tmp;
  }
  elmfb_status st = run_gram(h, ELMFB_FP64, pairs, target, s);
  if (st != ELMFB_OK) return st;
  if (!dense_map) {
    for (size_t p = 0; p < pairs.size(); ++p)
      HIP_OR_FAIL(h, hipMemcpyAsync(gdiag + (int64_t)owner[p] * KK, target + (int64_t)p * KK,
                                    (size_t)KK * 8, hipMemcpyDeviceToDevice, s));
    HIP_OR_FAIL(h, hipStreamSynchronize(s));
    dfree(h, target);
  }
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_diag_off, offs.data(), offs.size() * 8,
                                hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(h, hipMemsetAsync(h->d_flag, 0, 4, s));
  HIP_OR_FAIL(h, launch_bj_factor(g, gdiag, h->d_diag_off, shift, rwork, h->d_rinv, h->d_rinvT,
                                  h->d_flag, s));
  // fold the preconditioner into the matrix: the store_prec rounding of M R^{-1} (inner solves of
  // the refinement) and M R^{-1} in FP64 (FP64 Krylov solves), each when it fits in free device
  // memory with an 8 GB margin and, under ELMFB_MEM_CAP, within the cap together with the
  // footprint; otherwise those solves apply R^{-1} in every step
  h->folded64 = h->folded_lo = false;
  {
    const int64_t es_lo = h->lo_prec == ELMFB_FP64 ? 0 : elem_size(h->lo_prec);
    const int64_t margin = (int64_t)8 << 30;
    int64_t folded_bytes = (h->d_Ahat_lo ? h->n_store * es_lo : 0) + (h->d_Ahat ? h->n_store * 8 : 0);
    auto fits = [&](int64_t bytes) {
      size_t free_b = 0, total_b = 0;
      if (h->mem_cap > 0 && h->bytes_device + folded_bytes + bytes > h->mem_cap) return false;
      const bool ok =
          hipMemGetInfo(&free_b, &total_b) == hipSuccess && (int64_t)free_b > bytes + margin;
      if (ok) folded_bytes += bytes;
      return ok;
    };
    if (es_lo && !h->d_Ahat_lo && fits(h->n_store * es_lo)) {
      HIP_OR_FAIL(h, dalloc_bytes(h, &h->d_Ahat_lo, h->n_store * es_lo));
      HIP_OR_FAIL(h, hipMemsetAsync(h->d_Ahat_lo, 0, (size_t)(h->n_store * es_lo), s));  // padding
    }
    if (!h->d_Ahat && fits(h->n_store * 8)) {
      HIP_OR_FAIL(h, dalloc(h, &h->d_Ahat, h->n_store * 8));
      HIP_OR_FAIL(h, hipMemsetAsync(h->d_Ahat, 0, (size_t)h->n_store * 8, s));           // padding
    }
    const bool lo_ok = es_lo && h->d_Ahat_lo;
    if ((lo_ok || h->d_Ahat) && !h->d_ftiles) {
      std::vector<Tile> ft;
      for (size_t b = 0; b < h->blocks.size(); ++b)
        for (int p0 = 0; p0 < h->blocks[b].n; p0 += 64) ft.push_back(Tile{(int32_t)b, p0});
      HIP_OR_FAIL(h, dalloc_bytes(h, (void**)&h->d_ftiles, (int64_t)(ft.size() * sizeof(Tile)) + 16));
      if (!ft.empty())
        HIP_OR_FAIL(h, hipMemcpy(h->d_ftiles, ft.data(), ft.size() * sizeof(Tile),
                                 hipMemcpyHostToDevice));
      h->n_ftiles = (int64_t)ft.size();
    }
    if (lo_ok || h->d_Ahat) {
      HIP_OR_FAIL(h, launch_bt_fold(lo_ok ? h->lo_prec : ELMFB_FP64, true, g.K, h->d_blocks,
                                    h->d_ftiles, h->n_ftiles, h->d_A, h->d_rinv, nullptr,
                                    h->d_Ahat, lo_ok ? h->d_Ahat_lo : nullptr, s));
      h->folded64 = h->d_Ahat != nullptr;
      h->folded_lo = lo_ok;
    }
  }
  int32_t nf = 0;
  HIP_OR_FAIL(h, hipMemcpyAsync(&nf, h->d_flag, 4, hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(h, hipStreamSynchronize(s));
  if (n_fallback) *n_fallback = nf;
  // an identity fallback leaves that block's columns unscaled, and their FP16 rounding may
  // overflow: such a copy is not used
  if (nf > 0 && h->lo_prec == ELMFB_FP16) h->folded_lo = false;
  h->bj_ready = true;
  return ELMFB_OK;
}

// One right-hand side: the one held in d_h.
static elmfb_status solve_one(elmfb_problem h, const elmfb_solve_opts* opts, double* coef_dev,
                              elmfb_solve_info* info, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!h || !opts || !coef_dev) return fail(h, ELMFB_E_INVALID, "NULL argument");
  if (!h->assembled) return fail(h, ELMFB_E_STATE, "solve before assemble");
  const int method = opts->method;
  h->hist_k = -1;   // the recorded bidiagonal is valid only after a solve that completes
  if (method != ELMFB_LSQR && method != ELMFB_CGLS && method != ELMFB_MIXED_IR &&
      method != ELMFB_NORMAL_CG && method != ELMFB_MIXED_IR_CG)
    return fail(h, ELMFB_E_UNSUPPORTED, "unknown solve method");
  const bool mixed = method == ELMFB_MIXED_IR || method == ELMFB_MIXED_IR_CG;
  const bool on_gram = method == ELMFB_NORMAL_CG || method == ELMFB_MIXED_IR_CG;
  if (opts->iter_lim < 0 || opts->check_every < 1 || opts->check_every > 100000)
    return fail(h, ELMFB_E_INVALID, "iter_lim >= 0 and 1 <= check_every <= 100000 required");
  if (!(opts->atol >= 0.0) || !(opts->btol >= 0.0))
    return fail(h, ELMFB_E_INVALID, "atol and btol must be >= 0");
  if (opts->n_check < 0 || (opts->n_check > 0 && (!opts->check_pts_dev || !opts->check_ref_dev)))
    return fail(h, ELMFB_E_INVALID, "check points need check_pts_dev and check_ref_dev");
  const bool bj = opts->precond != 0;
  if (h->geo.n_bc > 0 && (mixed || on_gram || bj))
    return fail(h, ELMFB_E_UNSUPPORTED,
                "soft-constraint rows: FP64 LSQR and CGLS without preconditioning only");
  if (bj && method == ELMFB_CGLS) return fail(h, ELMFB_E_UNSUPPORTED, "CGLS has no preconditioner");
  if (bj && !h->bj_ready) return fail(h, ELMFB_E_STATE, "precondition before solving with it");
  if (mixed && (opts->inner_iters < 1 || opts->outer_lim < 0))
    return fail(h, ELMFB_E_INVALID, "refinement needs inner_iters >= 1 and outer_lim >= 0");
  if (on_gram) {
    if (h->gram_prec < 0 || h->gram_which != 1)
      return fail(h, ELMFB_E_STATE, "CG on the Gram blocks needs elmfb_gram(h, prec, 1) first");
    const elmfb_status e = gcg_prepare(h);
    if (e != ELMFB_OK) return e;
  }
  if (method == ELMFB_MIXED_IR) {
    if (!h->d_A_lo) return fail(h, ELMFB_E_STATE, "MIXED_IR needs a low-precision stored copy");
    if (h->lo_prec == ELMFB_FP16 && !(bj && h->folded_lo))
      return fail(h, ELMFB_E_UNSUPPORTED,
                  "FP16 inner solves run on the folded copy of M R^-1: precondition (no identity "
                  "fallback) and set precond");
  }
  const Geo& g = h->geo;
  hipStream_t caller = (hipStream_t)stream;
  hipStream_t s = h->stream;
  HIP_OR_FAIL(h, hipEventRecord(h->ev_in, caller));
  HIP_OR_FAIL(h, hipStreamWaitEvent(s, h->ev_in, 0));

  if (method == ELMFB_CGLS && h->anorm_f < 0.0) {
    HIP_OR_FAIL(h, launch_sumsq_entries(ELMFB_FP64, h->d_A, h->n_store, h->d_red, kRedBlocks, s));
    HIP_OR_FAIL(h, launch_reduce_to(h->d_red, kRedBlocks, h->d_scalar, s));
    double ss = 0.0, sb = 0.0;
    HIP_OR_FAIL(h, hipMemcpyAsync(&ss, h->d_scalar, 8, hipMemcpyDeviceToHost, s));
    if (g.n_bc > 0) {   // ||[N; B]||_F^2 = ||N||_F^2 + ||B||_F^2
      HIP_OR_FAIL(h, launch_sumsq(h->d_bc, (int64_t)g.n_bc * g.n_phi, h->d_red, 1, s));
      HIP_OR_FAIL(h, hipMemcpyAsync(&sb, h->d_red, 8, hipMemcpyDeviceToHost, s));
    }
    HIP_OR_FAIL(h, hipStreamSynchronize(s));
    h->anorm_f = std::sqrt(ss + sb);
  }
  if (opts->n_check > h->eval_cap) {
    dfree(h, h->d_eval);
    h->d_eval = nullptr;
    h->eval_cap = 0;
    HIP_OR_FAIL(h, dalloc(h, &h->d_eval, opts->n_check * 8));
    h->eval_cap = opts->n_check;
  }

  SolveState init{};
  init.atol = opts->atol;
  init.btol = opts->btol;
  init.iter_lim = mixed ? opts->inner_iters : opts->iter_lim;
  init.target = opts->n_check > 0 ? opts->target_rel_l2 : 0.0;
  init.rel_l2 = -1.0;
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_state, &init, sizeof(init), hipMemcpyHostToDevice, s));

  SolveState st{};
  int total_iters = 0, outer = 0;
  double outer_rnorm = -1.0;
  const double* result = h->d_x;
  if (!mixed) {
    const bool fold = bj && h->folded64;
    const KCtx c = on_gram ? KCtx{h->d_G, h->gram_prec, h->d_h, bj, false, h->d_A}
                           : KCtx{fold ? (const void*)h->d_Ahat : (const void*)h->d_A, ELMFB_FP64,
                                  h->d_h, bj, bj && !fold, h->d_A};
    // CG on G works on the coefficients themselves; LSQR with block-Jacobi on R x
    const bool recover = bj && !on_gram;
    if (on_gram)
      HIP_OR_FAIL(h, gcg_start(h, c, opts->x0_dev, s));
    else
      HIP_OR_FAIL(h, solve_init(h, c, method, opts->x0_dev, s));
    // FP64 LSQR on a system that fits in one CU's LDS runs whole steps in one workgroup
    const bool one_wg = method == ELMFB_LSQR && !on_gram && !bj && one_workgroup_fits(h);
    HIP_OR_FAIL(h, hipMemcpyAsync(&st, h->d_state, sizeof(st), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(h, hipStreamSynchronize(s));
    while (!st.done) {
      if (one_wg)
        HIP_OR_FAIL(h, launch_lsqr_persistent(g, h->d_blocks, h->d_cov, h->d_A, h->d_bc, h->d_u,
                                              h->d_v, h->d_w, h->d_x, h->d_state, h->d_hist,
                                              opts->check_every, h->n_block_points,
                                              h->n_store, &h->persist_lds_mode, s));
      else
        HIP_OR_FAIL(h, run_iterations(h, c, method, opts->check_every, opts->use_graph != 0, s));
      if (opts->n_check > 0) {
        const double* xcur = h->d_x;
        if (recover) {
          HIP_OR_FAIL(h, launch_bj_recover(g, h->d_rinvT, h->d_x, opts->x0_dev, h->d_c, s));
          xcur = h->d_c;
        }
        HIP_OR_FAIL(h, check_solution(h, opts, xcur, s));
      }
      HIP_OR_FAIL(h, hipMemcpyAsync(&st, h->d_state, sizeof(st), hipMemcpyDeviceToHost, s));
      HIP_OR_FAIL(h, hipStreamSynchronize(s));
    }
    if (recover) {
      HIP_OR_FAIL(h, launch_bj_recover(g, h->d_rinvT, h->d_x, opts->x0_dev, h->d_c, s));
      result = h->d_c;
    }
    total_iters = st.itn;
    if (st.target_hit) st.istop = 8;
  } else {
    // FP64 refinement: c = x0; repeat r = h - A c (FP64), d = inner LSQR on the low copy, c += d
    if (opts->x0_dev)
      HIP_OR_FAIL(h, launch_copy(opts->x0_dev, h->d_c, g.n_phi, s));
    else
      HIP_OR_FAIL(h, hipMemsetAsync(h->d_c, 0, (size_t)g.n_phi * 8, s));
    // the inner solve: LSQR on the low-precision copy (MIXED_IR), in preconditioned coordinates
    // with block-Jacobi, or CG on the stored Gram blocks with rhs M^T r (MIXED_IR_CG)
    const bool fold = bj && h->folded_lo;
    const KCtx inner = on_gram ? KCtx{h->d_G, h->gram_prec, h->d_r, bj, false, h->d_A}
                               : KCtx{fold ? (const void*)h->d_Ahat_lo : (const void*)h->d_A_lo,
                                      h->lo_prec, h->d_r, bj, bj && !fold, h->d_A};
    const int inner_method = on_gram ? ELMFB_NORMAL_CG : ELMFB_LSQR;
    const bool recover = bj && !on_gram;
    const int rw = rows_wg(g);
    int istop = 7;
    for (outer = 0; outer < opts->outer_lim; ++outer) {
      HIP_OR_FAIL(h, launch_mv_blocks(g, ELMFB_FP64, h->d_blocks, h->d_tiles,
                                      (int64_t)h->tiles.size(), h->d_A, h->d_c, nullptr,
                                      h->d_tpart, nullptr, s));
      HIP_OR_FAIL(h, launch_gather_rows(g, h->d_blocks, h->d_cov, h->d_tpart, ROW_RESID, h->d_r,
                                        h->d_h, nullptr, red_slot(h, 3), rw, s));
      HIP_OR_FAIL(h, launch_reduce_to(red_slot(h, 3), rw, h->d_scalar, s));
      if (on_gram)
        HIP_OR_FAIL(h, gcg_start(h, inner, nullptr, s));
      else
        HIP_OR_FAIL(h, solve_init(h, inner, ELMFB_LSQR, nullptr, s));
      int left = opts->inner_iters;
      bool hit = false;
      while (left > 0) {
        const int n = std::min(left, opts->check_every);
        HIP_OR_FAIL(h, run_iterations(h, inner, inner_method, n, opts->use_graph != 0, s));
        left -= n;
        if (opts->n_check > 0 && left > 0) {
          // trial solution c + d after this part of the inner solve
          if (recover)
            HIP_OR_FAIL(h, launch_bj_recover(g, h->d_rinvT, h->d_x, h->d_c, h->d_xt, s));
          else {
            HIP_OR_FAIL(h, launch_copy(h->d_c, h->d_xt, g.n_phi, s));
            HIP_OR_FAIL(h, launch_axpy(1.0, h->d_x, h->d_xt, g.n_phi, s));
          }
          HIP_OR_FAIL(h, check_solution(h, opts, h->d_xt, s));
          HIP_OR_FAIL(h, hipMemcpyAsync(&st, h->d_state, sizeof(st), hipMemcpyDeviceToHost, s));
          HIP_OR_FAIL(h, hipStreamSynchronize(s));
          if (st.target_hit) {
            HIP_OR_FAIL(h, launch_copy(h->d_xt, h->d_c, g.n_phi, s));
            hit = true;
            break;
          }
        } else if (left > 0) {
          HIP_OR_FAIL(h, hipMemcpyAsync(&st, h->d_state, sizeof(st), hipMemcpyDeviceToHost, s));
          HIP_OR_FAIL(h, hipStreamSynchronize(s));
        }
        if (left > 0 && st.done) break;   // the inner LSQR met its own stopping test
      }
      if (!hit) {
        if (recover)
          HIP_OR_FAIL(h, launch_bj_recover(g, h->d_rinvT, h->d_x, h->d_c, h->d_c, s));
        else
          HIP_OR_FAIL(h, launch_axpy(1.0, h->d_x, h->d_c, g.n_phi, s));
        if (opts->n_check > 0) HIP_OR_FAIL(h, check_solution(h, opts, h->d_c, s));
      }
      HIP_OR_FAIL(h, hipMemcpyAsync(&st, h->d_state, sizeof(st), hipMemcpyDeviceToHost, s));
      HIP_OR_FAIL(h, hipStreamSynchronize(s));
      total_iters += st.itn;
      if (st.target_hit) {
        istop = 8;
        ++outer;
        break;
      }
      if (st.done && st.itn == 0 && st.istop == 0) {
        // the inner solve stopped before its first step: the FP64 residual is zero or
        // orthogonal to the range (M^T r = 0), so c already solves the least-squares problem
        istop = 0;
        ++outer;
        break;
      }
    }
    st.istop = istop;
    result = h->d_c;
    // the residual of the returned coefficients, in FP64
    HIP_OR_FAIL(h, launch_mv_blocks(g, ELMFB_FP64, h->d_blocks, h->d_tiles,
                                    (int64_t)h->tiles.size(), h->d_A, h->d_c, nullptr,
                                    h->d_tpart, nullptr, s));
    HIP_OR_FAIL(h, launch_gather_rows(g, h->d_blocks, h->d_cov, h->d_tpart, ROW_RESID, h->d_r,
                                      h->d_h, nullptr, red_slot(h, 3), rw, s));
    HIP_OR_FAIL(h, launch_reduce_to(red_slot(h, 3), rw, h->d_scalar, s));
    double rr = 0.0;
    HIP_OR_FAIL(h, hipMemcpyAsync(&rr, h->d_scalar, 8, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(h, hipStreamSynchronize(s));
    outer_rnorm = std::sqrt(rr);
  }
  HIP_OR_FAIL(h, hipMemcpyAsync(coef_dev, result, (size_t)g.n_phi * 8, hipMemcpyDeviceToDevice, s));
  HIP_OR_FAIL(h, hipEventRecord(h->ev_out, s));
  HIP_OR_FAIL(h, hipStreamWaitEvent(caller, h->ev_out, 0));
  // the bidiagonalisation kept in d_hist belongs to the last LSQR run of this solve
  h->hist_k = (method == ELMFB_LSQR || method == ELMFB_MIXED_IR) ? st.itn : -1;
  if (info) {
    info->istop = st.istop;
    info->iters = total_iters;
    info->outer_iters = outer;
    info->rnorm = mixed ? outer_rnorm : st.rnorm;
    info->arnorm = st.arnorm;
    info->anorm = st.anorm;
    info->xnorm = st.xnorm;
    info->rel_l2 = st.rel_l2;
    info->ms_solve =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return ELMFB_OK;
}

extern "C" elmfb_status elmfb_solve(elmfb_problem h, const elmfb_solve_opts* opts,
                                    double* coef_dev, elmfb_solve_info* info, void* stream) {
  if (!h || !opts || !coef_dev) return fail(h, ELMFB_E_INVALID, "NULL argument");
  if (!h->assembled) return fail(h, ELMFB_E_STATE, "solve before assemble");
  const int R = opts->n_rhs > 1 ? opts->n_rhs : 1;
  if (R > h->n_rhs)
    return fail(h, ELMFB_E_INVALID, "n_rhs exceeds the right-hand sides of the last assembly");
  const Geo& g = h->geo;
  const int64_t nrt = g.n_rows + g.n_bc;
  for (int r = 0; r < R; ++r) {
    // the r-th right-hand side into d_h, ordered before the solve on the caller's stream
    if (h->n_rhs > 1)
      HIP_OR_FAIL(h, hipMemcpyAsync(h->d_h, h->d_hs + (int64_t)r * nrt, (size_t)nrt * 8,
                                    hipMemcpyDeviceToDevice, (hipStream_t)stream));
    elmfb_solve_opts o = *opts;
    o.n_rhs = 1;
    if (o.x0_dev) o.x0_dev += (int64_t)r * g.n_phi;
    if (o.n_check > 0) o.check_ref_dev += (int64_t)r * o.n_check;
    elmfb_solve_info* inf = info ? info + r : nullptr;
    const elmfb_status e = solve_one(h, &o, coef_dev + (int64_t)r * g.n_phi, inf, stream);
    if (e != ELMFB_OK) return e;
    if (inf) {
      inf->ms_assemble = h->ms_assemble;
      inf->acond = -1.0;
      if (opts->estimate_cond && h->hist_k > 0) {
        double smax = 0.0, smin = 0.0;
        int32_t k = 0;
        if (elmfb_condition_estimate(h, &smax, &smin, &k) == ELMFB_OK && smin > 0.0)
          inf->acond = smax / smin;
      }
    }
  }
  return ELMFB_OK;
}

elmfb_status elmfb_time_gram_mv(elmfb_problem h, int32_t reps, double* ms_host, void* stream) {
  if (!h || !ms_host || reps < 1) return fail(h, ELMFB_E_INVALID, "bad argument");
  if (h->gram_prec < 0 || h->gram_which != 1)
    return fail(h, ELMFB_E_STATE, "time_gram_mv needs elmfb_gram(h, prec, 1) first");
  const elmfb_status es = gcg_prepare(h);
  if (es != ELMFB_OK) return es;
  hipStream_t s = (hipStream_t)stream;
  const Geo& g = h->geo;
  std::vector<double> ones((size_t)g.n_phi, 1.0);
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_w, ones.data(), (size_t)g.n_phi * 8, hipMemcpyHostToDevice, s));
  hipEvent_t e0, e1, e2;
  HIP_OR_FAIL(h, hipEventCreate(&e0));
  HIP_OR_FAIL(h, hipEventCreate(&e1));
  HIP_OR_FAIL(h, hipEventCreate(&e2));
  // pass 1 alone (pairs), then both passes (pairs + rows)
  hipError_t e = hipEventRecord(e0, s);
  for (int i = 0; i < reps && e == hipSuccess; ++i)
    e = launch_gram_mv_pairs_only(g, h->gram_prec, h->d_gcg_pairs, h->gram_npairs, h->d_G,
                                  h->d_w, h->d_gcg_part, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  for (int i = 0; i < reps && e == hipSuccess; ++i)
    e = gram_mv(h, h->d_w, h->d_vt, nullptr, red_slot(h, 0), s);
  if (e == hipSuccess) e = hipEventRecord(e2, s);
  if (e == hipSuccess) e = hipEventSynchronize(e2);
  float t01 = 0.f, t12 = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t01, e0, e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&t12, e1, e2);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipEventDestroy(e2);
  HIP_OR_FAIL(h, e);
  ms_host[0] = (double)t01 / reps;
  ms_host[1] = (double)t12 / reps;
  return ELMFB_OK;
}

}  // extern "C"
