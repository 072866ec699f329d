// Handle of one planned least-squares problem: host tables, device memory, solver state.
// Internal to the library (shared by the runtime translation units).
#pragma once

#include <map>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"

using namespace elmfb;

struct elmfb_problem_s {
  elmfb_problem_desc desc{};
  Geo geo{};
  std::string err;

  // host tables
  std::vector<DevBlock> blocks;
  std::vector<Tile> tiles, chunks;
  std::vector<int32_t> chunk_start, cov;
  std::vector<AxisSeg> segs;
  std::vector<int32_t> bmap;    // per level, (jx, jy) of the full grid -> kept block or -1
  std::vector<int32_t> block_pidx;   // per kept block: index among all subdomains (parameters)
  int n_sub_full = 0;           // subdomains of the full per-level grids
  int64_t n_lsum = 0;           // grid indices of the per-axis window-sum tables (L domain)
  int64_t nnz = 0, n_block_points = 0, n_tab = 0;
  int64_t n_store = 0;          // stored elements per matrix copy, row padding included
  int64_t bytes_device = 0;
  int64_t mem_cap = 0;          // ELMFB_MEM_CAP at definition (0: no cap)

  // device memory
  std::vector<void*> allocs;
  DevBlock* d_blocks = nullptr;
  Tile* d_tiles = nullptr;
  Tile* d_chunks = nullptr;
  int32_t* d_cstart = nullptr;
  int32_t* d_cov = nullptr;
  AxisSeg* d_segs = nullptr;
  double* d_tab = nullptr;
  double* d_W = nullptr;
  double* d_b = nullptr;
  double* d_A = nullptr;        // FP64 matrix (always)
  void* d_A_lo = nullptr;       // optional FP32/BF16 copy
  int lo_prec = ELMFB_FP64;     // FP64: no copy
  double* d_h = nullptr;
  double* d_tpart = nullptr;
  double* d_part = nullptr;
  double* d_red = nullptr;      // 4 * kRedBlocks * 2 partial sums
  double* d_u = nullptr;        // LSQR u / CGLS r
  double* d_t = nullptr;        // CGLS t = A p
  double* d_v = nullptr;        // LSQR v / CGLS s
  double* d_w = nullptr;        // LSQR w / CGLS p
  double* d_x = nullptr;
  double* d_vt = nullptr;       // n_phi scratch (preconditioned directions)
  double* d_xt = nullptr;       // n_phi scratch
  double* d_c = nullptr;        // n_phi: refinement iterate / recovered solution
  double* d_r = nullptr;        // n_rows: refinement residual
  double* d_scalar = nullptr;   // scratch scalar
  SolveState* d_state = nullptr;
  int32_t* d_flag = nullptr;
  double* d_bc = nullptr;       // soft-constraint rows, dense [n_bc][n_phi]
  double* d_bcpts = nullptr;    // Dirichlet points [n][2], then their values [n]
  int32_t* d_bmap = nullptr;    // block map
  double* d_lsum = nullptr;     // per-axis window sums of an L-shaped domain
  BcSpec bcs{};                 // their conditions
  double* d_hist = nullptr;     // (alpha_{i+1}, beta_{i+1}) of the last LSQR run, i < kHistCap
  int32_t hist_k = -1;          // steps of that run (-1: the last solve ran no LSQR)
  double* d_eval = nullptr;     // solution-check buffer
  int64_t eval_cap = 0;

  // Gram blocks
  std::vector<GramPair> pairs_all;      // every overlapping pair, i <= j
  std::vector<int64_t> diag_pair;       // per block: index of (j, j) in pairs_all
  int gram_prec = -1, gram_which = -1;
  int64_t gram_npairs = 0;
  void* d_G = nullptr;
  int64_t G_bytes = 0;
  void* d_gpart = nullptr;
  int64_t gpart_bytes = 0;
  GramPair* d_gpairs = nullptr;
  int64_t gpairs_cap = 0;
  GramChunk* d_gchunks = nullptr;
  int64_t gchunks_cap = 0;
  int32_t* d_gmulti = nullptr;
  int64_t gmulti_cap = 0;
  std::vector<GramPair> gram_pairs_host;   // the pairs of the last elmfb_gram call
  int64_t gram_gen = 0;                    // counts elmfb_gram calls
  int64_t gram_nchunks = 0, gram_nmulti = 0;   // tables of the last Gram launch

  // CG on the Gram blocks: device copy of the stored pairs, per block-row tables of partials,
  // partials [2 n_pairs][K], and one extra coefficient vector for the preconditioner
  int64_t gcg_gen = -1;                    // gram_gen the tables were built for
  GramPair* d_gcg_pairs = nullptr;
  int32_t* d_gcg_rowptr = nullptr;
  int32_t* d_gcg_idx = nullptr;
  double* d_gcg_part = nullptr;
  double* d_gcg_tmp = nullptr;

  // block-Jacobi factors
  double* d_bj_work = nullptr;
  double* d_rinv = nullptr;
  double* d_rinvT = nullptr;
  int64_t* d_diag_off = nullptr;
  bool bj_ready = false;
  // the preconditioner folded into the matrix: M R^{-1} in FP64 (folded64) and its store_prec
  // rounding (folded_lo), each formed when device memory allows
  bool folded64 = false, folded_lo = false;
  double* d_Ahat = nullptr;
  void* d_Ahat_lo = nullptr;
  Tile* d_ftiles = nullptr;
  int64_t n_ftiles = 0;

  bool assembled = false;
  int n_rhs = 1;                // right-hand sides of the last assembly
  double* d_hs = nullptr;       // [n_rhs][n_rows + n_bc] when n_rhs > 1
  int64_t hs_cap = 0;           // doubles held by d_hs
  double ms_assemble = 0.0;     // host wall time of the last assembly
  int persist_lds_mode = -1;    // one-workgroup LSQR: 1 matrix in LDS, 0 vectors only, -1 undecided
  double anorm_f = -1.0;        // exact Frobenius norm of the stored matrix (lazy)
  hipStream_t stream = nullptr; // internal stream for captured solves
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::map<std::vector<int64_t>, hipGraphExec_t> graphs;   // captured iteration loops
};

namespace elmfb {

elmfb_status fail(elmfb_problem h, elmfb_status code, const std::string& msg);

#define HIP_OR_FAIL(h, expr)                                                             \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::elmfb::fail((h), ELMFB_E_DEVICE,                                          \
                           std::string(#expr) + ": " + hipGetErrorString(e_));           \
  } while (0)

inline int64_t elem_size(int prec) { return prec == ELMFB_FP64 ? 8 : (prec == ELMFB_FP32 ? 4 : 2); }

hipError_t dalloc_bytes(elmfb_problem h, void** p, int64_t bytes);
template <typename T>
hipError_t dalloc(elmfb_problem h, T** p, int64_t bytes) {
  void* q = nullptr;
  hipError_t e = dalloc_bytes(h, &q, bytes);
  if (e == hipSuccess) *p = static_cast<T*>(q);
  return e;
}
void dfree(elmfb_problem h, void* p);

// Looks up this device's address of the fixed scratch array of elmfb_rmatvec_noalloc (once per
// device; the current device must be the handle's).
hipError_t noalloc_init_device();

// Descriptor checks and the host-side decomposition plan of one problem (no device work).
std::string validate_desc(const elmfb_problem_desc* d);
std::string plan_problem(elmfb_problem h);
// the library's draw of W, b for a descriptor without them (elmfb_draw_features)
int64_t feature_param_count(const elmfb_problem_desc& d);
void draw_feature_params(const elmfb_problem_desc& d, double* W, double* b);

}  // namespace elmfb
