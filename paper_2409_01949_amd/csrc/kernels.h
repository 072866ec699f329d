// Host-side launchers of the gfx950 kernels (one translation unit per kernel family).
#pragma once

#include "common.h"

namespace elmfb {

// Axis segment: the grid range one subdomain covers along one axis of one level.
struct AxisSeg {
  int32_t level, axis, j, m0, m1, tab_off;
};

// ---- assembly (k_assemble.hip)
hipError_t launch_axis_sums(const Geo& g, const int32_t* cov, double* lsum, hipStream_t s);
hipError_t launch_axis_tables(const Geo& g, const AxisSeg* segs, int n_segs, const int32_t* cov,
                              double* tab, hipStream_t s);
// writes the FP64 matrix into A and, if lo_prec is FP32 or BF16, its rounded copy into A_lo
hipError_t launch_assemble(const Geo& g, int lo_prec, const DevBlock* blocks, const Tile* tiles,
                           int64_t n_tiles, const double* tab, const double* W, const double* b,
                           double* A, void* A_lo, hipStream_t s);
hipError_t launch_rhs(const Geo& g, const double* f, double* h, int32_t* bad, hipStream_t s);
hipError_t launch_points(const Geo& g, double* xy, hipStream_t s);

// ---- block-sparse products (k_matvec.hip)
enum RowMode { ROW_STORE = 0, ROW_LSQR_U = 1, ROW_RESID = 2, ROW_STORE_SQ = 3 };
enum ColMode { COL_STORE = 0, COL_LSQR_V = 1, COL_STORE_SQ = 2 };

// stage 1 of y = A v: per block point t[p] = sum_k A[k][p] v[q0+k] * (*vscale)
hipError_t launch_mv_blocks(const Geo& g, int prec, const DevBlock* blocks, const Tile* tiles,
                            int64_t n_tiles, const void* A, const double* v, const double* vscale,
                            double* tpart, const SolveState* st, hipStream_t s);
// stage 2: y[r] = sum over covering blocks of t, then the row epilogue; partial sums of squares
// into red[0..n_wg)
hipError_t launch_gather_rows(const Geo& g, const DevBlock* blocks, const int32_t* cov,
                              const double* tpart, int mode, double* out, const double* bvec,
                              const SolveState* st, double* red, int n_wg, hipStream_t s);
// stage 1 of x = A^T u: per chunk partial dot products [n_chunks][K]
hipError_t launch_rmv_chunks(const Geo& g, int prec, const DevBlock* blocks, const Tile* chunks,
                             int64_t n_chunks, const void* A, const double* u,
                             const double* uscale, double* part, const SolveState* st,
                             hipStream_t s);
// stage 2: x[q] = sum over the block's chunks, then the column epilogue
hipError_t launch_rmv_finish(const Geo& g, const int32_t* chunk_start, const double* part,
                             int mode, double* out, const SolveState* st, double* red, int n_wg,
                             hipStream_t s);
// the same with the soft-constraint rows bc [n_bc][n_phi] (NULL: none) applied to the rows
// n_rows.. of u, scaled by *uscale when given
hipError_t launch_rmv_finish(const Geo& g, const int32_t* chunk_start, const double* part,
                             int mode, double* out, const SolveState* st, double* red, int n_wg,
                             const double* bc, const double* u, const double* uscale,
                             hipStream_t s);
// Soft-constraint rows (k_bc.hip): assemble them (and their right-hand side entries h[n_rows..]),
// and their part of y = M v: rows n_rows.. of out in the given RowMode, one partial squared norm
// to *red (not for ROW_STORE)
hipError_t launch_bc_assemble(const Geo& g, const BcSpec& bc, const DevBlock* blocks,
                              const double* W, const double* b, double* Bm, double* h,
                              hipStream_t s);
hipError_t launch_bc_assemble_pts(const Geo& g, const DevBlock* blocks, const double* W,
                                  const double* b, double* Bm, double* h, hipStream_t s);
// workgroups of launch_bc_rows, each writing one norm partial
int bc_row_wgs(const Geo& g);
hipError_t launch_bc_rows(const Geo& g, const double* Bm, const double* v, const double* vscale,
                          int mode, double* out, const double* bvec, const SolveState* st,
                          double* red, hipStream_t s);
int rows_wg(const Geo& g);
int cols_wg(const Geo& g);

// ---- LSQR in one workgroup for systems that fit in LDS (k_persistent.hip): up to n_iter
// steps on the FP64 matrix, the state carried in st and the vectors u, v, w, x
constexpr size_t kPersistMaxLds = 65536;
constexpr int64_t kPersistMaxEntries = 1 << 17;   // stored entries the one CU re-reads per step
// LDS bytes of a launch, with or without the matrix copy of n_store entries
size_t persistent_lds_bytes(const Geo& g, int64_t n_pts, int64_t n_store, bool a_in_lds);
hipError_t launch_lsqr_persistent(const Geo& g, const DevBlock* blocks, const int32_t* cov,
                                  const double* A, const double* bc, double* u, double* v,
                                  double* w, double* x, SolveState* st, double* hist, int n_iter,
                                  int64_t n_pts, int64_t n_store, int* lds_mode, hipStream_t s);

// ---- Krylov recurrences (k_solver.hip)
hipError_t launch_sumsq(const double* x, int64_t n, double* red, int n_wg, hipStream_t s);
hipError_t launch_lsqr_init(SolveState* st, const double* red_b, int nb, const double* red_u,
                            int nu, hipStream_t s);
// hist (may be NULL): the (alpha, beta) pairs of the bidiagonalisation, kHistCap of them
hipError_t launch_lsqr_init_alpha(SolveState* st, const double* red, int n, double* hist,
                                  hipStream_t s);
hipError_t launch_init_xw(const Geo& g, const double* x0, double* x, double* w, const double* v,
                          const SolveState* st, hipStream_t s);
hipError_t launch_lsqr_beta(SolveState* st, const double* red, int n, double* hist,
                            hipStream_t s);
hipError_t launch_lsqr_alpha(SolveState* st, const double* red, int n, double* hist,
                             hipStream_t s);
hipError_t launch_lsqr_update(const Geo& g, double* x, double* w, const double* v,
                              const SolveState* st, double* red, int n_wg, hipStream_t s);
hipError_t launch_lsqr_stop(SolveState* st, const double* red, int n, hipStream_t s);
hipError_t launch_cgls_init(SolveState* st, const double* red_b, int nb, const double* red_r,
                            int nr, const double* red_s, int ns, double anorm_f, hipStream_t s);
hipError_t launch_copy(const double* src, double* dst, int64_t n, hipStream_t s);
hipError_t launch_cgls_step_a(SolveState* st, const double* red, int n, hipStream_t s);
hipError_t launch_cgls_update_x(const Geo& g, double* x, const double* p, const SolveState* st,
                                hipStream_t s);
hipError_t launch_cgls_update_r(const Geo& g, double* r, const double* t, const SolveState* st,
                                double* red, int n_wg, hipStream_t s);
hipError_t launch_cgls_step_b(SolveState* st, const double* red_r, int nr, const double* red_s,
                              int ns, hipStream_t s);
hipError_t launch_cgls_update_p(const Geo& g, double* p, const double* sv, const SolveState* st,
                                hipStream_t s);
hipError_t launch_sumsq_entries(int prec, const void* A, int64_t n, double* red, int n_wg,
                                hipStream_t s);
hipError_t launch_reduce_to(const double* red, int n, double* out, hipStream_t s);
hipError_t launch_axpy(double a, const double* x, double* y, int64_t n, hipStream_t s);

// ---- Gram blocks (k_gram.hip)
// y = G p from the stored upper Gram blocks (pass 1 per stored block into part [2 n_pairs][K],
// pass 2 per output coefficient with its block-row table row_ptr/idx); red gets p . y partials.
hipError_t launch_gram_mv(const Geo& g, int gram_prec, const GramPair* pairs, int64_t n_pairs,
                          const void* G, const int32_t* row_ptr, const int32_t* idx,
                          const double* p, double* part, double* y, const SolveState* st,
                          double* red, int n_wg, hipStream_t s);
hipError_t launch_gram_mv_pairs_only(const Geo& g, int gram_prec, const GramPair* pairs,
                                     int64_t n_pairs, const void* G, const double* p, double* part,
                                     hipStream_t s);
// CG on the Gram blocks (FP64 vectors and scalars).
hipError_t launch_gcg_init(SolveState* st, const double* red_b, int nb, const double* red_r,
                           int nr, const double* red_z, int nz, hipStream_t s);
hipError_t launch_gcg_alpha(SolveState* st, const double* red, int n, hipStream_t s);
hipError_t launch_gcg_update(const Geo& g, double* a, double* r, const double* p, const double* q,
                             const SolveState* st, double* red, int n_wg, hipStream_t s);
hipError_t launch_dot(const double* x, const double* y, int64_t n, const SolveState* st,
                      double* red, int n_wg, hipStream_t s);
hipError_t launch_gcg_beta(SolveState* st, const double* red_r, int nr, const double* red_z,
                           int nz, hipStream_t s);
hipError_t launch_gcg_pupdate(const Geo& g, double* p, const double* z, const SolveState* st,
                              int init, hipStream_t s);
hipError_t launch_gram(const Geo& g, int prec, const DevBlock* blocks, const GramPair* pairs,
                       const GramChunk* chunks, int64_t n_chunks, const int32_t* multi,
                       int64_t n_multi, const void* A, void* G, void* part, hipStream_t s);
size_t gram_smem_bytes(int prec, int K);

// ---- block-Jacobi preconditioner (k_precond.hip)
int bj_wg(const Geo& g);
hipError_t launch_bj_factor(const Geo& g, const double* G, const int64_t* diag_off, double shift,
                            double* work, double* rinv, double* rinvT, int32_t* nfail,
                            hipStream_t s);
hipError_t launch_bj_apply(const Geo& g, const double* rinvT, const double* v,
                           const double* scale, double* y, const SolveState* st, hipStream_t s);
hipError_t launch_bj_apply_t(const Geo& g, const double* rinv, const double* x, int mode,
                             double* out, const SolveState* st, double* red, hipStream_t s);
hipError_t launch_bj_recover(const Geo& g, const double* rinvT, const double* y, const double* x0,
                             double* x, hipStream_t s);

// ---- batches (k_batch.hip)
struct BSeg {
  AxisSeg s;
  int32_t inst;
  int32_t pad;
};
hipError_t launch_bt_tables(const Geo* geos, const BSeg* segs, int n_segs, const int32_t* cov,
                            double* tab, hipStream_t s);
hipError_t launch_bt_assemble(int lo_prec, const Geo* geos, const DevBlock* blocks,
                              const Tile* tiles, int64_t n_tiles, const double* tab,
                              const double* W, const double* b, double* A, void* A_lo,
                              hipStream_t s);
hipError_t launch_bt_rhs(const Geo* geos, const InstInfo* insts, const RowTile* rt, int64_t n_rt,
                         int R, const double* f, double* h, int32_t* bad, hipStream_t s);
// runs NULL: one workgroup per block (n_grid blocks); else one per run of <= 256 points (n_grid
// runs, blk = -1 for padding).  kmax: largest nk of the blocks (<= kPatchMaxK; sets the dynamic
// LDS of the coefficients)
hipError_t launch_bt_mvb(int prec, const DevBlock* blocks, const Tile* runs, int64_t n_grid,
                         int kmax, const void* A, const double* v, int R, const SolveState* st,
                         double* tpart, hipStream_t s, int fa = 8);
hipError_t launch_bt_gather(const Geo* geos, const InstInfo* insts, const DevBlock* blocks,
                            const int32_t* cov, const RowTile* rt, int64_t n_rt,
                            const double* tpart, int mode, int R, double* out, const double* bvec,
                            const SolveState* st, double* red, hipStream_t s, int rpt = 1);
// tp: points per LDS stage, one of kBtTileChoices (64 not for FP64)
// one workgroup per column slice; red receives per-slice partials
hipError_t launch_bt_rmvb(int prec, int tp, const Geo* geos, const InstInfo* insts,
                          const DevBlock* blocks, const ColSlice* slices, int64_t n_slices,
                          const void* A, const double* u, int R, const SolveState* st, int mode,
                          double* out, double* red, hipStream_t s);
// perm (may be NULL): original column of every column of the blocks' order (patch blocks)
hipError_t launch_bt_bj_recover(const DevBlock* blocks, int64_t n_blocks, const double* rc,
                                const int64_t* foff, const int32_t* perm, int R, const double* y,
                                const double* x0, double* x, hipStream_t s);
hipError_t launch_bt_axpy(int64_t n, const double* y, double* x, hipStream_t s);
hipError_t launch_bt_recover_plain(int64_t n, const double* y, const double* x0, double* x,
                                   hipStream_t s);
// two_panels: some task lies off the diagonal (blocks of more than 128 columns)
hipError_t launch_bt_gram_diag(const DevBlock* blocks, const GramTask* tasks, int64_t n_tasks,
                               bool two_panels, const double* A, const int64_t* goff, double* G,
                               hipStream_t s);
// blocks blk0 .. blk0 + n_blocks - 1; kmax: their largest nk (<= kBatchMaxK; sets the dynamic
// LDS of two packed triangles)
hipError_t launch_bt_bj_factor(const DevBlock* blocks, int blk0, int64_t n_blocks,
                               const double* G, const int64_t* goff, const int64_t* foff, int kmax,
                               double shift, double* rc, int32_t* nfail, hipStream_t s);
// blocks of up to kPatchMaxK columns: W scratch beside G (both nk x nk at goff); G is overwritten
hipError_t launch_bt_bj_factor_blocked(const DevBlock* blocks, int blk0, int64_t n_blocks,
                                       double* G, double* W, const int64_t* goff,
                                       const int64_t* foff, double shift, double* rc,
                                       int32_t* nfail, hipStream_t s);
// patch blocks (FP64, their own layout) from the subdomain blocks of the assembled M
hipError_t launch_bt_expand(const Geo* geos, const DevBlock* pblocks, const Tile* runs,
                            int64_t n_runs, const DevBlock* blocks, const int32_t* members,
                            const int32_t* moff, const double* A, double* Ap, hipStream_t s);
// full: rc holds R^{-1} as K x K row-major per block (foff unused); else column-packed at foff
// kmax: largest nk of the blocks (<= kPatchMaxK, <= 256 with full); runs of
// fold_run_points(kmax) points; Ahat may be NULL (low-precision result only) or A itself
int fold_run_points(int kmax);
hipError_t launch_bt_fold(int lo_prec, bool full, int kmax, const DevBlock* blocks,
                          const Tile* ftiles, int64_t n_ftiles, const double* A, const double* rc,
                          const int64_t* foff, double* Ahat, void* Ahat_lo, hipStream_t s);
// ot (may be NULL): outer state of a refined solve; pairs it marks done are frozen, the others
// stop their inner LSQR once its residual estimate is inner_rel times the outer target
hipError_t launch_bt_lsqr_init(SolveState* st, const InstInfo* insts, int n_inst, int R,
                               const double* red_b, const double* red_u, double atol, double btol,
                               int iter_lim, const BtOuter* ot, double inner_rel, hipStream_t s);
hipError_t launch_bt_outer_check(BtOuter* ot, const SolveState* st, const InstInfo* insts,
                                 int n_inst, int R, const double* red_r, const double* red_a,
                                 double atol, int mode, double btol, int outer_lim,
                                 hipStream_t s);
hipError_t launch_bt_count_outer(const BtOuter* ot, int n, int32_t* out, hipStream_t s);
hipError_t launch_bt_lsqr_init_alpha(SolveState* st, const InstInfo* insts, int n_inst, int R,
                                     const double* red, hipStream_t s);
hipError_t launch_bt_lsqr_beta(SolveState* st, const InstInfo* insts, int n_inst, int R,
                               const double* red, hipStream_t s);
hipError_t launch_bt_lsqr_alpha(SolveState* st, const InstInfo* insts, int n_inst, int R,
                                const double* red, hipStream_t s);
hipError_t launch_bt_update(const Geo* geos, const InstInfo* insts, const ColTile* ct, int64_t n_ct,
                            int R, double* x, double* w, const double* v, const SolveState* st,
                            double* red, hipStream_t s);
hipError_t launch_bt_lsqr_stop(SolveState* st, const InstInfo* insts, int n_inst, int R,
                               const double* red, hipStream_t s);
hipError_t launch_bt_count_active(const SolveState* st, int n, int32_t* out, hipStream_t s);
hipError_t launch_bt_pack(const InstInfo* insts, const int64_t* sizes, int n_inst, int R,
                          int64_t total, const double* src, double* dst, int to_interleaved,
                          int use_cols, hipStream_t s);

// ---- warm-start MLP (k_mlp.hip)
enum { MLP_EPI_F32 = 0, MLP_EPI_BIAS = 1, MLP_EPI_BIAS_TANH = 2, MLP_EPI_DTANH = 3 };
struct MlpGemm {
  int M, N, K;
  const uint16_t* A;       // A(m, k) = A[m sam + k sak], bfloat16 bits
  int64_t sam, sak;
  const uint16_t* B;       // B(k, n) = B[k sbk + n sbn]
  int64_t sbk, sbn;
  int epi;
  const float* bias;       // [N] (BIAS, BIAS_TANH)
  const uint16_t* act;     // [M][ldo] activations (DTANH)
  float* out_f32;          // F32, BIAS
  uint16_t* out_bf16;      // BIAS_TANH, DTANH
  int64_t ldo;
};
// ws: FP32 workspace of mlp_gemm_ws_floats(M, N, K) floats for split-k products (F32 epilogue
// only; NULL: no split)
int mlp_gemm_splits(int M, int N, int K);
int64_t mlp_gemm_ws_floats(int M, int N, int K);
hipError_t launch_mlp_gemm(const MlpGemm& p, float* ws, hipStream_t s);
hipError_t launch_mlp_to_bf16(int64_t n, const float* x, uint16_t* y, hipStream_t s);
hipError_t launch_mlp_loss(int64_t n, const float* y, const float* t, uint16_t* g, double* part,
                           int n_part, double* loss, hipStream_t s);
// part: mlp_colsum_chunks(M) x N floats of partial sums
int mlp_colsum_chunks(int M);
hipError_t launch_mlp_colsum(int M, int N, const uint16_t* g, float* part, float* db,
                             hipStream_t s);
hipError_t launch_mlp_modulate(int64_t n, int K, int n_mod, const float* z, const float* f,
                               float* y, hipStream_t s);
hipError_t launch_mlp_mod_loss(int64_t n, int K, int n_mod, const float* z, const float* f,
                               const float* t, uint16_t* gz, double* part, int n_part,
                               double* loss, hipStream_t s);
hipError_t launch_mlp_adam(int64_t n, float* prm, const float* grad, float* m1, float* m2,
                           uint16_t* pb, float lr, float b1, float b2, float eps, float c1,
                           float c2, hipStream_t s);

// ---- evaluation (k_evaluate.hip)
hipError_t launch_evaluate(const Geo& g, const double* W, const double* b, const double* coef,
                           const double* pts, int64_t n_pts, double* u, hipStream_t s);
hipError_t launch_check_rel_l2(const double* u, const double* ref, int64_t n, SolveState* st,
                               double* red, int n_wg, hipStream_t s);

}  // namespace elmfb
