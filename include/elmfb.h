/*
 * elmfb.h -- C ABI of the MI355X (gfx950) multilevel ELM-FBPINN least-squares library.
 *
 * The library assembles and solves the structured linear least-squares system of a
 * multilevel ELM-FBPINN (Sec. 3 of "ELM-FBPINNs: An Efficient Multilevel Random Feature
 * Method"):   min_a || M a - h ||,   M = sum_l sum_j V_j^T M_j W_j   (eq. multilevel_ls,
 * eq. multilevel_domain_decomp), for a linear operator on a box domain with a regular
 * collocation grid, L levels of overlapping subdomains with partition-of-unity windows
 * (Sec. 4.1, eq. window_func) and K fixed random tanh features per subdomain.
 *
 * Conventions for every entry point:
 *   - Every call returns an elmfb_status; 0 is success.  No C++ exception crosses the ABI.
 *     On failure elmfb_last_error(handle) (or elmfb_last_error(NULL) for calls that failed
 *     before a handle existed) returns a message; the message lives until the next failing
 *     call on the same thread.
 *   - Pointers named *_dev are device pointers (hipMalloc'ed or any device allocation, for
 *     example a torch tensor's data pointer) owned by the caller.  They must stay valid until
 *     the work enqueued on the given stream has completed.  The library never frees them.
 *   - Pointers named *_host are host pointers owned by the caller, read during the call only.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.  Calls enqueue
 *     their device work on that stream.  elmfb_solve blocks the host at its check points
 *     (it reads the stopping state back), every other call is asynchronous.
 *   - Arguments are checked before any device work is enqueued; a rejected call changes
 *     nothing.  Device failures map to ELMFB_E_DEVICE with the HIP error text.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Row order of every vector over collocation points is x-major (row n = ix*ny + iy);
 *     column (coefficient) order is q = sum_{m<l} J_m K + j K + k with the subdomain index
 *     j = jx*Jy + jy (Sec. 3 "Indexing conventions", 0-based here).
 */
#ifndef ELMFB_H_
#define ELMFB_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ELMFB_ABI_VERSION 5
#define ELMFB_MAX_LEVELS 8
#define ELMFB_MAX_BC 4
#define ELMFB_MAX_BC_PTS 4096

typedef int32_t elmfb_status;
enum {
  ELMFB_OK = 0,
  ELMFB_E_INVALID = 1,     /* bad argument or descriptor                                    */
  ELMFB_E_NOMEM = 2,       /* device footprint does not fit (checked before allocating)      */
  ELMFB_E_DEVICE = 3,      /* HIP runtime failure or no usable gfx950 device                 */
  ELMFB_E_STATE = 4,       /* call out of order (e.g. solve before assemble)                 */
  ELMFB_E_NUMERIC = 5,     /* non-finite input values                                        */
  ELMFB_E_UNSUPPORTED = 6  /* valid but not implemented combination                          */
};

/* Linear operators N of the PDE N[u] = f (Sec. 3 "Problem and model definition"). */
enum {
  ELMFB_OP_D1 = 1,          /* du/dx, dim = 1                                                */
  ELMFB_OP_NEG_LAPLACE = 2, /* -Laplace(u), dim = 2                                          */
  ELMFB_OP_IDENTITY = 3,    /* u itself (evaluation / projection matrices), dim 1 or 2       */
  ELMFB_OP_OSCILLATOR = 4,  /* m u'' + mu u' + k u, (m, mu, k) = op_coef, dim 1 (Sec. 4.2
                               eq. harm_oscillator)                                        */
  ELMFB_OP_HELMHOLTZ = 5    /* Laplace(u) + k^2 u, k^2 = op_coef[0], dim 2 (Sec. 4.4
                               eq. helmholtz_problem)                                      */
};

/* Domains (dim 2).  ELMFB_DOMAIN_L is the box without its upper-right quarter
 * Q = (mid_x, hi_x] x (mid_y, hi_y], mid = (lo + hi)/2 (Sec. 4.4 eq. helmholtz_problem):
 *   - the collocation rows are the grid points outside Q; row-space vectors keep the full grid
 *     (row n = ix*ny + iy), and the rows of grid points in Q are identically zero (matrix and
 *     right-hand side), so they do not change the least-squares problem; the row scale is
 *     1/sqrt(N_I) with N_I the number of grid points outside Q;
 *   - a subdomain whose centre lies in Q is discarded (Sec. 4.1: rectangular subdomains outside
 *     the L are dropped; 16 x 16 keeps 192, 8 x 8 keeps 48); the kept ones are numbered in level,
 *     then x-major order, and each window is normalised over the kept subdomains of its level;
 *   - W_host / b_host still hold the parameters of every subdomain of each level's full
 *     J_x x J_y grid (in that full order); the library takes the kept subdomains' rows. */
enum { ELMFB_DOMAIN_BOX = 0, ELMFB_DOMAIN_L = 1 };

/* Inputs of the random features (Sec. 3: a shallow network per subdomain; the paper does not
 * state how its inputs are scaled).  LOCAL: xbar = (x - mu_j)/sigma_l, the subdomain's own
 * coordinates; GLOBAL: xbar = x. */
enum { ELMFB_INPUT_LOCAL = 0, ELMFB_INPUT_GLOBAL = 1 };

/* Hard-constraint factor C(x) multiplying the network (Sec. 4.3 "Hard boundary constraints"). */
enum {
  ELMFB_ANSATZ_NONE = 0,        /* C = 1                                                     */
  ELMFB_ANSATZ_TANH_ORIGIN = 1, /* C = tanh(w x), dim 1: u(0) = 0                            */
  ELMFB_ANSATZ_TANH_BOX = 2     /* C = prod_i tanh(w (x_i - lo_i)) tanh(w (hi_i - x_i))      */
};

/* Storage precisions.  ELMFB_FP16 is IEEE binary16 (11 significant bits, finite range
 * +-65504): meant for the block-Jacobi-folded matrix M R^{-1}, whose columns have norm <= 1. */
enum { ELMFB_FP64 = 0, ELMFB_FP32 = 1, ELMFB_BF16 = 2, ELMFB_FP16 = 3 };

/* Or'd into the precision argument of elmfb_copy_blocks / elmfb_batch_copy_blocks: copy the
 * block-Jacobi-folded matrix M R^{-1} (FP64) or its low-precision rounding instead of M. */
#define ELMFB_COPY_FOLDED 0x100

/* Solvers (Sec. 4.1 "Optimisation and solvers": LSQR; the others are alternatives on the
 * same matrix). */
enum {
  ELMFB_LSQR = 0,       /* Paige-Saunders LSQR on block-sparse A v / A^T u, FP64 recurrences  */
  ELMFB_CGLS = 1,       /* CG on the normal equations in factored form, FP64                 */
  ELMFB_MIXED_IR = 2,   /* FP64 iterative refinement: r = h - A c with the FP64 matrix, the
                           correction from inner_iters LSQR steps on the stored FP32/BF16/FP16
                           copy (FP64 vectors and recurrences), c += d in FP64; outer_lim
                           steps (istop 7), fewer when the inner solve stops before its first
                           step (r = 0 or A^T r = 0: istop 0)                                 */
  ELMFB_NORMAL_CG = 3,  /* CG on the normal equations G a = M^T h with G the Gram blocks of
                           elmfb_gram(h, prec, 1) (FP64 or FP32 entries; FP64 vectors and
                           scalars); precond = 1: block-Jacobi PCG, z = R^{-1} R^{-T} r        */
  ELMFB_MIXED_IR_CG = 4 /* FP64 iterative refinement with the correction d from inner_iters CG
                           steps on the stored Gram blocks: r = h - M c, g = M^T r (FP64),
                           G d = g, c += d                                                    */
};

typedef struct elmfb_problem_s* elmfb_problem;

/* Problem descriptor.  The grid has n_points[a] points per axis, endpoints included:
 * x_m = lo + m*((hi-lo)/(n-1)), last point = hi.  Level l has J[l][a] subdomains along axis a
 * with centres lo + j*h, h = (hi-lo)/(J-1), and half-width delta*h/2 (J = 1: the whole axis,
 * window factor 1).  For dim = 1 the second entries of lo/hi/n_points/J are ignored.
 * W_host [n_phi][dim] and b_host [n_phi] are the fixed hidden weights and biases of the
 * random features tanh(W_q . xbar + b_q) (xbar per input_norm), in column order q; with both
 * NULL the library draws them from `seed` (elmfb_draw_features). */
typedef struct {
  int32_t abi_version;               /* must be ELMFB_ABI_VERSION                            */
  int32_t dim;                       /* 1 or 2                                               */
  int32_t op;                        /* ELMFB_OP_*                                           */
  int32_t ansatz;                    /* ELMFB_ANSATZ_*                                       */
  double ansatz_omega;               /* w of the hard-constraint factor                      */
  double lo[2], hi[2];               /* domain box, lo < hi                                  */
  int32_t n_points[2];               /* >= 2 per used axis                                   */
  int32_t n_levels;                  /* 1..ELMFB_MAX_LEVELS                                  */
  int32_t J[ELMFB_MAX_LEVELS][2];    /* subdomains per axis per level, >= 1                  */
  double delta;                      /* width ratio, > 0                                     */
  int32_t K;                         /* features per subdomain, 1..256                       */
  int32_t store_prec;                /* extra low-precision copy of the matrix for inner
                                        solves: ELMFB_FP32 or ELMFB_BF16 (rounded to nearest
                                        even from FP64); ELMFB_FP64 = no copy.  The FP64
                                        matrix is always stored.                            */
  const double* W_host;              /* [n_phi][dim]                                         */
  const double* b_host;              /* [n_phi]                                              */
  double op_coef[3];                 /* ELMFB_OP_OSCILLATOR: (m, mu, k); ignored otherwise    */
  /* Soft-constraint rows (Sec. 3 "Definition of the system matrices", matrix B), dim 1 only:
   * condition b adds the row sqrt(lambda_b) (1/L) D^order_b[omega_j phi_q C](x_b) with right-hand
   * side sqrt(lambda_b) g_b (one point per condition, N_B^(b) = 1).  They follow the N_I
   * collocation rows: rows N_I .. N_I + n_bc - 1 of every row-space vector.  Only the FP64
   * LSQR and CGLS solves accept them (the Gram, block-Jacobi and refinement paths return
   * ELMFB_E_UNSUPPORTED). */
  int32_t n_bc;                      /* 0..ELMFB_MAX_BC                                      */
  int32_t bc_order[ELMFB_MAX_BC];    /* 0: the value, 1: the first derivative at x_b         */
  double bc_x[ELMFB_MAX_BC];         /* x_b, inside [lo, hi]                                 */
  double bc_weight[ELMFB_MAX_BC];    /* sqrt(lambda_b) > 0                                   */
  double bc_value[ELMFB_MAX_BC];     /* g_b                                                  */
  /* ABI 3 */
  int32_t domain;                    /* ELMFB_DOMAIN_BOX or ELMFB_DOMAIN_L (dim 2)           */
  /* Dirichlet rows at given points of a 2D problem (Sec. 3 matrix B; the boundary term
   * lambda_bc (1/N_B) sum_b (u(x_b) - g_b)^2 of the Helmholtz loss, Sec. 4.4): row b is
   * bc_pts_weight (1/L) omega_j(x_b) phi_q(x_b) C(x_b) with right-hand side bc_pts_weight g_b
   * (bc_pts_weight = sqrt(lambda_bc / N_B) reproduces that loss).  They follow the collocation
   * rows like the 1D conditions and take the same paths (FP64 LSQR and CGLS only). */
  int32_t n_bc_pts;                  /* 0..ELMFB_MAX_BC_PTS (dim 2, with n_bc = 0)          */
  const double* bc_pts_host;         /* [n_bc_pts][2], inside the box                       */
  const double* bc_pts_val_host;     /* [n_bc_pts] g_b                                      */
  double bc_pts_weight;              /* > 0                                                 */
  /* ABI 4 */
  int32_t input_norm;                /* ELMFB_INPUT_LOCAL or ELMFB_INPUT_GLOBAL              */
  uint64_t seed;                     /* stream of the drawn W, b (W_host = b_host = NULL)    */
  double w_range[2], b_range[2];     /* W ~ U[w_range[0], w_range[1]), b ~ U[b_range...)
                                        when drawn; lo <= hi, finite                         */
} elmfb_problem_desc;

typedef struct {
  int64_t n_rows;          /* grid points (row-space length before the soft-constraint rows) */
  int64_t n_phi;           /* columns N_Phi = K * sum_l prod_a J[l][a]                       */
  int64_t nnz;             /* stored entries = K * sum_j |I_j|                               */
  int64_t n_blocks;        /* subdomains over all levels                                    */
  int64_t n_block_points;  /* sum_j |I_j|                                                   */
  int64_t bytes_device;    /* device memory held by the handle                              */
  int64_t n_pairs;         /* overlapping subdomain pairs (i <= j), all levels               */
  int64_t n_bc;            /* soft-constraint rows (the 1D conditions or the Dirichlet rows at
                              points); row-space vectors hold n_rows + n_bc                    */
  int64_t n_interior;      /* collocation rows that belong to the domain (n_rows on a box)   */
} elmfb_sizes;

typedef struct {
  int32_t method;          /* ELMFB_LSQR | ELMFB_CGLS                                       */
  int32_t iter_lim;        /* maximum iterations (>= 0)                                     */
  int32_t check_every;     /* iterations per captured graph replay / host check, >= 1       */
  int32_t use_graph;       /* 1: capture the iteration loop in a hipGraph and replay it     */
  int32_t precond;         /* 1: right block-Jacobi preconditioning (LSQR and MIXED_IR);
                              needs elmfb_precondition first                               */
  int32_t inner_iters;     /* MIXED_IR: LSQR steps per refinement step (>= 1)               */
  int32_t outer_lim;       /* MIXED_IR: maximum refinement steps (>= 0)                     */
  double atol, btol;       /* Paige-Saunders stopping tolerances (>= 0); conlim is off      */
  const double* x0_dev;    /* optional warm start [n_rhs][n_phi] (NULL: zero)               */
  /* optional stop on the solution error: every check_every iterations u_tilde is evaluated
   * at check_pts_dev [n_check][dim] and the solve stops once
   * ||u - check_ref|| / ||check_ref|| <= target_rel_l2 (check_ref_dev [n_rhs][n_check]).
   * n_check = 0 disables it. */
  const double* check_pts_dev;
  const double* check_ref_dev;
  int64_t n_check;
  double target_rel_l2;
  /* ABI 3 */
  int32_t n_rhs;           /* right-hand sides solved with the assembled matrix, 1 (also for
                              0) up to the n_rhs of the last elmfb_assemble                  */
  int32_t estimate_cond;   /* 1: fill info.acond (host bisection on the recorded bidiagonal,
                              O(60 k) operations for k LSQR steps)                          */
} elmfb_solve_opts;

typedef struct {
  int32_t istop;           /* 0 x0 exact, 1 ||r|| test, 2 ||A^T r|| test, 4/5 the same at
                              machine precision, 7 iteration limit, 8 rel-L2 target reached */
  int32_t iters;           /* Krylov iterations (MIXED_IR: inner iterations in total)       */
  int32_t outer_iters;     /* MIXED_IR refinement steps                                     */
  double rnorm;            /* ||h - A x|| (LSQR estimate / CGLS recurrence; MIXED_IR: of the
                              returned coefficients, recomputed with the FP64 matrix)         */
  double arnorm;           /* ||A^T (h - A x)||                                              */
  double anorm;            /* LSQR Frobenius-norm estimate; CGLS: exact ||A||_F              */
  double xnorm;            /* ||x||                                                          */
  double rel_l2;           /* last rel-L2 check value (-1 if none ran)                      */
  double ms_solve;         /* host wall time of this right-hand side's solve                 */
  /* ABI 3 */
  double acond;            /* with opts.estimate_cond: sigma_max / sigma_min of the Golub-Kahan
                              bidiagonal of the last LSQR run (a lower bound on the condition
                              number of the operator it ran on; see elmfb_condition_estimate);
                              otherwise, or without an LSQR step, -1                         */
  double ms_assemble;      /* host wall time of the last elmfb_assemble                      */
} elmfb_solve_info;

/* Validate the descriptor, plan the decomposition (subdomain boxes on the grid, offsets),
 * check the device footprint against free memory and against the environment variable
 * ELMFB_MEM_CAP (bytes, if set and > 0; ELMFB_E_NOMEM before any allocation), allocate the
 * handle's device memory and upload W, b and the tables.  Needs a gfx950 device
 * (ELMFB_E_DEVICE otherwise).  Sec. 3, Sec. 4.1. */
elmfb_status elmfb_define_problem(const elmfb_problem_desc* desc, elmfb_problem* out);

/* The random-feature parameters the library draws for `desc` (Sec. 3: W and b fixed at random;
 * the generator is not stated): for parameter q of the full per-level subdomain grids (level,
 * then subdomain in x-major order, then feature k; the layout of W_host and b_host),
 * W[q][a] = U(4q + a) over w_range and b[q] = U(4q + 3) over b_range, where U(c) is
 * lo + (hi - lo) ((z >> 11) 2^-53) and z the SplitMix64 output (Steele, Lea and Flood 2014)
 * of state seed + (c + 1) 0x9e3779b97f4a7c15 (mod 2^64), each operation rounded on its own.
 * W_host [n_params][dim] and b_host [n_params] are caller-owned host arrays with
 * n_params = K sum_l prod_a J[l][a]; only the geometry fields, seed and ranges of desc are read.
 * Returns ELMFB_E_INVALID for NULL pointers, bad levels or ranges. */
elmfb_status elmfb_draw_features(const elmfb_problem_desc* desc, double* W_host, double* b_host);

/* Sizes of the planned system: rows (Sec. 3 "Problem and model definition", the collocation
 * points), columns N_Phi = K sum_l J_l (Sec. 3 "Indexing conventions"), stored entries of the
 * blocks M_j over I_j x K_j (Sec. 3 eq. multilevel_domain_decomp), overlapping pairs. */
elmfb_status elmfb_query(elmfb_problem h, elmfb_sizes* out_host);

/* The regular collocation grid [n_rows][dim] in row order, computed on the device (Sec. 4.1:
 * regularly spaced collocation points; both endpoints included). */
elmfb_status elmfb_points(elmfb_problem h, double* xy_dev, void* stream);

/* Assemble every block M_j [K][|I_j|] (feature-major) of the system matrix in the stored
 * precision and the right-hand sides h_r = f_r/sqrt(N_I) from f_dev [n_rhs][n_rows] (Sec. 3
 * "Definition of the vectors" and "Definition of the system matrices"):
 *     M_{n,q} = Op[C omega_j phi_q](x_n) / (sqrt(N_I) L).
 * The matrix is assembled once for all n_rhs (1..1024) right-hand sides, which elmfb_solve
 * then solves with it.  Entries are computed in FP64 and rounded once (round-to-nearest-even)
 * to the stored precision.  ELMFB_E_NUMERIC if f holds a non-finite value (checked on the
 * device).  Synchronises the stream (its wall time is reported as info.ms_assemble). */
elmfb_status elmfb_assemble(elmfb_problem h, const double* f_dev, int32_t n_rhs, void* stream);

/* y_dev [n_rows + n_bc] = M v_dev [n_phi] (block-sparse, Sec. 3 eq. multilevel_domain_decomp;
 * the soft-constraint rows follow the collocation rows). */
elmfb_status elmfb_matvec(elmfb_problem h, const double* v_dev, double* y_dev, void* stream);

/* x_dev [n_phi] = M^T u_dev [n_rows + n_bc]. */
elmfb_status elmfb_rmatvec(elmfb_problem h, const double* u_dev, double* x_dev, void* stream);

/* x_dev [n_phi] = M^T u_dev [n_rows + n_bc] exactly as elmfb_rmatvec computes it (the same
 * kernels and summation order: bit-identical results), for callers that cannot allocate device
 * memory -- code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The call allocates nothing: its per-chunk partial sums (one double per feature and per chunk
 * of <= 2048 points of a subdomain) live in a fixed scratch array of 2^18 doubles (2 MiB) that
 * the library holds on every device it runs on until the process ends (its address on a device
 * is looked up by elmfb_define_problem).  A problem needing more partials than that is refused
 * with ELMFB_E_UNSUPPORTED before any device work (use elmfb_rmatvec).  Every call on one device
 * shares that device's array: calls that overlap on one device (other streams, other threads)
 * race and must be serialised by the caller.  Asynchronous on `stream`. */
elmfb_status elmfb_rmatvec_noalloc(elmfb_problem h, const double* u_dev, double* x_dev,
                                   void* stream);

/* Copy the assembled right-hand sides h [n_rhs][n_rows + n_bc] (FP64; Sec. 3 "Definition of
 * the vectors": f/sqrt(N_I), then the soft-constraint values). */
elmfb_status elmfb_copy_rhs(elmfb_problem h, double* h_dev, void* stream);

/* Copy the soft-constraint rows B [n_bc][n_phi] (FP64, dense; nothing when n_bc = 0; Sec. 3
 * "Definition of the system matrices", the matrix B). */
elmfb_status elmfb_copy_bc(elmfb_problem h, double* dst_dev, void* stream);

/* Copy the stored blocks of the FP64 matrix (prec = ELMFB_FP64) or of its low-precision copy
 * (prec = the descriptor's store_prec) as raw values, blocks in column order, each [K][|I_j|]
 * with the block's points in row-major order of its box, into dst_dev; and the block table
 * into table_host [n_blocks][8] as int64: level, jx, jy, ix0, nx, iy0, ny, element offset.
 * prec | ELMFB_COPY_FOLDED copies the folded M R^{-1} of elmfb_precondition in that precision
 * instead (ELMFB_E_STATE if it was not formed).  Either pointer may be NULL.  (The blocks M_j of
 * Sec. 3 eq. multilevel_domain_decomp, M = sum_j V_j^T M_j W_j.) */
elmfb_status elmfb_copy_blocks(elmfb_problem h, int32_t prec, void* dst_dev, int64_t* table_host,
                               void* stream);

/* Solve min ||M x - h|| (Sec. 3 eq. multilevel_ls) into coef_dev [n_phi].  LSQR follows
 * Paige & Saunders (damp 0, no condition limit, stop tests on ||r|| and ||A^T r||), as the
 * method's reference solver does (Sec. 4.1).  Non-convergence is not an error: istop = 7.
 * ELMFB_NORMAL_CG and ELMFB_MIXED_IR_CG solve the normal equations G a = M^T h (the least-squares
 * minimiser when M has full column rank) on the Gram blocks of the last elmfb_gram(h, prec, 1)
 * call (ELMFB_E_STATE without it); CG stops when ||g - G a|| <= btol ||g|| (istop 1), on a
 * breakdown p.Gp <= 0 (istop 3: G is not positive definite in its stored precision) or after
 * iter_lim (inner_iters) steps (istop 7); rnorm then reports ||g - G a||, except for the
 * refinements, which report the FP64 residual ||h - M c||.  x0_dev warm-starts ELMFB_NORMAL_CG.
 * FP64 LSQR without block-Jacobi on a system whose vectors fit in 64 KB of LDS (at most 2^17
 * stored entries) runs check_every steps per launch in one workgroup; the environment variable
 * ELMFB_PERSISTENT=0 selects the multi-workgroup steps instead (same iteration, other summation
 * order).  info_host may be NULL. */
elmfb_status elmfb_solve(elmfb_problem h, const elmfb_solve_opts* opts, double* coef_dev,
                         elmfb_solve_info* info_host, void* stream);

/* Gram blocks G_ij = M_i^T M_j over the rows shared by subdomains i and j (the normal
 * equations of Sec. 3 eq. multilevel_ls restricted by eq. multilevel_domain_decomp), computed
 * on the matrix cores from the matrix copy of precision `prec` (ELMFB_FP64: the FP64 matrix,
 * FP64 products; ELMFB_FP32 / ELMFB_BF16: the stored low-precision copy, FP32 accumulation).
 * which = 0: diagonal blocks only; 1: every overlapping pair i <= j.  The blocks are held by
 * the handle (FP64 or FP32) until the next elmfb_gram call. */
elmfb_status elmfb_gram(elmfb_problem h, int32_t prec, int32_t which, void* stream);

/* elmfb_gram, then the same Gram computation `reps` more times between HIP events on `stream`:
 * ms_host = the average duration of one computation (all its kernels), flops_host (may be NULL)
 * = 2 K^2 times the shared points summed over the computed pairs (the useful MFMA work; K is
 * padded to 16 on the matrix cores).  The stored blocks are those of elmfb_gram afterwards.
 * Blocks the host until the timing completes.  (Measurement support for the Gram blocks of the
 * normal equations of Sec. 3 eq. multilevel_ls.) */
elmfb_status elmfb_time_gram(elmfb_problem h, int32_t prec, int32_t which, int32_t reps,
                             double* ms_host, double* flops_host, void* stream);

/* Copy the Gram blocks of the last elmfb_gram call (n_pairs x K x K values, FP64 for
 * prec = FP64 else FP32, row index = feature of i) into dst_dev and the pair table
 * [n_pairs][3] (bi, bj, element offset) into pairs_host; *n_pairs_host receives the count.
 * Either pointer may be NULL.  (G_ij = M_i^T M_j over the shared rows, Sec. 3
 * eq. multilevel_domain_decomp.) */
elmfb_status elmfb_copy_gram(elmfb_problem h, void* dst_dev, int64_t* pairs_host,
                             int64_t* n_pairs_host, void* stream);

/* Build the block-Jacobi preconditioner used by opts.precond: for every subdomain the upper
 * Cholesky factor R_j of G_jj + lambda_j I, lambda_j = shift * trace(G_jj)/K, from FP64 Gram
 * blocks, and R_j^{-1}.  A block that does not factor is retried with 100x the shift up to 8
 * times, then replaced by the identity; *n_fallback_host (may be NULL) receives that count.
 * The preconditioned matrix M R^{-1} is also formed once (FP64 matrix cores): its store_prec
 * rounding (4 or 2 nnz bytes) for the inner solves of ELMFB_MIXED_IR and the FP64 matrix (8 nnz
 * bytes) for FP64 solves, each when it fits in free device memory with an 8 GB margin and,
 * under the ELMFB_MEM_CAP of the definition, within the cap with the footprint;
 * preconditioned steps on a folded copy need no per-step R^{-1} products, the others apply R^{-1}
 * in every step.  M and its copy are unchanged.
 * A later elmfb_assemble discards the factors.  shift must be > 0.  Blocks until done. */
elmfb_status elmfb_precondition(elmfb_problem h, double shift, int32_t* n_fallback_host,
                                void* stream);

/* Conditioning of the system from the last solve's Krylov process (the paper reports kappa(M)
 * of its systems from the SVD, Sec. 4): LSQR's Golub-Kahan bidiagonalisation builds the
 * (k+1) x k lower bidiagonal B_k = U_{k+1}^T A V_k (alpha_1..alpha_k on the diagonal,
 * beta_2..beta_{k+1} below), whose singular values lie within those of the operator A it ran
 * on: sigma_max(B_k) grows toward sigma_max(A) and sigma_min(B_k) falls toward sigma_min(A), so
 * sigma_max / sigma_min is a lower bound on kappa(A) that tightens with k (in floating point
 * without reorthogonalisation the extreme values still converge; interior ones repeat).
 * A is M for ELMFB_LSQR, M R^{-1} with precond = 1, and for ELMFB_MIXED_IR the low-precision
 * operator of the last inner solve.  Every LSQR run records its first kHistCap = 32768 steps.
 * Writes sigma_max and sigma_min of B_k and k (may be NULL); ELMFB_E_STATE if the last solve
 * ran no LSQR step.  Blocks until done. */
elmfb_status elmfb_condition_estimate(elmfb_problem h, double* sigma_max_host,
                                      double* sigma_min_host, int32_t* k_host);

/* The same for a bidiagonal given on the host (no device work): ab_host[2i] = alpha_{i+1},
 * ab_host[2i + 1] = beta_{i+1} for i = 0..k (beta_1 is not used).  Extreme singular values by
 * bisection on the (2k+1) x (2k+1) Golub-Kahan matrix [0 B; B^T 0] in tridiagonal form, whose
 * eigenvalues are 0 and +-sigma_i: relative accuracy also for tiny sigma_min (Demmel and Kahan
 * 1990), down to 1e-300 sigma_max.  ELMFB_E_NUMERIC for an all-zero or non-finite input. */
elmfb_status elmfb_bidiag_sigma(const double* ab_host, int32_t k, double* sigma_max_host,
                                double* sigma_min_host);

/* u_dev [n_rhs][n_pts] = C(x) (1/L) sum_l sum_j omega_j(x) sum_k coef_q phi_q(x) at arbitrary
 * points pts_dev [n_pts][dim] for each of the n_rhs (>= 1) coefficient vectors coef_dev
 * [n_rhs][n_phi] (Sec. 3 eq. multilevel_solution with the hard-constraint factor). */
elmfb_status elmfb_evaluate(elmfb_problem h, const double* coef_dev, int32_t n_rhs,
                            const double* pts_dev, int64_t n_pts, double* u_dev, void* stream);

/* Time the kernels of the two products of one LSQR/CGLS iteration on `stream` with HIP events:
 * the per-block-point pass of y = M v, the per-chunk pass of x = M^T u, then the row gather that
 * completes y and the column pass that completes x (each writing its vector and its norm
 * partials, as in an LSQR step), each launched `reps` times back to back on the stored matrix
 * copy of precision `prec` (ELMFB_FP64 or the descriptor's store_prec), with v = 1, u = 1.
 * Writes the average duration of one launch in milliseconds to ms_host[0] (M v, first pass),
 * ms_host[1] (M^T u, first pass), ms_host[2] (gather) and ms_host[3] (column pass): ms_host
 * holds 4 doubles.  Overwrites the solver's work vectors.  Blocks the host until the timing
 * completes.  (Measurement support for the products of Sec. 3 eq. multilevel_domain_decomp.) */
elmfb_status elmfb_time_kernels(elmfb_problem h, int32_t prec, int32_t reps, double* ms_host,
                                void* stream);

/* ---- batches: many independent problems solved together -------------------------------- */

typedef struct elmfb_batch_s* elmfb_batch;

/* Define n independent problems (descs[i] as for elmfb_define_problem, every instance with
 * K <= 128 and the same store_prec), each with n_rhs (1..8) right-hand sides that share its
 * matrix.  Every kernel of the assembly and of the Krylov iteration then processes all instances
 * and right-hand sides in one launch (the instances are concatenated; row and column work comes
 * in tiles of one instance).  The footprint is checked before allocating (ELMFB_E_NOMEM). */
elmfb_status elmfb_define_batch(const elmfb_problem_desc* descs, int32_t n, int32_t n_rhs,
                                elmfb_batch* out);

/* offsets_host [n+1][2]: first global row and column of every instance, then the totals;
 * totals_host: summed sizes (n_pairs = 0).  Either may be NULL.  (The sizes of Sec. 3 per
 * instance, concatenated.) */
elmfb_status elmfb_batch_query(elmfb_batch b, int64_t* offsets_host, elmfb_sizes* totals_host);

/* Sizes of every instance: per_instance_host [n] (n_rows, n_phi, nnz, n_blocks, n_block_points,
 * n_interior as for a single problem; bytes_device = the instance's share of the stored matrix
 * entries and vectors; n_pairs = n_bc = 0). */
elmfb_status elmfb_batch_query_instances(elmfb_batch b, elmfb_sizes* per_instance_host);

/* Copy the stored blocks of every instance into dst_dev: prec = ELMFB_FP64 (M) or the batch's
 * store_prec (its rounded copy, until elmfb_batch_precondition replaces it), or either or'd with
 * ELMFB_COPY_FOLDED for the folded M_b R_b^{-1} in FP64 or its rounding (after
 * elmfb_batch_precondition; with patch factors, the patch blocks of
 * elmfb_batch_precondition_patches); ELMFB_E_STATE when that copy is not held.  Each block is
 * [K][nx*ny], points in row-major order of its box.  The block table goes into table_host
 * [n_blocks][8] as int64: instance, level, ix0, nx, iy0, ny, K (the block's columns), element
 * offset; blocks are ordered by instance, then by column; a folded copy of patch factors has
 * elmfb_batch_patch_info's block count.  Either pointer may be NULL. */
elmfb_status elmfb_batch_copy_blocks(elmfb_batch b, int32_t prec, void* dst_dev,
                                     int64_t* table_host, void* stream);

/* Assemble every instance (FP64 plus the store_prec copy) and h = f/sqrt(N_I) per right-hand
 * side.  f_dev holds instance i at f_dev + n_rhs*row_off_i as [n_rhs][n_rows_i]. */
elmfb_status elmfb_batch_assemble(elmfb_batch b, const double* f_dev, void* stream);

/* Y = M V for every instance and right-hand side, V at n_rhs*col_off_i as [n_rhs][n_phi_i] and
 * Y at n_rhs*row_off_i as [n_rhs][n_rows_i]; rmatvec: X = M^T U in the same layouts. */
elmfb_status elmfb_batch_matvec(elmfb_batch b, const double* v_dev, double* y_dev, void* stream);
elmfb_status elmfb_batch_rmatvec(elmfb_batch b, const double* u_dev, double* x_dev, void* stream);

/* Right block-Jacobi preconditioner for every block of every instance, as elmfb_precondition
 * does for one problem (Sec. 5 "Conditioning and redundancy" motivates it): the diagonal Gram
 * block G_b = M_b^T M_b (FP64, matrix cores), the Cholesky factor R_b of
 * G_b + shift trace(G_b)/K_b I and R_b^{-1}, then the preconditioned matrix M_b R_b^{-1} formed
 * once (FP64, matrix cores; its store_prec rounding replaces the low-precision copy of M), so
 * preconditioned Krylov steps cost what plain ones do.  shift in (0, 1).  n_fallback_host (may
 * be NULL) receives the number of blocks whose factorisation failed at every retry (100x larger
 * shift, 8 times) and got the identity.  Keeps 8 (nnz + sum_b K_b (K_b+1)/2) bytes on the device;
 * temporary: 16 sum_b K_b^2 bytes.  A later elmfb_batch_assemble discards it.  Synchronises
 * the stream. */
elmfb_status elmfb_batch_precondition(elmfb_batch b, double shift, int32_t* n_fallback_host,
                                      void* stream);

/* Block-Jacobi over patches: as elmfb_batch_precondition, with the blocks of the preconditioner
 * formed by `patch` (1..4) consecutive subdomains along each axis of a level (patch^d
 * neighbouring subdomains; the last patch along an axis keeps what is left), so the columns of
 * neighbouring subdomains, whose features nearly coincide on the shared points (the redundancy of
 * Sec. 5 "Conditioning and redundancy"), are orthonormalised together.  A patch block holds the
 * columns of its members, member by member in x-major order, on the bounding box of their boxes
 * (zero where a member's window vanishes); R_p is the Cholesky factor of
 * M_p^T M_p + shift trace(M_p^T M_p)/nk_p I (nk_p = the patch's columns, at most 512:
 * ELMFB_E_INVALID otherwise), and M_p R_p^{-1} is formed once in FP64 and in store_prec in the
 * patch layout (the low-precision copy of M itself is kept).  Preconditioned solves then run on
 * the patch blocks and return x = R^{-1} y; their coefficients y are in patch column order,
 * which elmfb_batch_patch_info reports.  patch = 1 is elmfb_batch_precondition.  Factors of one
 * patch size are held at a time.  Keeps 8 (dense + sum_p nk_p (nk_p+1)/2) bytes, plus the
 * store_prec copy, on the device (dense: stored entries of the patch blocks); temporary: up to
 * 4 GiB of Gram scratch, taken in chunks of patches.  Block-Jacobi coordinates
 * (elmfb_batch_set_coords) need patch = 1 (ELMFB_E_UNSUPPORTED).  Synchronises the stream. */
elmfb_status elmfb_batch_precondition_patches(elmfb_batch b, double shift, int32_t patch,
                                              int32_t* n_fallback_host, void* stream);

/* The patch size of the factors held (1 before any preconditioning) in patch_host, the number of
 * blocks of their folded matrix (patch blocks, or the subdomain blocks for patch 1) in
 * n_blocks_host, the entries elmfb_batch_copy_blocks copies of it in n_entries_host, and in
 * perm_host [n_phi] (int32, may be NULL) for every column of the patch column order its column
 * of x (the identity for patch 1).  Any pointer may be NULL.  (Bookkeeping of the preconditioner
 * above.) */
elmfb_status elmfb_batch_patch_info(elmfb_batch b, int32_t* patch_host, int64_t* n_blocks_host,
                                    int64_t* n_entries_host, int32_t* perm_host);

/* Time the candidate point-tile sizes (16, 32, 64 points per LDS stage) of the batched M^T U
 * pass on the assembled matrix copy of precision `prec` (ELMFB_FP64 or the batch's store_prec),
 * `reps` launches each (1..1000), and keep the fastest for later solves of that precision.
 * ms_host [3] (may be NULL) receives the average milliseconds per launch (-1: not available for
 * this precision; FP64 has no 64-point variant); chosen_host (may be NULL) the tile kept.
 * Overwrites the solver's work vectors; synchronises. */
elmfb_status elmfb_batch_autotune(elmfb_batch b, int32_t prec, int32_t reps, double* ms_host,
                                  int32_t* chosen_host, void* stream);

/* Time the three matrix passes of one batched Krylov step on `stream` with HIP events, each
 * launched `reps` times (1..1000) back to back on the assembled matrix copy of precision `prec`
 * (ELMFB_FP64 or the batch's store_prec), with V = 1, U = 1: ms_host[0] the per-block pass of
 * Y = M V, ms_host[1] the row gather that completes Y (with its norm partials), ms_host[2] the
 * per-block pass of X = M^T U at the current point tile (with its norm partials); ms_host holds
 * 3 doubles.  Overwrites the solver's work vectors; blocks the host until the timing
 * completes.  (Measurement support for the products of Sec. 3 eq. multilevel_domain_decomp.) */
elmfb_status elmfb_batch_time_kernels(elmfb_batch b, int32_t prec, int32_t reps, double* ms_host,
                                      void* stream);

/* Launch shapes of the three matrix passes of a batched Krylov step (the batching of the
 * method's products, Sec. 3 eq. multilevel_domain_decomp, per instance and right-hand side). */
typedef struct {
  int32_t rmvb_tile;       /* points per LDS stage of the M^T U pass: 16, 32, 64 (not FP64)   */
  int32_t mvb_ahead;       /* feature entries each lane loads ahead in the M V pass: 4, 8, 16 */
  int32_t gather_rows;     /* rows per thread of the row gather completing M V: 1 or 2       */
  int32_t from_cache;      /* set by elmfb_batch_tune: 1 = taken from the cache, nothing timed */
  double ms_rmvb[3];       /* ms per launch of each M^T U tile (16, 32, 64); -1 not timed     */
  double ms_mvb[3];        /* of each M V look-ahead (4, 8, 16)                                */
  double ms_gather[2];     /* of each gather shape (1, 2 rows per thread)                      */
} elmfb_batch_shape;

/* Time every candidate shape of the three matrix passes on the assembled matrix copy of
 * precision `prec` (ELMFB_FP64 or the batch's store_prec), `reps` launches each (1..1000)
 * after a warm-up launch, keep the fastest of each for later solves of that precision and
 * write them with the timings to out (may be NULL).  The choice is also cached for the process
 * under (operator, precision, largest K rounded up to a multiple of 16, stored entries rounded
 * down to a power of two, right-hand sides); with use_cache = 1 a batch of a cached class takes
 * the cached shapes without timing (out->from_cache = 1).  Shapes change only launch
 * configurations: M^T U tiles and gather shapes change summation order within rounding, the
 * M V look-ahead does not.  Overwrites the solver's work vectors; synchronises. */
elmfb_status elmfb_batch_tune(elmfb_batch b, int32_t prec, int32_t reps, int32_t use_cache,
                              elmfb_batch_shape* out, void* stream);

/* Set the three shapes for matrix precision `prec` by hand (the gather shape is shared by all
 * precisions); ELMFB_E_INVALID for a shape outside the candidates. */
elmfb_status elmfb_batch_set_shape(elmfb_batch b, int32_t prec, const elmfb_batch_shape* shape);

/* Set the point tile of the batched M^T U pass for matrix precision `prec` by hand (16, 32, or
 * 64 except for ELMFB_FP64), as elmfb_batch_autotune would keep it. */
elmfb_status elmfb_batch_set_tile(elmfb_batch b, int32_t prec, int32_t tile);

/* Coefficients in block-Jacobi coordinates: with preconditioned = 1, elmfb_batch_solve takes x0
 * and returns its result as y = R x per block (the coordinates of M R^{-1}, whose block columns
 * are orthonormal over each support up to the shift), which suits learned warm starts; such
 * solves need precond = 1.  0 (the default) restores x. */
elmfb_status elmfb_batch_set_coords(elmfb_batch b, int32_t preconditioned);

/* x_dev = R^{-1} y_dev per block (both in the V layout): coefficients from block-Jacobi
 * coordinates.  Needs elmfb_batch_precondition; overwrites the solver's work vectors. */
elmfb_status elmfb_batch_from_coords(elmfb_batch b, const double* y_dev, double* x_dev,
                                     void* stream);

/* Solve every (instance, right-hand side) with its own recurrence and stop tests (Sec. 4.1:
 * LSQR, Paige-Saunders, damp 0; FP64 recurrences).
 *   method ELMFB_LSQR: LSQR on the FP64 matrix with atol, btol, iter_lim;
 *   method ELMFB_MIXED_IR: FP64 refinement c += d with d from inner LSQR on the store_prec copy
 *     (at most inner_iters steps; an inner solve also stops once its residual estimate is half
 *     the outer target), the residual r = h - M c recomputed with the FP64 matrix after each
 *     step; a pair stops when ||r|| <= btol ||h|| (istop 1), when atol > 0 and
 *     ||M^T r|| <= atol ||M|| ||r|| (istop 2, least-squares optimality; FP64 products, ||M|| the
 *     inner LSQR's estimate) or after outer_lim steps (istop 7).
 * precond = 1 runs on the preconditioned matrix of elmfb_batch_precondition (M R^{-1}, and its
 * low-precision rounding for MIXED_IR) and returns x = R^{-1} y.  After elmfb_batch_precondition
 * an unpreconditioned MIXED_IR solve needs elmfb_batch_assemble again (ELMFB_E_STATE).  No warm start and no check points.  The iteration loop over the
 * whole batch is captured in a hipGraph (use_graph) of check_every steps; the host reads the
 * number of pairs still running after each replay.  coef_dev in the V layout; info_host
 * [n*n_rhs] (instance-major) may be NULL; MIXED_IR reports the true FP64 residual as rnorm. */
elmfb_status elmfb_batch_solve(elmfb_batch b, const elmfb_solve_opts* opts, double* coef_dev,
                               elmfb_solve_info* info_host, void* stream);

/* Release everything the batch handle owns (NULL: no-op); the message of its last failing call
 * (NULL handle: of the calling thread).  Resource management of the handles above; no
 * computation of the paper. */
void elmfb_batch_destroy(elmfb_batch b);
const char* elmfb_batch_last_error(elmfb_batch b);

/* ---- learned warm start: a small MLP trained on the method's own solutions --------------- */

/* A fully connected tanh network for predicting coefficient blocks from problem parameters
 * (warm starts for the Krylov solve; not part of the paper's method, whose own optimiser
 * settings it uses: Adam with learning rate 1e-3, Sec. 4.1).  Layers l = 0..n_layers-1 map
 * dims[l] -> dims[l+1]: z = a W_l^T + b_l with W_l [dims[l+1]][dims[l]] row-major; hidden layers
 * a = tanh(z), the last layer is linear.  Samples are rows: x [batch][dims[0]], y
 * [batch][dims[n_layers]], FP32.  Products take bfloat16 operands (round to nearest even: the
 * input, the weights, the hidden activations and the back-propagated gradients) with FP32
 * accumulation on the matrix cores; master weights, biases and Adam moments are FP32.
 * Parameters are one flat FP32 vector [W_0, b_0, W_1, b_1, ...]. */
typedef struct elmfb_mlp_s* elmfb_mlp;

typedef struct {
  double lr, beta1, beta2, eps;   /* Adam (Kingma & Ba 2015); lr > 0, betas in [0,1), eps > 0 */
} elmfb_adam;

/* dims_host [n_layers+1] (1..65536 each), n_layers 1..16, max_batch 1..2^24.  n_mod = 1: the model
 * output is the last layer z.  n_mod > 1 (dividing dims[n_layers] = n_mod K): the output is
 * modulated by per-sample weights f [batch][n_mod], y[k] = sum_i f_i z[i K + k] (a model linear in
 * f, for targets that are linear in some problem parameters).  Parameters start at zero; set them
 * with elmfb_mlp_set_params. */
elmfb_status elmfb_mlp_create(int32_t n_layers, const int32_t* dims_host, int32_t n_mod,
                              int32_t max_batch, elmfb_mlp* out);
/* Number of flat parameters (sum over layers of dims[l+1] (dims[l] + 1)). */
elmfb_status elmfb_mlp_query(elmfb_mlp m, int64_t* n_params_host);
/* Copy the flat parameters in (also resets the Adam moments and step count) or out. */
elmfb_status elmfb_mlp_set_params(elmfb_mlp m, const float* params_host);
elmfb_status elmfb_mlp_get_params(elmfb_mlp m, float* params_host);
/* Gradient of the last elmfb_mlp_train_step, same layout as the parameters. */
elmfb_status elmfb_mlp_get_grads(elmfb_mlp m, float* grads_host);
/* y_dev [batch][K] = model(x_dev [batch][dims[0]], f_dev [batch][n_mod]) (f_dev ignored and may
 * be NULL when n_mod = 1; K = dims[n_layers] / n_mod), 1 <= batch <= max_batch. */
elmfb_status elmfb_mlp_forward(elmfb_mlp m, const float* x_dev, const float* f_dev,
                               int32_t batch, float* y_dev, void* stream);
/* Loss = mean over the batch and the K outputs of (y - t)^2, t_dev [batch][K]; gradient by
 * back-propagation; then one Adam step when opt is not NULL (opt NULL: gradient only).
 * loss_host (may be NULL; then the call does not synchronise) receives the loss before the
 * step. */
elmfb_status elmfb_mlp_train_step(elmfb_mlp m, const float* x_dev, const float* f_dev,
                                  const float* t_dev, int32_t batch, const elmfb_adam* opt,
                                  double* loss_host, void* stream);
/* Release the network (NULL: no-op); the message of its last failing call (NULL: of the calling
 * thread).  Resource management; no computation of the paper. */
void elmfb_mlp_destroy(elmfb_mlp m);
const char* elmfb_mlp_last_error(elmfb_mlp m);

/* Time y = G p on the Gram blocks of the last elmfb_gram(h, prec, 1) call (the operator of
 * ELMFB_NORMAL_CG) with HIP events on `stream`, p = 1, `reps` times each: ms_host[0] = one
 * launch of the per-block pass alone (reads every stored block once), ms_host[1] = both passes.
 * Overwrites the solver's work vectors; blocks the host until the timing completes.
 * (Measurement support for CG on the normal equations of Sec. 3 eq. multilevel_ls.) */
elmfb_status elmfb_time_gram_mv(elmfb_problem h, int32_t reps, double* ms_host, void* stream);

/* Release everything the handle owns (device memory, graphs, streams).  NULL is a no-op.
 * Resource management; no computation of the paper. */
void elmfb_destroy(elmfb_problem h);

/* Message of the last failing call on this handle (NULL: of the calling thread).  Error
 * reporting; no computation of the paper. */
const char* elmfb_last_error(elmfb_problem h);

#ifdef __cplusplus
}
#endif
#endif /* ELMFB_H_ */
