"""CPU FP64 oracle for the multilevel ELM-FBPINN least-squares system.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark use it, as the independent reference the
HIP path is compared against.

It is a plain, slow, obviously correct restatement of the method (Sec. 3 and
Sec. 4.1 of the paper), written in NumPy float64, with every formula derived
afresh in 1D/2D form (no per-axis factorisation tricks, no blocking beyond the
block decomposition M = sum_l sum_j V^T M_j W of Sec. 3, "Multilevel
domain-decomposition structure").  It shares no code with the GPU library.

Modules
  geometry  grid points, subdomain centres and half-widths, supports I_j, blocks, pairs
  basis     windows (eq. window_func), random features, hard-constraint ansatz,
            operator rows N_{n,q}
  assemble  dense and block-wise assembly of M and h (Sec. 3 definitions)
  linalg    Householder QR, LSQR, CGLS, Gram blocks, normal-equation CG, refinement
  evaluate  u_hat at arbitrary points (eq. multilevel_solution), rel-L2, e_L1 (eq. l1_error)
  lowprec   round-to-nearest-even to float32 / bfloat16
  mlp       tanh MLP forward, manual backward, Adam
"""
