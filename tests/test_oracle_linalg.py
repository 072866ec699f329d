"""Pins of the oracle's solvers, Gram blocks, refinement, rounding and evaluation against
textbook facts: QR vs LAPACK, LSQR finite termination, LSQR = CGLS in exact arithmetic,
SciPy's LSQR iterates, Gram = M^T M, refinement convergence, bfloat16 rounding."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from inputs import configs, feature_params
from oracle import assemble as asm
from oracle import evaluate as ev
from oracle import geometry as geo
from oracle import linalg
from oracle import lowprec


def _tiny_system():
    spec = configs.tiny1d()
    W, b = feature_params(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    M = asm.dense_from_blocks(blocks, spec.n_rows, len(blocks) * spec.K)
    h = asm.rhs(spec, configs.forcing(spec))
    return spec, W, b, blocks, M, h


def _well_conditioned(m=60, n=20, cond=10.0, seed=0):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.geomspace(1.0, 1.0 / cond, n)
    return (U * s) @ V.T, rng.standard_normal(m)


def test_householder_matches_lapack():
    _, _, _, _, M, h = _tiny_system()
    x = linalg.householder_lstsq(M, h)
    ref = np.linalg.lstsq(M, h, rcond=None)[0]
    cond = np.linalg.cond(M)
    assert np.linalg.norm(x - ref) <= cond * 1e-15 * 10 * np.linalg.norm(ref)


def test_lsqr_orthonormal_columns_one_step():
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 8)))
    h = rng.standard_normal(30)
    r = linalg.lsqr(lambda v: Q @ v, lambda u: Q.T @ u, h, 8, atol=1e-14, btol=1e-14, iter_lim=1)
    assert np.allclose(r.x, Q.T @ h, atol=1e-14)
    # the stopping test recognises the exact least-squares solution after one step
    r = linalg.lsqr(lambda v: Q @ v, lambda u: Q.T @ u, h, 8, atol=1e-12, btol=1e-12)
    assert r.itn == 1 and r.istop in (2, 5)


def test_lsqr_diagonal_finite_termination():
    """A diagonal matrix with n distinct singular values: the Krylov space is exhausted after n
    steps, so LSQR returns the exact solution at step n."""
    d = np.array([3.0, 1.5, 0.7, 0.2, 0.05])
    A = np.vstack([np.diag(d), np.zeros((3, 5))])
    rng = np.random.default_rng(2)
    h = rng.standard_normal(8)
    r = linalg.lsqr(lambda v: A @ v, lambda u: A.T @ u, h, 5, atol=0, btol=0, iter_lim=5)
    assert np.allclose(r.x, h[:5] / d, rtol=1e-10)
    r4 = linalg.lsqr(lambda v: A @ v, lambda u: A.T @ u, h, 5, atol=0, btol=0, iter_lim=4)
    assert not np.allclose(r4.x, h[:5] / d, rtol=1e-3)


def test_lsqr_equals_cgls_iterates():
    """LSQR and CGLS generate the same iterates in exact arithmetic (Paige & Saunders 1982);
    compared over the first 10 steps, before the residual reaches rounding level and the two
    recurrences' rounding errors take over."""
    A, h = _well_conditioned()
    ks = tuple(range(1, 11))
    r1 = linalg.lsqr(lambda v: A @ v, lambda u: A.T @ u, h, A.shape[1], atol=0, btol=0,
                     iter_lim=10, snapshot_at=ks)
    r2 = linalg.cgls(lambda v: A @ v, lambda u: A.T @ u, h, A.shape[1], np.linalg.norm(A),
                     atol=0, btol=0, iter_lim=10, snapshot_at=ks)
    for k in ks:
        assert np.linalg.norm(r1.snapshots[k] - r2.snapshots[k]) <= 1e-12 * np.linalg.norm(r1.snapshots[k])


def test_lsqr_matches_scipy_iterates():
    """Same iterates as SciPy's LSQR over the first steps; later, where the residual nearly
    stagnates and the iterates become sensitive to rounding, the residual norms still agree."""
    A, h = _well_conditioned(cond=1e3, seed=3)
    for k in (1, 2, 3, 4, 5):
        ours = linalg.lsqr(lambda v: A @ v, lambda u: A.T @ u, h, A.shape[1], atol=0, btol=0,
                           iter_lim=k).x
        theirs = spla.lsqr(A, h, atol=0, btol=0, conlim=0, iter_lim=k)[0]
        assert np.linalg.norm(ours - theirs) <= 1e-12 * np.linalg.norm(theirs)
    for k in (12, 20):
        ours = linalg.lsqr(lambda v: A @ v, lambda u: A.T @ u, h, A.shape[1], atol=0, btol=0,
                           iter_lim=k).x
        theirs = spla.lsqr(A, h, atol=0, btol=0, conlim=0, iter_lim=k)[0]
        assert abs(np.linalg.norm(A @ ours - h) - np.linalg.norm(A @ theirs - h)) <= \
            1e-3 * np.linalg.norm(h)


def test_lsqr_converges_to_qr_solution():
    _, _, _, blocks, M, h = _tiny_system()
    n = M.shape[1]
    r = linalg.lsqr(lambda v: asm.matvec(blocks, v, M.shape[0]),
                    lambda u: asm.rmatvec(blocks, u, n), h, n, atol=1e-14, btol=1e-14,
                    iter_lim=2000)
    ref = linalg.householder_lstsq(M, h)
    cond = np.linalg.cond(M)
    assert np.linalg.norm(r.x - ref) <= 1e-14 * cond * np.linalg.norm(ref)
    assert abs(r.rnorm - np.linalg.norm(M @ ref - h)) <= 1e-10


def test_lsqr_warm_start():
    """Starting from x0 solves for the correction of h - M x0; a converged x0 stops at once."""
    A, h = _well_conditioned(seed=4)
    full = linalg.lsqr(lambda v: A @ v, lambda u: A.T @ u, h, A.shape[1], atol=1e-14, btol=1e-14)
    again = linalg.lsqr(lambda v: A @ v, lambda u: A.T @ u, h, A.shape[1], atol=1e-10,
                        btol=1e-10, x0=full.x)
    assert again.itn <= 1
    assert np.allclose(again.x, full.x, atol=1e-12)


def test_gram_blocks_equal_dense_normal_matrix():
    spec = configs.small2d()
    W, b = feature_params(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    n = len(blocks) * spec.K
    M = asm.dense_from_blocks(blocks, spec.n_rows, n)
    pairs = geo.overlap_pairs(spec, [blk.rows for blk in blocks])
    G = linalg.gram_blocks(blocks, pairs)
    assert set(G.keys()) == set(pairs)
    D = np.zeros((n, n))
    for (i, j), g in G.items():
        qi, qj = blocks[i].sd.q0, blocks[j].sd.q0
        D[qi:qi + spec.K, qj:qj + spec.K] = g
        D[qj:qj + spec.K, qi:qi + spec.K] = g.T
    ref = M.T @ M
    assert np.abs(D - ref).max() <= 1e-14 * np.abs(ref).max()
    for (i, j), g in G.items():
        if i == j:
            assert np.array_equal(g, g.T) or np.abs(g - g.T).max() <= 1e-15 * np.abs(g).max()
    lam = np.linalg.eigvalsh(ref)
    assert lam.min() >= -1e-12 * lam.max()
    rng = np.random.default_rng(5)
    p = rng.standard_normal(n)
    assert np.allclose(linalg.gram_apply(G, blocks, p), ref @ p, rtol=0,
                       atol=1e-13 * np.abs(ref @ p).max())


def test_normal_cg_solves_spd():
    A, _ = _well_conditioned(m=40, n=12, cond=5.0, seed=6)
    G = A.T @ A
    g = np.random.default_rng(7).standard_normal(12)
    d = linalg.normal_cg(lambda p: G @ p, g, 12)
    assert np.allclose(d, np.linalg.solve(G, g), rtol=1e-10)


def test_pcg_reduces_to_cg_and_exact_preconditioner_solves_in_one_step():
    """Preconditioned CG with M = I is plain CG step for step; with M = G the first step is
    exact; with a block-diagonal M it still terminates in n steps (n = 12); a warm start at the
    solution leaves it there."""
    A, _ = _well_conditioned(m=50, n=12, cond=30.0, seed=16)
    G = A.T @ A
    g = np.random.default_rng(17).standard_normal(12)
    ref = np.linalg.solve(G, g)
    for k in (1, 3, 7):
        assert np.array_equal(linalg.normal_pcg(lambda p: G @ p, g, k),
                              linalg.normal_cg(lambda p: G @ p, g, k))
    d1 = linalg.normal_pcg(lambda p: G @ p, g, 1, apply_Minv=lambda r: np.linalg.solve(G, r))
    assert np.allclose(d1, ref, rtol=1e-12, atol=0)
    Mb = np.zeros_like(G)
    for s0 in (0, 5):
        Mb[s0:s0 + 5 + 2 * (s0 > 0), s0:s0 + 5 + 2 * (s0 > 0)] = \
            G[s0:s0 + 5 + 2 * (s0 > 0), s0:s0 + 5 + 2 * (s0 > 0)]
    dn = linalg.normal_pcg(lambda p: G @ p, g, 12, apply_Minv=lambda r: np.linalg.solve(Mb, r))
    assert np.allclose(dn, ref, rtol=1e-9, atol=0)
    d0 = linalg.normal_pcg(lambda p: G @ p, g, 5, x0=ref)
    assert np.allclose(d0, ref, rtol=1e-12, atol=0)


def test_block_jacobi_inverse_apply_inverts_the_shifted_diagonal_blocks():
    """z = (R^T R)^{-1} r per block equals solving with G_jj + lambda I."""
    from oracle import assemble as asm
    spec = configs.small1d_multilevel()
    W, b = feature_params(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    shift = 1e-6
    facs = linalg.block_jacobi_factors(blocks, shift)
    n = len(blocks) * spec.K
    r = np.random.default_rng(18).standard_normal(n)
    z = linalg.block_jacobi_inverse_apply(blocks, facs, r)
    for blk in blocks:
        K = spec.K
        G = blk.M.T @ blk.M
        lam = shift * np.trace(G) / K
        sl = slice(blk.sd.q0, blk.sd.q0 + K)
        assert np.allclose((G + lam * np.eye(K)) @ z[sl], r[sl], rtol=0,
                           atol=1e-8 * np.abs(r[sl]).max())


def test_refinement_reaches_working_precision():
    """With kappa(G) u_32 << 1, refinement around a float32 inner solve converges to the float64
    least-squares solution (classical iterative refinement)."""
    A, h = _well_conditioned(m=80, n=24, cond=20.0, seed=8)
    G32 = (A.T @ A).astype(np.float32)
    c, hist = linalg.refine(lambda v: A @ v, lambda u: A.T @ u, h, 24,
                            lambda p: G32 @ p, n_outer=12, n_inner=24)
    ref = np.linalg.lstsq(A, h, rcond=None)[0]
    assert np.linalg.norm(c - ref) <= 1e-13 * np.linalg.norm(ref)
    assert hist[-1][1] < 1e-10 * hist[0][1]


def test_bf16_rounding_against_torch_and_ties():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(9)
    x32 = (rng.standard_normal(20000) * np.exp(rng.uniform(-30, 30, 20000))).astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(lowprec.to_bf16(x32.astype(np.float64)), ref)
    # ties and double-rounding cases, decided from the definition
    assert lowprec.to_bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0            # tie -> even
    assert lowprec.to_bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2 ** -6  # tie -> even (up)
    assert lowprec.to_bf16(np.array([1.0 + 2.0 ** -8 + 2.0 ** -30]))[0] == 1.0 + 2.0 ** -7
    assert lowprec.to_bf16(np.array([-(1.0 + 2.0 ** -8 + 2.0 ** -30)]))[0] == -(1.0 + 2.0 ** -7)
    assert np.isinf(lowprec.to_bf16(np.array([3.5e38]))[0])
    assert lowprec.to_f32(np.array([1.0 + 2.0 ** -24]))[0] == 1.0


def test_fp16_rounding_against_numpy_and_ties():
    """IEEE binary16 rounding: numpy's one-step float64 -> float16 cast (a separate
    implementation) on a wide random sample, and the tie, double-rounding, subnormal and
    overflow cases by hand."""
    rng = np.random.default_rng(11)
    x = rng.uniform(1, 2, 200000) * 2.0 ** rng.integers(-30, 17, 200000) * rng.choice([-1, 1], 200000)
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(lowprec.to_fp16(x), ref)
    f = lambda v: lowprec.to_fp16(np.array([v]))[0]
    assert f(1.0 + 2.0 ** -11) == 1.0                          # tie -> even (down)
    assert f(1.0 + 3 * 2.0 ** -11) == 1.0 + 2.0 ** -9          # tie -> even (up)
    assert f(1.0 + 2.0 ** -11 + 2.0 ** -40) == 1.0 + 2.0 ** -10  # no double rounding via FP32
    assert f(2.0 ** -25) == 0.0 and f(3 * 2.0 ** -26) == 2.0 ** -24   # subnormal spacing 2^-24
    assert f(2.0 ** -14 - 2.0 ** -26) == 2.0 ** -14           # rounds up into the normal range
    assert f(65519.0) == 65504.0 and np.isinf(f(65520.0))      # largest finite, overflow tie


def test_evaluate_single_feature_closed_form():
    """One level, one subdomain, one feature: u = C(x) a tanh(W xbar + b)."""
    spec = configs.tiny1d(K=1, J=1, n=10)
    W, b = feature_params(spec)
    x = np.linspace(-1, 1, 13)[:, None]
    u = ev.evaluate(spec, W, b, np.array([2.5]), x)
    ref = np.tanh(spec.ansatz_omega * x[:, 0]) * 2.5 * np.tanh(W[0, 0] * x[:, 0] + b[0])
    assert np.allclose(u, ref, rtol=1e-15, atol=1e-15)


def test_metrics():
    u = np.array([1.0, 2.0, 3.0, 4.0])
    ue = np.array([1.0, 2.0, 3.0, 5.0])
    assert ev.e_l1(u, ue) == pytest.approx(0.25 / np.std(ue))
    assert np.std(ue) == pytest.approx(np.sqrt(np.mean((ue - ue.mean()) ** 2)))
    assert ev.rel_l2(u, ue) == pytest.approx(1.0 / np.linalg.norm(ue))


def _tiny2d_blocks():
    spec = configs.small2d()
    W, b = feature_params(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    return spec, blocks


def test_block_jacobi_factors_reconstruct_shifted_gram():
    """R_j^T R_j = G_jj + lambda_j I, and R_j upper triangular with a positive diagonal."""
    spec, blocks = _tiny2d_blocks()
    facs = linalg.block_jacobi_factors(blocks, 1e-10)
    for blk, R in zip(blocks, facs):
        G = blk.M.T @ blk.M
        lam = 1e-10 * np.trace(G) / spec.K
        assert np.allclose(np.triu(R), R)
        assert np.all(np.diag(R) > 0)
        E = R.T @ R - (G + lam * np.eye(spec.K))
        assert np.abs(E).max() <= 1e-12 * np.abs(G).max()


def test_folded_blocks_are_orthonormalised_and_equal_the_product():
    """M_j R_j^{-1} from fold_blocks: its Gram matrix is I - lambda_j R_j^{-T} R_j^{-1} (from
    R_j^T R_j = G_jj + lambda_j I), i.e. orthonormal columns up to the shift, and the folded
    system's products equal M (R^{-1} y) and R^{-T} (M^T u).  Shift 1e-6 keeps cond(G + lambda I)
    near 1e6, so the identity holds to ~1e-10 in floating point."""
    spec, blocks = _tiny2d_blocks()
    shift = 1e-6
    facs = linalg.block_jacobi_factors(blocks, shift)
    folded = linalg.fold_blocks(blocks, facs)
    for blk, fb, R in zip(blocks, folded, facs):
        G = blk.M.T @ blk.M
        lam = shift * np.trace(G) / spec.K
        Ri = np.linalg.inv(R)
        E = fb.M.T @ fb.M - (np.eye(spec.K) - lam * Ri.T @ Ri)
        assert np.abs(E).max() <= 1e-8
        assert np.array_equal(fb.rows, blk.rows)
    n = len(blocks) * spec.K
    N = spec.n_rows
    rng = np.random.default_rng(4)
    y, u = rng.standard_normal(n), rng.standard_normal(N)
    a = asm.matvec(folded, y, N)
    b = asm.matvec(blocks, linalg.block_apply(blocks, facs, y), N)
    assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b)
    a = asm.rmatvec(folded, u, n)
    b = linalg.block_apply(blocks, facs, asm.rmatvec(blocks, u, n), transpose=True)
    assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b)


def test_preconditioned_lsqr_reaches_least_squares_solution():
    """Right preconditioning changes the iteration, not the minimiser: on a full-rank system it
    converges to the QR solution."""
    _, _, _, blocks, M, h = _tiny_system()
    n = M.shape[1]
    facs = linalg.block_jacobi_factors(blocks, 1e-14)
    x, res = linalg.preconditioned_lsqr(lambda v: M @ v, lambda u: M.T @ u, blocks, facs, h, n,
                                        atol=1e-15, btol=1e-15, iter_lim=500)
    ref = linalg.householder_lstsq(M, h)
    assert np.linalg.norm(M @ x - h) <= np.linalg.norm(M @ ref - h) * (1 + 1e-9)
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)
    # warm start: the correction from x0 reaches the same minimiser
    x2, _ = linalg.preconditioned_lsqr(lambda v: M @ v, lambda u: M.T @ u, blocks, facs, h, n,
                                       x0=0.5 * ref, atol=1e-15, btol=1e-15, iter_lim=500)
    assert np.linalg.norm(x2 - ref) <= 1e-8 * np.linalg.norm(ref)


def test_refine_lsqr_fp32_inner_fixed_points():
    """Refinement with the residual in float64 and the correction from LSQR on the float32-rounded
    matrix: on a consistent system it converges to the exact solution; on an inconsistent one
    its fixed point satisfies M_lo^T (h - M c) = 0 (the correction of a converged step is zero),
    which differs from the float64 minimiser by a term proportional to the optimal residual."""
    A, h = _well_conditioned(m=90, n=30, cond=50.0, seed=10)
    A32 = lowprec.to_f32(A)
    x_true = np.random.default_rng(3).standard_normal(30)
    hc = A @ x_true
    run = lambda rhs: linalg.refine_lsqr(lambda v: A @ v, lambda u: A.T @ u, lambda v: A32 @ v,
                                         lambda u: A32.T @ u, rhs, 30, n_outer=10, n_inner=60)
    c, _ = run(hc)
    assert np.linalg.norm(c - x_true) <= 1e-13 * np.linalg.norm(x_true)
    c, _ = run(h)
    g = A32.T @ (h - A @ c)
    assert np.linalg.norm(g) <= 1e-12 * np.linalg.norm(A32.T @ h)
    ref = np.linalg.lstsq(A, h, rcond=None)[0]
    r_opt = np.linalg.norm(h - A @ ref)
    assert np.linalg.norm(A @ (c - ref)) <= 1e-5 * r_opt


def test_bidiagonal_singular_values_interlace_and_terminate():
    """The Golub-Kahan bidiagonal recorded by LSQR: its extreme singular values stay inside M's
    (sigma_max(B_k) grows toward sigma_max(M), sigma_min(B_k) shrinks toward sigma_min(M)); for M
    with three distinct singular values the Krylov space has dimension 3, so B_3's singular values
    are exactly those three; the recorded alpha_1, beta_1 are ||M^T h|| / ||h|| and ||h||."""
    M, _ = _well_conditioned(m=60, n=20, cond=30.0, seed=3)
    h = np.random.default_rng(4).standard_normal(60)
    sv = np.linalg.svd(M, compute_uv=False)
    res = linalg.lsqr(lambda v: M @ v, lambda u: M.T @ u, h, 20, atol=0, btol=0, iter_lim=20)
    assert res.bidiag[0][1] == pytest.approx(np.linalg.norm(h), rel=1e-15)
    assert res.bidiag[0][0] == pytest.approx(np.linalg.norm(M.T @ h) / np.linalg.norm(h), rel=1e-14)
    prev_max, prev_min = 0.0, np.inf
    for k in (1, 2, 5, 10, 15, 20):
        s = linalg.bidiag_singular_values(res.bidiag, k)
        assert len(s) == k
        assert s[0] <= sv[0] * (1 + 1e-12) and s[-1] >= sv[-1] * (1 - 1e-12)
        assert s[0] >= prev_max * (1 - 1e-12) and s[-1] <= prev_min * (1 + 1e-12)
        prev_max, prev_min = s[0], s[-1]
    assert prev_max == pytest.approx(sv[0], rel=1e-12)
    rng = np.random.default_rng(5)
    U, _ = np.linalg.qr(rng.standard_normal((40, 12)))
    V, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    M3 = (U * np.repeat([2.0, 1.0, 0.5], 4)) @ V.T
    h3 = rng.standard_normal(40)
    res3 = linalg.lsqr(lambda v: M3 @ v, lambda u: M3.T @ u, h3, 12, atol=0, btol=0, iter_lim=3)
    assert np.allclose(linalg.bidiag_singular_values(res3.bidiag, 3), [2.0, 1.0, 0.5],
                       rtol=1e-12, atol=0)


def test_bidiagonal_extreme_values_by_bisection():
    """The extreme singular values of B_k from bisection on the Golub-Kahan tridiagonal equal the
    dense SVD's on a recorded LSQR bidiagonal (every k up to 60); and on a hand-built bidiagonal
    with known singular values (a diagonal B_k padded with a zero last row: alpha_i on the
    diagonal, beta = 0 below, so sigma_i = alpha_i) they are exact also when sigma_min is 1e-13
    of sigma_max, where squaring (B^T B) would lose every digit."""
    M, _ = _well_conditioned(m=90, n=60, cond=1e4, seed=7)
    h = np.random.default_rng(8).standard_normal(90)
    res = linalg.lsqr(lambda v: M @ v, lambda u: M.T @ u, h, 60, atol=0, btol=0, iter_lim=60)
    for k in (1, 2, 7, 30, 60):
        s = linalg.bidiag_singular_values(res.bidiag, k)
        smax, smin = linalg.bidiag_extreme_singular_values(res.bidiag, k)
        assert smax == pytest.approx(s[0], rel=1e-13)
        assert smin == pytest.approx(s[-1], rel=1e-10)
    alphas = [3.0, 1.0, 2.5e-13, 0.7]
    bid = [(alphas[0], 1.0)] + [(alphas[i], 0.0) for i in range(1, 4)] + [(0.0, 0.0)]
    smax, smin = linalg.bidiag_extreme_singular_values(bid, 4)
    assert smax == pytest.approx(3.0, rel=1e-15)
    assert smin == pytest.approx(2.5e-13, rel=1e-12)
