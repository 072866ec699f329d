"""GPU parity of the FP64 hot path against the CPU oracle: assembled blocks, block-sparse
products, LSQR and CGLS iterates, evaluation.  Every call goes through the C ABI."""
import dataclasses

import numpy as np
import pytest

from inputs import configs, feature_params
from inputs.problems import grid_points
from oracle import assemble as asm
from oracle import evaluate as ev
from oracle import geometry as geo
from oracle import linalg
from oracle import lowprec

from gpu_util import block_rows, build, dev, device_blocks, n_y, torch_mod

pytestmark = pytest.mark.gpu

SPECS = [configs.tiny1d(), configs.small1d_multilevel(), configs.small2d(), configs.ode1d(),
         configs.medium2d()]


@pytest.fixture(scope="module", params=SPECS, ids=lambda s: s.name)
def case(request):
    spec = request.param
    P, W, b, f = build(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    h = asm.rhs(spec, f)
    yield spec, P, W, b, f, blocks, h
    P.destroy()


def test_sizes_and_structure(case):
    """Same decomposition: block boxes equal the oracle's supports I_j, same nnz and N_Phi."""
    spec, P, W, b, f, blocks, h = case
    assert P.sizes["n_rows"] == spec.n_rows
    assert P.sizes["n_phi"] == len(blocks) * spec.K
    assert P.sizes["nnz"] == sum(len(blk.rows) for blk in blocks) * spec.K
    table = P.copy_blocks()
    for row, blk in zip(table, blocks):
        assert np.array_equal(block_rows(row, n_y(spec)), blk.rows)


def test_points_bit_exact(case):
    spec, P, *_ = case
    torch = torch_mod()
    xy = torch.empty(spec.n_rows * spec.dim, dtype=torch.float64, device="cuda")
    P.points(xy)
    got = xy.cpu().numpy().reshape(spec.n_rows, spec.dim)
    assert np.array_equal(got, geo.points(spec))


def test_assembled_entries_fp64(case):
    """Entries agree with the oracle to 1e-12 of the block's largest entry (FP64, different
    operation order: per-axis envelope factors on the GPU, direct 2D sums in the oracle)."""
    spec, P, W, b, f, blocks, h = case
    got = device_blocks(P, spec.K)
    worst = 0.0
    for (row, Mg), blk in zip(got, blocks):
        scale = max(np.abs(blk.M).max(), 1e-300)
        err = np.abs(Mg - blk.M).max() / scale
        worst = max(worst, err)
    print(f"{spec.name}: max blockwise relative entry error {worst:.2e}")
    assert worst <= 1e-12


def test_rhs(case):
    spec, P, W, b, f, blocks, h = case
    torch = torch_mod()
    hv = torch.empty(spec.n_rows, dtype=torch.float64, device="cuda")
    P.copy_rhs(hv)
    assert np.array_equal(hv.cpu().numpy(), h)


def test_matvec_and_rmatvec(case):
    spec, P, W, b, f, blocks, h = case
    torch = torch_mod()
    rng = np.random.default_rng(11)
    n = P.sizes["n_phi"]
    v = rng.standard_normal(n)
    u = rng.standard_normal(spec.n_rows)
    y = torch.empty(spec.n_rows, dtype=torch.float64, device="cuda")
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    P.matvec(dev(v), y)
    P.rmatvec(dev(u), x)
    yo = asm.matvec(blocks, v, spec.n_rows)
    xo = asm.rmatvec(blocks, u, n)
    ey = np.linalg.norm(y.cpu().numpy() - yo) / np.linalg.norm(yo)
    ex = np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo)
    print(f"{spec.name}: A v rel err {ey:.2e}, A^T u rel err {ex:.2e}")
    assert ey <= 1e-12 and ex <= 1e-12


def _oracle_spread(spec, blocks, h, n, method, k, W, b, xt):
    """The oracle against itself on row-permuted copies of the system (identical in exact
    arithmetic): the rounding sensitivity of the k-th iterate, in u on the test grid and in
    ||r||, as the largest difference over three permutations."""
    N = spec.n_rows
    M = asm.dense_from_blocks(blocks, N, n)
    run = linalg.lsqr if method == "lsqr" else \
        (lambda mv, rmv, hh, nn, **kw: linalg.cgls(mv, rmv, hh, nn, 1.0, **kw))
    a = run(lambda v: asm.matvec(blocks, v, N), lambda u: asm.rmatvec(blocks, u, n), h, n,
            atol=0, btol=0, iter_lim=k)
    ua = ev.evaluate(spec, W, b, a.x, xt)
    du = dr = 0.0
    for seed in range(3):
        perm = np.random.default_rng(seed).permutation(N)
        Mp, hp = M[perm], h[perm]
        c = run(lambda v: Mp @ v, lambda u: Mp.T @ u, hp, n, atol=0, btol=0, iter_lim=k)
        du = max(du, ev.rel_l2(ev.evaluate(spec, W, b, c.x, xt), ua))
        dr = max(dr, abs(c.rnorm - a.rnorm) / a.rnorm)
    return a, du, dr


@pytest.mark.parametrize("method,ks", [("lsqr", (1, 5, 10, 20)), ("cgls", (3, 8))])
def test_krylov_iterates_match(case, method, ks):
    """Matched iterates: the k-th GPU iterate equals the oracle's, in u on the test grid and in
    ||r||, to max(1e-10, 50 x the oracle's own spread under row permutations of the same
    system).  These systems have condition numbers up to ~1e15: once the Krylov recurrence
    loses orthogonality its iterates depend on rounding, for the oracle as for the GPU."""
    spec, P, W, b, f, blocks, h = case
    torch = torch_mod()
    n = P.sizes["n_phi"]
    xt = grid_points(spec, spec.meta["n_test"])
    for k in ks:
        coef = torch.empty(n, dtype=torch.float64, device="cuda")
        info = P.solve(coef, method=method, iter_lim=k, atol=0.0, btol=0.0, check_every=3)
        ref, spread_u, spread_r = _oracle_spread(spec, blocks, h, n, method, k, W, b, xt)
        cg = coef.cpu().numpy()
        # both stop at the iteration limit, or both at a machine-precision test a step apart
        assert abs(info["iters"] - ref.itn) <= 1
        if ref.itn < k:
            continue
        du = ev.rel_l2(ev.evaluate(spec, W, b, cg, xt), ev.evaluate(spec, W, b, ref.x, xt))
        dr = abs(info["rnorm"] - ref.rnorm) / ref.rnorm
        tol_u, tol_r = max(1e-10, 50 * spread_u), max(1e-10, 50 * spread_r)
        print(f"{spec.name} {method} k={k}: u diff {du:.2e} (tol {tol_u:.1e}), "
              f"||r|| diff {dr:.2e} (tol {tol_r:.1e})")
        assert du <= tol_u
        assert dr <= tol_r


def test_condition_estimate_from_the_bidiagonal(case):
    """elmfb_condition_estimate after k LSQR steps: sigma_max and sigma_min of the Golub-Kahan
    bidiagonal B_k the device built equal those of the oracle's B_k (dense SVD) within
    max(1e-10, 50x the oracle's own spread under row permutations), and lie within the dense
    SVD's extreme singular values of M; after CGLS there is no bidiagonal (ELMFB_E_STATE)."""
    from paper_2409_01949_amd import elmfb
    spec, P, W, b, f, blocks, h = case
    torch = torch_mod()
    n = P.sizes["n_phi"]
    N = spec.n_rows
    M = asm.dense_from_blocks(blocks, N, n)
    sv = np.linalg.svd(M, compute_uv=False)
    for k in (5, 15):
        coef = torch.empty(n, dtype=torch.float64, device="cuda")
        P.solve(coef, method="lsqr", iter_lim=k, atol=0.0, btol=0.0, check_every=5)
        smax, smin, kk = P.condition_estimate()
        ref = linalg.lsqr(lambda v: asm.matvec(blocks, v, N), lambda u: asm.rmatvec(blocks, u, n),
                          h, n, atol=0, btol=0, iter_lim=k)
        kr = min(k, ref.itn)
        s = linalg.bidiag_singular_values(ref.bidiag, kr)
        spread_max = spread_min = 0.0
        for seed in range(3):
            perm = np.random.default_rng(seed).permutation(N)
            Mp, hp = M[perm], h[perm]
            rp = linalg.lsqr(lambda v: Mp @ v, lambda u: Mp.T @ u, hp, n, atol=0, btol=0,
                             iter_lim=kr)
            sp = linalg.bidiag_singular_values(rp.bidiag, kr)
            spread_max = max(spread_max, abs(sp[0] - s[0]) / s[0])
            spread_min = max(spread_min, abs(sp[-1] - s[-1]) / s[-1])
        print(f"{spec.name} k={k}: sigma_max {smax:.6e} vs {s[0]:.6e}, sigma_min {smin:.6e} vs "
              f"{s[-1]:.6e} (spreads {spread_max:.1e}, {spread_min:.1e}); M: {sv[0]:.6e}, "
              f"{sv[-1]:.3e}")
        assert kk == kr
        assert abs(smax - s[0]) / s[0] <= max(1e-10, 50 * spread_max)
        assert abs(smin - s[-1]) / s[-1] <= max(1e-10, 50 * spread_min)
        assert smax <= sv[0] * (1 + 1e-10)
        assert smin >= sv[-1] * (1 - 1e-10)
    coef = torch.empty(n, dtype=torch.float64, device="cuda")
    P.solve(coef, method="cgls", iter_lim=3, atol=0.0, btol=0.0, check_every=3)
    with pytest.raises(elmfb.ElmfbError):
        P.condition_estimate()


def test_lsqr_converges_to_least_squares_solution():
    """On a well-conditioned system (kappa ~ 2e4) LSQR runs to its stopping test and returns
    the least-squares minimiser: u equal to the QR solution's to 1e-10."""
    spec = configs.tiny1d()
    P, W, b, f = build(spec)
    torch = torch_mod()
    blocks = asm.assemble_blocks(spec, W, b)
    n = P.sizes["n_phi"]
    M = asm.dense_from_blocks(blocks, spec.n_rows, n)
    h = asm.rhs(spec, f)
    xq = linalg.householder_lstsq(M, h)
    coef = torch.empty(n, dtype=torch.float64, device="cuda")
    info = P.solve(coef, iter_lim=5000, atol=1e-14, btol=1e-14, check_every=25)
    xt = grid_points(spec, spec.meta["n_test"])
    du = ev.rel_l2(ev.evaluate(spec, W, b, coef.cpu().numpy(), xt), ev.evaluate(spec, W, b, xq, xt))
    print(f"tiny1d converged: istop {info['istop']} after {info['iters']}, u vs QR {du:.2e}")
    assert info["istop"] in (1, 2, 4, 5)
    assert du <= 1e-10
    P.destroy()


def test_evaluate_matches_oracle(case):
    spec, P, W, b, f, blocks, h = case
    torch = torch_mod()
    rng = np.random.default_rng(12)
    n = P.sizes["n_phi"]
    coef = rng.standard_normal(n)
    xt = grid_points(spec, spec.meta["n_test"])
    u = torch.empty(xt.shape[0], dtype=torch.float64, device="cuda")
    P.evaluate(dev(coef), dev(xt), u)
    ref = ev.evaluate(spec, W, b, coef, xt)
    err = np.abs(u.cpu().numpy() - ref).max() / np.abs(ref).max()
    print(f"{spec.name}: evaluate max rel err {err:.2e}")
    assert err <= 1e-12


def test_graph_and_eager_solves_agree(case, monkeypatch):
    """The multi-workgroup LSQR replayed as a graph and launched eagerly: the same bits (the
    one-workgroup path, which small systems take by default, has its own chunking test)."""
    monkeypatch.setenv("ELMFB_PERSISTENT", "0")
    spec, P, *_ = case
    torch = torch_mod()
    n = P.sizes["n_phi"]
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    c = torch.empty(n, dtype=torch.float64, device="cuda")
    ia = P.solve(a, iter_lim=40, atol=0, btol=0, check_every=7, use_graph=True)
    ic = P.solve(c, iter_lim=40, atol=0, btol=0, check_every=40, use_graph=False)
    assert ia["iters"] == ic["iters"] == 40
    assert torch.equal(a, c)   # deterministic reductions: bit-identical


def test_warm_start_and_zero_iterations(case):
    spec, P, *_ = case
    torch = torch_mod()
    n = P.sizes["n_phi"]
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    info = P.solve(x, iter_lim=0)
    assert info["iters"] == 0 and torch.count_nonzero(x) == 0
    P.solve(x, iter_lim=30, atol=0, btol=0)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    i2 = P.solve(y, iter_lim=30, atol=0, btol=0, x0=x)
    # restarting from x_30 cannot increase the residual
    i1 = P.solve(torch.empty_like(x), iter_lim=30, atol=0, btol=0)
    assert i2["rnorm"] <= i1["rnorm"] * (1 + 1e-12)
