"""GPU parity of CG on the assembled Gram blocks: the normal-equation solver (plain and
block-Jacobi preconditioned, FP64 and FP32 Gram storage) and the FP64 refinement around it,
against the oracle's CG on its own Gram blocks."""
import numpy as np
import pytest

from inputs import configs
from oracle import assemble as asm
from oracle import geometry as geo
from oracle import linalg
from oracle import lowprec

from gpu_util import build, torch_mod

pytestmark = pytest.mark.gpu

SPECS = [configs.small1d_multilevel(), configs.small2d()]


@pytest.fixture(scope="module", params=SPECS, ids=lambda s: s.name)
def case(request):
    spec = request.param
    P, W, b, f = build(spec, store_prec="fp32")
    blocks = asm.assemble_blocks(spec, W, b)
    h = asm.rhs(spec, f)
    pairs = geo.overlap_pairs(spec, [blk.rows for blk in blocks])
    yield spec, P, blocks, h, pairs
    P.destroy()


def _solve(P, n, **kw):
    torch = torch_mod()
    coef = torch.empty(n, dtype=torch.float64, device="cuda")
    info = P.solve(coef, **kw)
    return coef.cpu().numpy(), info


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_normal_cg_iterates(case):
    """CG on the FP64 Gram blocks: GPU iterates equal the oracle's CG on its Gram blocks within
    max(1e-9, 50x the oracle's own spread, measured against CG on the dense M^T M, whose
    products are summed in another order); the reported residual is ||g - G a||."""
    spec, P, blocks, h, pairs = case
    n = P.sizes["n_phi"]
    N = spec.n_rows
    P.gram("fp64", "all")
    G = linalg.gram_blocks(blocks, pairs)
    M = asm.dense_from_blocks(blocks, N, n)
    Gd = M.T @ M
    g = asm.rmatvec(blocks, h, n)
    for k in (1, 3, 5, 10):
        a, info = _solve(P, n, method="normal_cg", iter_lim=k, atol=0, btol=0, check_every=5)
        ref = linalg.normal_pcg(lambda p: linalg.gram_apply(G, blocks, p), g, k)
        alt = linalg.normal_pcg(lambda p: Gd @ p, g, k)
        tol = max(1e-9, 50 * _rel(alt, ref))
        err = _rel(a, ref)
        rr = np.linalg.norm(g - linalg.gram_apply(G, blocks, a))
        print(f"{spec.name} normal-cg k={k}: coef diff {err:.2e} (tol {tol:.1e}), "
              f"||g - G a|| {info['rnorm']:.6e} vs {rr:.6e}")
        assert info["iters"] == k and info["istop"] == 7
        assert err <= tol
        assert abs(info["rnorm"] - rr) <= max(1e-6 * rr, 1e-12 * np.linalg.norm(g))


def test_normal_pcg_iterates(case):
    """Block-Jacobi preconditioned CG (z = R^{-1} R^{-T} r, shift 1e-6) against the oracle's
    preconditioned CG with its own factors, within max(1e-9, 50x the oracle's spread when its
    factors come from row-permuted blocks: G_jj + lambda I has condition up to K/shift, so its
    factors depend on the summation order at that level)."""
    spec, P, blocks, h, pairs = case
    n = P.sizes["n_phi"]
    shift = 1e-6
    assert P.precondition(shift) == 0
    P.gram("fp64", "all")
    G = linalg.gram_blocks(blocks, pairs)
    facs = linalg.block_jacobi_factors(blocks, shift)
    g = asm.rmatvec(blocks, h, n)
    Minv = lambda r: linalg.block_jacobi_inverse_apply(blocks, facs, r)
    rng = np.random.default_rng(1)
    perm_blocks = []
    for blk in blocks:
        pp = rng.permutation(blk.M.shape[0])
        perm_blocks.append(asm.Block(blk.sd, blk.rows[pp], blk.M[pp]))
    facs_alt = linalg.block_jacobi_factors(perm_blocks, shift)
    Minv_alt = lambda r: linalg.block_jacobi_inverse_apply(blocks, facs_alt, r)
    Gp = lambda p: linalg.gram_apply(G, blocks, p)
    for k in (1, 3, 5, 10):
        a, info = _solve(P, n, method="normal_cg", iter_lim=k, atol=0, btol=0, check_every=5,
                         precond=True)
        ref = linalg.normal_pcg(Gp, g, k, apply_Minv=Minv)
        tol = max(1e-9, 50 * _rel(linalg.normal_pcg(Gp, g, k, apply_Minv=Minv_alt), ref))
        err = _rel(a, ref)
        print(f"{spec.name} normal-pcg k={k}: coef diff {err:.2e} (tol {tol:.1e})")
        assert err <= tol


def test_normal_cg_fp32_gram(case):
    """CG on Gram blocks stored in FP32 (accumulated in FP32 on the matrix cores from the FP32
    copy): early iterates against the oracle's CG on the Gram blocks of the rounded entries
    (products in FP64); the FP32 accumulation of the blocks moves them by about 1e-6, hence
    1e-4."""
    spec, P, blocks, h, pairs = case
    n = P.sizes["n_phi"]
    P.gram("fp32", "all")
    G = linalg.gram_blocks(blocks, pairs, entry_map=lowprec.to_f32)
    g = asm.rmatvec(blocks, h, n)
    for k in (1, 2, 3):
        a, info = _solve(P, n, method="normal_cg", iter_lim=k, atol=0, btol=0, check_every=5)
        ref = linalg.normal_pcg(lambda p: linalg.gram_apply(G, blocks, p), g, k)
        err = _rel(a, ref)
        print(f"{spec.name} normal-cg fp32 gram k={k}: coef diff {err:.2e}")
        assert err <= 1e-4


def test_mixed_ir_cg_matches_oracle_refinement(case):
    """FP64 refinement with CG on the Gram blocks as the inner solve (r = h - M c, g = M^T r,
    G d = g by 5 CG steps, c += d): after 1, 2 and 3 outer steps equal to the oracle's
    refinement (FP64 Gram blocks, FP64 CG) within 1e-8, and the reported residual is the FP64
    ||h - M c||."""
    spec, P, blocks, h, pairs = case
    n = P.sizes["n_phi"]
    N = spec.n_rows
    P.gram("fp64", "all")
    G = linalg.gram_blocks(blocks, pairs)
    inner = 5
    for outer in (1, 2, 3):
        c, info = _solve(P, n, method="mixed_ir_cg", inner_iters=inner, outer_lim=outer,
                         atol=0, btol=0, check_every=5)
        ref, hist = linalg.refine(lambda v: asm.matvec(blocks, v, N),
                                  lambda u: asm.rmatvec(blocks, u, n), h, n,
                                  lambda p: linalg.gram_apply(G, blocks, p), outer, inner,
                                  lo_dtype=np.float64)
        err = _rel(c, ref)
        r = np.linalg.norm(h - asm.matvec(blocks, c, N))
        print(f"{spec.name} mixed-ir-cg outer={outer}: coef diff {err:.2e}, ||r|| "
              f"{info['rnorm']:.6e} vs {r:.6e}")
        assert info["outer_iters"] == outer and info["iters"] == outer * inner
        assert err <= 1e-8
        assert abs(info["rnorm"] - r) <= 1e-9 * np.linalg.norm(h)


def test_normal_cg_stops_on_its_test_and_needs_all_pairs():
    """Preconditioned CG run to btol stops with istop 1, and its final ||g - G a|| meets the
    test (within a factor 2 for the drift of the updated residual) by the oracle's products; CG
    without the full set of Gram blocks is refused."""
    spec = configs.small1d_multilevel()
    P, W, b, f = build(spec, store_prec="fp32")
    n = P.sizes["n_phi"]
    blocks = asm.assemble_blocks(spec, W, b)
    h = asm.rhs(spec, f)
    pairs = geo.overlap_pairs(spec, [blk.rows for blk in blocks])
    P.gram("fp64", "diag")
    with pytest.raises(Exception, match="elmfb_gram"):
        _solve(P, n, method="normal_cg", iter_lim=5, atol=0, btol=0)
    P.precondition(1e-6)
    P.gram("fp64", "all")
    btol = 1e-8
    a, info = _solve(P, n, method="normal_cg", iter_lim=5000, atol=0, btol=btol, check_every=50,
                     precond=True)
    G = linalg.gram_blocks(blocks, pairs)
    g = asm.rmatvec(blocks, h, n)
    rr = np.linalg.norm(g - linalg.gram_apply(G, blocks, a))
    print(f"{spec.name} normal-pcg to btol {btol}: istop {info['istop']}, iters {info['iters']}, "
          f"||g - G a|| / ||g|| = {rr / np.linalg.norm(g):.2e}")
    assert info["istop"] == 1
    # the recursively updated residual the test reads may drift from g - G a by rounding
    assert rr <= 2 * btol * np.linalg.norm(g)
    P.destroy()


def test_time_gram_mv_runs_and_leaves_products_valid(case):
    """The timing entry point runs both passes on the stored blocks and reports positive
    durations; a CG solve afterwards still matches the oracle's first step."""
    spec, P, blocks, h, pairs = case
    n = P.sizes["n_phi"]
    P.gram("fp64", "all")
    ms = P.time_gram_mv(3)
    assert ms[0] > 0 and ms[1] >= ms[0] * 0.5
    G = linalg.gram_blocks(blocks, pairs)
    g = asm.rmatvec(blocks, h, n)
    a, _ = _solve(P, n, method="normal_cg", iter_lim=1, atol=0, btol=0)
    ref = linalg.normal_pcg(lambda p: linalg.gram_apply(G, blocks, p), g, 1)
    assert _rel(a, ref) <= 1e-9


def test_time_gram_counts_the_useful_flops(case):
    """elmfb_time_gram leaves the blocks of elmfb_gram behind and counts 2 K^2 times the shared
    points summed over the oracle's overlapping pairs."""
    spec, P, blocks, h, pairs = case
    ms, flops = P.time_gram("fp64", "all", reps=2)
    shared = sum(np.intersect1d(blocks[i].rows, blocks[j].rows).size for i, j in pairs)
    assert ms > 0 and flops == 2.0 * spec.K * spec.K * shared
    G = linalg.gram_blocks(blocks, pairs)
    n = P.sizes["n_phi"]
    g = asm.rmatvec(blocks, h, n)
    a, _ = _solve(P, n, method="normal_cg", iter_lim=1, atol=0, btol=0)
    assert _rel(a, linalg.normal_pcg(lambda p: linalg.gram_apply(G, blocks, p), g, 1)) <= 1e-9
