"""GPU parity of the Gram blocks (matrix cores, FP64 / FP32 / BF16 / FP16 inputs), the low-precision
stored copies, block-Jacobi preconditioned LSQR and FP64 refinement around low-precision inner
LSQR, against the CPU oracle."""
import numpy as np
import pytest

from inputs import configs, feature_params
from inputs.problems import grid_points
from oracle import assemble as asm
from oracle import evaluate as ev
from oracle import geometry as geo
from oracle import linalg
from oracle import lowprec

from gpu_util import (build, check_rounded_fold, dev, device_blocks, fold_tolerance, n_ambiguous,
                      torch_mod)

pytestmark = pytest.mark.gpu

SPECS = [configs.small1d_multilevel(), configs.small2d(), configs.medium2d()]


@pytest.fixture(scope="module", params=SPECS, ids=lambda s: s.name)
def case32(request):
    spec = request.param
    P, W, b, f = build(spec, store_prec="fp32")
    blocks = asm.assemble_blocks(spec, W, b)
    yield spec, P, W, b, f, blocks, asm.rhs(spec, f)
    P.destroy()


def test_low_precision_copies_round_to_nearest_even(case32):
    """The stored FP32 copy equals the oracle's entries rounded to nearest even, up to one unit
    in the last place where the FP64 values differ in their last bits."""
    spec, P, W, b, f, blocks, h = case32
    got = device_blocks(P, spec.K, "fp32")
    bad = 0
    total = 0
    for (row, Mg), blk in zip(got, blocks):
        ref = lowprec.to_f32(blk.M)
        ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(Mg - ref) <= ulp)
        bad += int(np.sum(Mg != ref))
        total += ref.size
    print(f"{spec.name}: fp32 copy differs from RNE(oracle) in {bad} of {total} entries (1 ulp)")
    assert bad <= max(2, total * 1e-5)


def _gram_dense(P, spec, prec):
    torch = torch_mod()
    P.gram(prec, "all")
    table = P.copy_gram()
    KK = spec.K * spec.K
    dt = torch.float64 if prec == "fp64" else torch.float32
    buf = torch.empty(len(table) * KK, dtype=dt, device="cuda")
    P.copy_gram(buf)
    torch.cuda.synchronize()
    host = buf.double().cpu().numpy()
    return {(int(bi), int(bj)): host[off:off + KK].reshape(spec.K, spec.K)
            for bi, bj, off in table}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gram_blocks(case32, prec):
    """G_ij = M_i^T M_j on the shared rows for every overlapping pair: the same pair set as the
    oracle; FP64 blocks to 1e-12 of the block max; FP32 blocks (from the FP32 copy, FP32
    accumulation) against the oracle's products of the rounded entries to 1e-5."""
    spec, P, W, b, f, blocks, h = case32
    pairs = geo.overlap_pairs(spec, [blk.rows for blk in blocks])
    emap = None if prec == "fp64" else lowprec.to_f32
    ref = linalg.gram_blocks(blocks, pairs, entry_map=emap)
    got = _gram_dense(P, spec, prec)
    assert set(got.keys()) == set(ref.keys())
    tol = 1e-12 if prec == "fp64" else 1e-5
    worst = 0.0
    for key, R in ref.items():
        err = np.abs(got[key] - R).max() / max(np.abs(R).max(), 1e-300)
        worst = max(worst, err)
    print(f"{spec.name} {prec}: {len(ref)} pairs, worst blockwise rel err {worst:.2e}")
    assert worst <= tol


def test_gram_blocks_bf16():
    """BF16 Gram blocks from a BF16 stored copy: against the oracle's products of the
    bfloat16-rounded entries, FP32 accumulation: 1e-5 of the block max."""
    spec = configs.small2d()
    P, W, b, f = build(spec, store_prec="bf16")
    blocks = asm.assemble_blocks(spec, W, b)
    got_blocks = device_blocks(P, spec.K, "bf16")
    for (row, Mg), blk in zip(got_blocks, blocks):
        ref = lowprec.to_bf16(blk.M)
        ulp = np.abs(ref) * 2.0 ** -7 + 1e-300
        assert np.all(np.abs(Mg - ref) <= ulp)
    pairs = geo.overlap_pairs(spec, [blk.rows for blk in blocks])
    ref = linalg.gram_blocks(blocks, pairs, entry_map=lowprec.to_bf16)
    got = _gram_dense(P, spec, "bf16")
    worst = max(np.abs(got[k] - R).max() / max(np.abs(R).max(), 1e-300) for k, R in ref.items())
    print(f"small2d bf16: worst blockwise rel err {worst:.2e}")
    assert worst <= 1e-5
    P.destroy()


def test_block_jacobi_lsqr_matches_oracle(case32):
    """Right block-Jacobi preconditioned LSQR with a shift that keeps G_jj + lambda I well
    conditioned (1e-6: the factors are then accurate to ~1e-10): GPU iterates equal the oracle's
    preconditioned LSQR iterates (u on the test grid) within max(1e-9, 50x the oracle's own
    spread under a row permutation)."""
    spec, P, W, b, f, blocks, h = case32
    torch = torch_mod()
    shift = 1e-6
    nf = P.precondition(shift)
    assert nf == 0
    n = P.sizes["n_phi"]
    N = spec.n_rows
    facs = linalg.block_jacobi_factors(blocks, shift)
    xt = grid_points(spec, spec.meta["n_test"])
    M = asm.dense_from_blocks(blocks, N, n)
    perm = np.random.default_rng(0).permutation(N)
    Mp, hp = M[perm], h[perm]
    for k in (1, 5, 10):
        coef = torch.empty(n, dtype=torch.float64, device="cuda")
        info = P.solve(coef, iter_lim=k, atol=0, btol=0, check_every=5, precond=True)
        x_ref, res = linalg.preconditioned_lsqr(lambda v: asm.matvec(blocks, v, N),
                                                lambda u: asm.rmatvec(blocks, u, n), blocks, facs,
                                                h, n, atol=0, btol=0, iter_lim=k)
        x_p, _ = linalg.preconditioned_lsqr(lambda v: Mp @ v, lambda u: Mp.T @ u, blocks, facs, hp,
                                            n, atol=0, btol=0, iter_lim=k)
        u_ref = ev.evaluate(spec, W, b, x_ref, xt)
        spread = ev.rel_l2(ev.evaluate(spec, W, b, x_p, xt), u_ref)
        du = ev.rel_l2(ev.evaluate(spec, W, b, coef.cpu().numpy(), xt), u_ref)
        tol = max(1e-9, 50 * spread)
        print(f"{spec.name} bj-lsqr k={k}: u diff {du:.2e} (tol {tol:.1e}), "
              f"rnorm {info['rnorm']:.6e} vs {res.rnorm:.6e}")
        assert du <= tol


def test_block_jacobi_small_shift(case32):
    """With the production shift 1e-12 the factors of the nearly singular G_jj + lambda I depend
    on rounding (condition ~1e12), so GPU and oracle preconditioners differ in the directions
    that barely matter: compare the residual norms after 20 steps (1e-3) and check that
    preconditioning beats plain LSQR."""
    spec, P, W, b, f, blocks, h = case32
    torch = torch_mod()
    n = P.sizes["n_phi"]
    N = spec.n_rows
    P.precondition(1e-12)
    facs = linalg.block_jacobi_factors(blocks, 1e-12)
    pre = P.solve(torch.empty(n, dtype=torch.float64, device="cuda"), iter_lim=20, atol=0, btol=0,
                  precond=True)
    _, res = linalg.preconditioned_lsqr(lambda v: asm.matvec(blocks, v, N),
                                        lambda u: asm.rmatvec(blocks, u, n), blocks, facs, h, n,
                                        atol=0, btol=0, iter_lim=20)
    plain = P.solve(torch.empty(n, dtype=torch.float64, device="cuda"), iter_lim=20, atol=0, btol=0)
    print(f"{spec.name}: ||r|| after 20 its: plain {plain['rnorm']:.4e}, preconditioned "
          f"{pre['rnorm']:.4e} (oracle {res.rnorm:.4e})")
    assert abs(pre["rnorm"] - res.rnorm) <= 1e-3 * res.rnorm
    assert pre["rnorm"] < plain["rnorm"]


def test_mixed_refinement_matches_oracle(case32):
    """FP64 refinement around inner LSQR on the FP32 copy of the block-Jacobi preconditioned
    matrix: the inner solves run on the FP32 rounding of M R^{-1} (formed once in FP64; K <= 128
    for all cases here), the FP64 residual on M, c += R^{-1} d.  GPU and oracle refinement agree
    after each of the first outer steps.  The FP32 copies come from FP64 products summed in
    different orders, so an entry next to a rounding boundary may round differently."""
    spec, P, W, b, f, blocks, h = case32
    torch = torch_mod()
    shift = 1e-6
    P.precondition(shift)
    n = P.sizes["n_phi"]
    N = spec.n_rows
    facs = linalg.block_jacobi_factors(blocks, shift)
    fb = linalg.fold_blocks(blocks, facs)
    lo = [asm.Block(blk.sd, blk.rows, lowprec.to_f32(blk.M)) for blk in fb]
    xt = grid_points(spec, spec.meta["n_test"])
    inner = 5
    for outer in (1, 2):
        coef = torch.empty(n, dtype=torch.float64, device="cuda")
        info = P.solve(coef, method="mixed_ir", inner_iters=inner, outer_lim=outer, check_every=5,
                       precond=True, atol=0, btol=0)
        # the same refinement in preconditioned coordinates: r = h - (M R^{-1}) c_y, x = R^{-1} c_y
        cy, hist = linalg.refine_lsqr(lambda v: asm.matvec(fb, v, N),
                                      lambda u: asm.rmatvec(fb, u, n),
                                      lambda v: asm.matvec(lo, v, N),
                                      lambda u: asm.rmatvec(lo, u, n), h, n, outer, inner)
        c = linalg.block_apply(blocks, facs, cy)
        du = ev.rel_l2(ev.evaluate(spec, W, b, coef.cpu().numpy(), xt), ev.evaluate(spec, W, b, c, xt))
        print(f"{spec.name} mixed outer={outer}: u diff {du:.2e}, outer ||r|| {info['rnorm']:.4e} "
              f"(oracle last {hist[-1]:.4e}), inner iters {info['iters']}")
        assert info["outer_iters"] == outer and info["iters"] == outer * inner
        assert du <= 1e-7


def test_fp16_copy_and_gram_blocks():
    """The IEEE binary16 stored copy equals the oracle's entries rounded to nearest even (one
    unit in the last place where the FP64 values differ in their last bits), and the FP16 Gram
    blocks (v_mfma_f32_16x16x32_f16, FP32 accumulation) match the oracle's products of the
    rounded entries to 1e-5 of the block max."""
    spec = configs.small2d()
    P, W, b, f = build(spec, store_prec="fp16")
    blocks = asm.assemble_blocks(spec, W, b)
    bad = total = 0
    for (row, Mg), blk in zip(device_blocks(P, spec.K, "fp16"), blocks):
        ref = lowprec.to_fp16(blk.M)
        ulp = np.maximum(np.abs(ref) * 2.0 ** -10, 2.0 ** -24)
        assert np.all(np.abs(Mg - ref) <= ulp)
        bad += int(np.sum(Mg != ref))
        total += ref.size
    print(f"small2d fp16 copy: {bad} of {total} entries one ulp off RNE(oracle)")
    assert bad <= max(2, total * 1e-5)
    pairs = geo.overlap_pairs(spec, [blk.rows for blk in blocks])
    ref = linalg.gram_blocks(blocks, pairs, entry_map=lowprec.to_fp16)
    got = _gram_dense(P, spec, "fp16")
    assert set(got.keys()) == set(ref.keys())
    worst = max(np.abs(got[k] - R).max() / max(np.abs(R).max(), 1e-300) for k, R in ref.items())
    print(f"small2d fp16 Gram: worst blockwise rel err {worst:.2e}")
    assert worst <= 1e-5
    P.destroy()


def test_mixed_refinement_fp16_folded_matches_oracle():
    """FP64 refinement around inner LSQR on the IEEE binary16 rounding of the folded matrix
    M R^{-1}: GPU and oracle agree after each of the first outer steps (the same protocol as the
    FP32 case); the refinement without the folded copy is refused.  An FP16 entry that rounds
    differently moves the result by far more than the tolerance, so the shift is 1e-2: no entry
    of the oracle's FP16 rounding then lies within fold_tolerance of a boundary (checked), and
    both sides run the same inner matrix."""
    spec = configs.small2d()
    torch = torch_mod()
    P, W, b, f = build(spec, store_prec="fp16")
    n = P.sizes["n_phi"]
    coef = torch.empty(n, dtype=torch.float64, device="cuda")
    with pytest.raises(Exception, match="FP16"):
        P.solve(coef, method="mixed_ir", inner_iters=5, outer_lim=1, precond=False, atol=0, btol=0)
    blocks = asm.assemble_blocks(spec, W, b)
    h = asm.rhs(spec, f)
    shift = 1e-2
    assert P.precondition(shift) == 0
    N = spec.n_rows
    facs = linalg.block_jacobi_factors(blocks, shift)
    fb = linalg.fold_blocks(blocks, facs)
    assert max(np.abs(blk.M).max() for blk in fb) <= 1.0 + 1e-12   # columns of norm <= 1
    for blk in fb:
        assert n_ambiguous(blk.M, lowprec.to_fp16, fold_tolerance(blk.M, spec.K, shift)) == 0
    lo = [asm.Block(blk.sd, blk.rows, lowprec.to_fp16(blk.M)) for blk in fb]
    xt = grid_points(spec, spec.meta["n_test"])
    inner = 5
    for outer in (1, 2):
        info = P.solve(coef, method="mixed_ir", inner_iters=inner, outer_lim=outer, check_every=5,
                       precond=True, atol=0, btol=0)
        cy, hist = linalg.refine_lsqr(lambda v: asm.matvec(fb, v, N),
                                      lambda u: asm.rmatvec(fb, u, n),
                                      lambda v: asm.matvec(lo, v, N),
                                      lambda u: asm.rmatvec(lo, u, n), h, n, outer, inner)
        c = linalg.block_apply(blocks, facs, cy)
        du = ev.rel_l2(ev.evaluate(spec, W, b, coef.cpu().numpy(), xt), ev.evaluate(spec, W, b, c, xt))
        print(f"{spec.name} fp16 mixed outer={outer}: u diff {du:.2e}, outer ||r|| "
              f"{info['rnorm']:.4e} (oracle last {hist[-1]:.4e})")
        assert info["outer_iters"] == outer and info["iters"] == outer * inner
        assert du <= 1e-7
    P.destroy()


@pytest.mark.parametrize("store", ["fp32", "fp16"])
@pytest.mark.parametrize("spec", [configs.small2d(), configs.medium2d()], ids=lambda s: s.name)
def test_folded_copies_match_oracle(spec, store):
    """elmfb_precondition forms M R^{-1} once: the FP64 folded blocks equal the oracle's
    M_j R_j^{-1} within the sensitivity of the shifted Cholesky factor (fold_tolerance), and the
    low-precision folded copy is their rounding to nearest even (an entry within that distance
    of a rounding boundary may round either way)."""
    P, W, b, f = build(spec, store_prec=store)
    blocks = asm.assemble_blocks(spec, W, b)
    shift = 1e-4
    P.precondition(shift)
    fb = linalg.fold_blocks(blocks, linalg.block_jacobi_factors(blocks, shift))
    rounding = lowprec.to_f32 if store == "fp32" else lowprec.to_fp16
    g64 = device_blocks(P, spec.K, "fp64", folded=True)
    glo = device_blocks(P, spec.K, store, folded=True)
    worst, nm, na = 0.0, 0, 0
    for (_, A64), (_, Alo), blk in zip(g64, glo, fb):
        tol = fold_tolerance(blk.M, spec.K, shift)
        err = np.abs(A64 - blk.M).max()
        worst = max(worst, err / tol)
        assert err <= tol
        m, a = check_rounded_fold(Alo, blk.M, rounding, tol)
        nm += m
        na += a
    print(f"{spec.name} {store}: FP64 fold worst {worst:.2f} of its tolerance; rounded copy "
          f"{nm} entries off the oracle's rounding, {na} within tolerance of a boundary")
    P.destroy()
