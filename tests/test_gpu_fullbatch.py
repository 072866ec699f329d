"""Parity of the batched path at the benchmark's full size and launch configuration: 512 ragged
2D Poisson instances (J ~ U{4..24}^2, K ~ U{64..128}, 20..60 points per subdomain cell), 8
right-hand sides each, FP64 matrix plus FP32 copy, every kernel one launch over the whole batch.
The oracle assembles a sample of the instances (the first and last, the largest, the widest, the
smallest and two drawn at random) and checks their slices of the batched results element by
element; the other 505 instances run in the same launches."""
import numpy as np
import pytest

from inputs import configs, feature_params
from oracle import assemble as asm
from oracle import linalg

from gpu_util import dev, torch_mod

pytestmark = pytest.mark.gpu

R = 8


@pytest.fixture(scope="module")
def full_batch():
    from paper_2409_01949_amd import Batch
    specs, _ = configs.batch_instances(n=512, seed=3, n_rhs=R)
    feats = [feature_params(s) for s in specs]
    print("# full batch: define + assemble", flush=True)
    B = Batch(specs, [w for w, _ in feats], [b for _, b in feats], R, store_prec="fp32")
    fs = [configs.batch_forcing(s) for s in specs]
    B.assemble(dev(np.concatenate([f.ravel() for f in fs])))
    size = [s.n_rows * s.K for s in specs]
    rng = np.random.default_rng(7)
    sample = sorted({0, len(specs) - 1, int(np.argmax(size)), int(np.argmin(size)),
                     int(np.argmax([s.K for s in specs])), *rng.choice(len(specs), 2, replace=False)})
    print(f"# oracle for instances {sample}", flush=True)
    oracle = {}
    for i in sample:
        s = specs[i]
        blocks = asm.assemble_blocks(s, *feats[i])
        oracle[i] = (s, blocks, np.stack([asm.rhs(s, fj) for fj in fs[i]]))
    yield B, specs, oracle
    B.destroy()


def _slice(B, vec, i, n, cols=True):
    o = B.offsets[i][1 if cols else 0]
    return vec[R * o:R * (o + n)].reshape(R, n)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_full_batch_sizes(full_batch):
    """Row and column offsets of all 512 instances follow from their grids and block counts."""
    B, specs, oracle = full_batch
    rows = np.cumsum([0] + [s.n_rows for s in specs])
    cols = np.cumsum([0] + [s.levels[0][0] * s.levels[0][1] * s.K for s in specs])
    assert np.array_equal(B.offsets[:, 0], rows)
    assert np.array_equal(B.offsets[:, 1], cols)
    for i, (s, bl, _) in oracle.items():
        assert len(bl) * s.K == cols[i + 1] - cols[i]


def test_full_batch_products(full_batch):
    """Y = M V and X = M^T U over the whole batch (the autotuned FP64 tile), the sampled
    instances' slices to 1e-12 of the oracle's products for all 8 right-hand sides."""
    B, specs, oracle = full_batch
    torch = torch_mod()
    rng = np.random.default_rng(11)
    v = rng.standard_normal(R * B.sizes["n_phi"])
    u = rng.standard_normal(R * B.sizes["n_rows"])
    B.autotune("fp64", reps=2)
    y = torch.empty(R * B.sizes["n_rows"], dtype=torch.float64, device="cuda")
    x = torch.empty(R * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
    B.matvec(dev(v), y)
    B.rmatvec(dev(u), x)
    yh, xh = y.cpu().numpy(), x.cpu().numpy()
    for i, (s, bl, _) in oracle.items():
        n = len(bl) * s.K
        vi, ui = _slice(B, v, i, n), _slice(B, u, i, s.n_rows, cols=False)
        yi, xi = _slice(B, yh, i, s.n_rows, cols=False), _slice(B, xh, i, n)
        for j in range(R):
            assert _rel(yi[j], asm.matvec(bl, vi[j], s.n_rows)) <= 1e-12, (i, j)
            assert _rel(xi[j], asm.rmatvec(bl, ui[j], n)) <= 1e-12, (i, j)


def test_full_batch_lsqr_iterates(full_batch):
    """5 LSQR steps for all 4,096 pairs; the sampled pairs equal the oracle's LSQR to 1e-9."""
    B, specs, oracle = full_batch
    torch = torch_mod()
    coef = torch.empty(R * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
    infos = B.solve(coef, iter_lim=5, atol=0.0, btol=0.0, check_every=5)
    ch = coef.cpu().numpy()
    for i, (s, bl, h) in oracle.items():
        n = len(bl) * s.K
        ci = _slice(B, ch, i, n)
        for j in range(R):
            ref = linalg.lsqr(lambda vv: asm.matvec(bl, vv, s.n_rows),
                              lambda uu: asm.rmatvec(bl, uu, n), h[j], n, atol=0, btol=0,
                              iter_lim=5)
            assert infos[i * R + j]["iters"] == 5
            assert _rel(ci[j], ref.x) <= 1e-9, (i, j)
            assert abs(infos[i * R + j]["rnorm"] - ref.rnorm) <= 1e-9 * ref.rnorm


def test_full_batch_block_jacobi_and_refinement(full_batch):
    """Block-Jacobi factors and the folded matrices of all 123,479 blocks (shift 1e-3): 5
    preconditioned LSQR steps on the FP64 folded matrix equal the oracle's per sampled pair to
    1e-8; then the FP64 refinement on the FP32 folded copy (2 outer steps of 5) reports for every
    sampled pair the residual ||h - M c|| that the oracle's products give for the returned
    coefficients (1e-9 of ||h||), and leaves it below ||h||."""
    B, specs, oracle = full_batch
    torch = torch_mod()
    shift = 1e-3
    nf = B.precondition(shift)
    assert nf == 0
    coef = torch.empty(R * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
    infos = B.solve(coef, iter_lim=5, atol=0.0, btol=0.0, check_every=5, precond=True)
    ch = coef.cpu().numpy()
    worst = 0.0
    for i, (s, bl, h) in oracle.items():
        n = len(bl) * s.K
        facs = linalg.block_jacobi_factors(bl, shift)
        ci = _slice(B, ch, i, n)
        for j in range(R):
            x_ref, res = linalg.preconditioned_lsqr(
                lambda vv: asm.matvec(bl, vv, s.n_rows), lambda uu: asm.rmatvec(bl, uu, n), bl,
                facs, h[j], n, atol=0, btol=0, iter_lim=5)
            worst = max(worst, _rel(ci[j], x_ref))
            assert abs(infos[i * R + j]["rnorm"] - res.rnorm) <= 1e-8 * res.rnorm
    print(f"full batch bj-lsqr k=5: worst coefficient rel diff {worst:.2e}")
    assert worst <= 1e-8
    infos = B.solve(coef, method="mixed_ir", inner_iters=5, outer_lim=2, check_every=5,
                    precond=True, atol=0.0, btol=0.0)
    ch = coef.cpu().numpy()
    for i, (s, bl, h) in oracle.items():
        n = len(bl) * s.K
        ci = _slice(B, ch, i, n)
        for j in range(R):
            r = np.linalg.norm(h[j] - asm.matvec(bl, ci[j], s.n_rows))
            assert abs(infos[i * R + j]["rnorm"] - r) <= 1e-9 * np.linalg.norm(h[j]), (i, j)
            assert r < np.linalg.norm(h[j])


def test_full_batch_patches(full_batch):
    """The benchmark's preconditioner: block-Jacobi over 2 x 2 patches of all 512 instances
    (shift 1e-6).  For the sampled instances the column order of the patch system equals the
    oracle's, 5 preconditioned LSQR steps on the FP64 folded patch matrix give the oracle's
    coefficients (x = R^{-1} y in the original column order) to 1e-8 and its ||r|| to 1e-8, and
    the FP64 refinement on the FP32 folded copy reports for every sampled pair the residual
    ||h - M c|| that the oracle's products give for the returned coefficients (1e-9 of ||h||)."""
    B, specs, oracle = full_batch
    torch = torch_mod()
    shift, P = 1e-6, 2
    print("# full batch: 2 x 2 patch preconditioner", flush=True)
    assert B.precondition(shift, patch=P) == 0
    info = B.patch_info(perm=True)
    assert info["patch"] == P
    pbs = {}
    for i, (s, bl, _) in oracle.items():
        pbs[i] = linalg.patch_blocks(bl, P)
        c0 = B.offsets[i][1]
        n = len(bl) * s.K
        np.testing.assert_array_equal(info["perm"][c0:c0 + n] - c0, linalg.patch_order(pbs[i]))
    coef = torch.empty(R * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
    infos = B.solve(coef, iter_lim=5, atol=0.0, btol=0.0, check_every=5, precond=True)
    ch = coef.cpu().numpy()
    worst = 0.0
    for i, (s, bl, h) in oracle.items():
        n = len(bl) * s.K
        pb = pbs[i]
        facs = linalg.block_jacobi_factors(pb, shift)
        fold = linalg.fold_blocks(pb, facs)
        ci = _slice(B, ch, i, n)
        for j in range(R):
            res = linalg.lsqr(lambda y: linalg.patch_matvec(fold, y, s.n_rows),
                              lambda u: linalg.patch_rmatvec(fold, u), h[j], n,
                              atol=0, btol=0, iter_lim=5)
            x_ref = linalg.patch_recover(pb, facs, res.x)
            worst = max(worst, _rel(ci[j], x_ref))
            assert infos[i * R + j]["iters"] == 5
            assert abs(infos[i * R + j]["rnorm"] - res.rnorm) <= 1e-8 * res.rnorm, (i, j)
    print(f"full batch patch-2 lsqr k=5: worst coefficient rel diff {worst:.2e}")
    assert worst <= 1e-8
    infos = B.solve(coef, method="mixed_ir", inner_iters=5, outer_lim=2, check_every=5,
                    precond=True, atol=0.0, btol=0.0)
    ch = coef.cpu().numpy()
    for i, (s, bl, h) in oracle.items():
        n = len(bl) * s.K
        ci = _slice(B, ch, i, n)
        for j in range(R):
            r = np.linalg.norm(h[j] - asm.matvec(bl, ci[j], s.n_rows))
            assert abs(infos[i * R + j]["rnorm"] - r) <= 1e-9 * np.linalg.norm(h[j]), (i, j)
            assert r < np.linalg.norm(h[j])
