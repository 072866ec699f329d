"""GPU parity of batches: ragged instances (different grids, levels, K, even dimensions) with
several right-hand sides, every kernel launched once over the whole batch, against the CPU
oracle applied instance by instance."""
import numpy as np
import pytest

from inputs import configs, feature_params
from oracle import assemble as asm
from oracle import linalg

from gpu_util import dev, torch_mod

pytestmark = pytest.mark.gpu

R = 3


def _batch_specs():
    specs, _ = configs.batch_instances(n=4, seed=11, n_rhs=R, J_range=(3, 6), K_range=(12, 30),
                                       p_range=(10.0, 30.0))
    return specs + [configs.small2d(), configs.small1d_multilevel()]


def _forcing(spec, r):
    if "rhs_amps" in spec.meta:
        return configs.batch_forcing(spec)[:r]
    base = configs.forcing(spec)
    return np.stack([base * (1.0 + 0.5 * j) for j in range(r)])


@pytest.fixture(scope="module")
def batch():
    from paper_2409_01949_amd import Batch
    specs = _batch_specs()
    feats = [feature_params(s) for s in specs]
    B = Batch(specs, [w for w, _ in feats], [b for _, b in feats], R)
    fs = [_forcing(s, R) for s in specs]
    B.assemble(dev(np.concatenate([f.ravel() for f in fs])))
    oracle = []
    for s, (W, b), f in zip(specs, feats, fs):
        blocks = asm.assemble_blocks(s, W, b)
        oracle.append((s, blocks, np.stack([asm.rhs(s, fj) for fj in f])))
    yield B, oracle
    B.destroy()


def test_batch_offsets(batch):
    B, oracle = batch
    rows = np.cumsum([0] + [s.n_rows for s, _, _ in oracle])
    cols = np.cumsum([0] + [len(bl) * s.K for s, bl, _ in oracle])
    assert np.array_equal(B.offsets[:, 0], rows)
    assert np.array_equal(B.offsets[:, 1], cols)
    assert B.sizes["nnz"] == sum(sum(len(blk.rows) for blk in bl) * s.K for s, bl, _ in oracle)


def test_batch_products(batch):
    """Y = M V and X = M^T U for every instance and right-hand side in one launch each."""
    B, oracle = batch
    torch = torch_mod()
    rng = np.random.default_rng(5)
    V = [rng.standard_normal((R, len(bl) * s.K)) for s, bl, _ in oracle]
    U = [rng.standard_normal((R, s.n_rows)) for s, _, _ in oracle]
    y = torch.empty(R * B.sizes["n_rows"], dtype=torch.float64, device="cuda")
    x = torch.empty(R * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
    B.matvec(dev(np.concatenate([v.ravel() for v in V])), y)
    B.rmatvec(dev(np.concatenate([u.ravel() for u in U])), x)
    yh, xh = y.cpu().numpy(), x.cpu().numpy()
    for i, (s, bl, _) in enumerate(oracle):
        n = len(bl) * s.K
        r0, c0 = B.offsets[i]
        yi = yh[R * r0:R * (r0 + s.n_rows)].reshape(R, s.n_rows)
        xi = xh[R * c0:R * (c0 + n)].reshape(R, n)
        for j in range(R):
            yo = asm.matvec(bl, V[i][j], s.n_rows)
            xo = asm.rmatvec(bl, U[i][j], n)
            assert np.linalg.norm(yi[j] - yo) <= 1e-12 * np.linalg.norm(yo)
            assert np.linalg.norm(xi[j] - xo) <= 1e-12 * np.linalg.norm(xo)


def test_batch_lsqr_iterates(batch):
    """Independent recurrences per (instance, rhs): after 5 steps every pair equals the oracle's
    single-problem LSQR iterate (early iterates, where rounding has not yet been amplified)."""
    B, oracle = batch
    torch = torch_mod()
    coef = torch.empty(R * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
    infos = B.solve(coef, iter_lim=5, atol=0.0, btol=0.0, check_every=2)
    ch = coef.cpu().numpy()
    for i, (s, bl, h) in enumerate(oracle):
        n = len(bl) * s.K
        c0 = B.offsets[i][1]
        ci = ch[R * c0:R * (c0 + n)].reshape(R, n)
        for j in range(R):
            ref = linalg.lsqr(lambda v: asm.matvec(bl, v, s.n_rows),
                              lambda u: asm.rmatvec(bl, u, n), h[j], n, atol=0, btol=0, iter_lim=5)
            info = infos[i * R + j]
            assert info["iters"] == ref.itn
            err = np.linalg.norm(ci[j] - ref.x) / np.linalg.norm(ref.x)
            assert err <= 1e-9, (i, j, err)
            assert abs(info["rnorm"] - ref.rnorm) <= 1e-9 * ref.rnorm


def test_batch_solve_to_residual_tolerance(batch):
    """Every pair stops on its own test ||r|| <= btol ||h||; the oracle's residual of the returned
    coefficients confirms it."""
    B, oracle = batch
    torch = torch_mod()
    coef = torch.empty(R * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
    infos = B.solve(coef, iter_lim=20000, atol=0.0, btol=1e-6, check_every=50)
    ch = coef.cpu().numpy()
    for i, (s, bl, h) in enumerate(oracle):
        n = len(bl) * s.K
        c0 = B.offsets[i][1]
        ci = ch[R * c0:R * (c0 + n)].reshape(R, n)
        for j in range(R):
            info = infos[i * R + j]
            r = np.linalg.norm(asm.matvec(bl, ci[j], s.n_rows) - h[j]) / np.linalg.norm(h[j])
            print(f"instance {i} rhs {j}: istop {info['istop']} after {info['iters']}, "
                  f"rel residual {r:.2e}")
            if info["istop"] == 1:
                assert r <= 1.05e-6
            else:
                assert info["istop"] in (2, 4, 5, 7)
