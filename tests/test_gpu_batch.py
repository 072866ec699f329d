"""GPU parity of batches: ragged instances (different grids, levels, K, even dimensions) with
several right-hand sides, every kernel launched once over the whole batch, against the CPU
oracle applied instance by instance."""
import numpy as np
import pytest

from inputs import configs, feature_params
from oracle import assemble as asm
from oracle import linalg, lowprec

from gpu_util import check_rounded_fold, dev, fold_tolerance, rounded_variants, torch_mod

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


def _make(store_prec, specs=None):
    from paper_2409_01949_amd import Batch
    specs = _batch_specs() if specs is None else specs
    feats = [feature_params(s) for s in specs]
    B = Batch(specs, [w for w, _ in feats], [b for _, b in feats], R, store_prec=store_prec)
    fs = [_forcing(s, R) for s in specs]
    B.assemble(dev(np.concatenate([f.ravel() for f in fs])))
    oracle = []
    for s, (W, b), f in zip(specs, feats, fs):
        blocks = asm.assemble_blocks(s, W, b)
        oracle.append((s, blocks, np.stack([asm.rhs(s, fj) for fj in f])))
    return B, oracle


@pytest.fixture(scope="module")
def batch():
    B, oracle = _make("fp64")
    yield B, oracle
    B.destroy()


@pytest.fixture(scope="module")
def batch32():
    B, oracle = _make("fp32")
    yield B, oracle
    B.destroy()


def _coefs(B, coef, oracle):
    ch = coef.cpu().numpy()
    out = []
    for i, (s, bl, _) in enumerate(oracle):
        n = len(bl) * s.K
        c0 = B.offsets[i][1]
        out.append(ch[R * c0:R * (c0 + n)].reshape(R, n))
    return out


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


def test_batch_rmatvec_every_tile(batch):
    """Every point-tile variant of the batched M^T U pass gives the oracle's product."""
    B, oracle = batch
    torch = torch_mod()
    rng = np.random.default_rng(9)
    U = [rng.standard_normal((R, s.n_rows)) for s, _, _ in oracle]
    x = torch.empty(R * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
    for tile in (16, 32):
        B.set_tile("fp64", tile)
        B.rmatvec(dev(np.concatenate([u.ravel() for u in U])), x)
        xh = x.cpu().numpy()
        for i, (s, bl, _) in enumerate(oracle):
            n = len(bl) * s.K
            c0 = B.offsets[i][1]
            xi = xh[R * c0:R * (c0 + n)].reshape(R, n)
            for j in range(R):
                xo = asm.rmatvec(bl, U[i][j], n)
                assert np.linalg.norm(xi[j] - xo) <= 1e-12 * np.linalg.norm(xo), (tile, i, j)
    ms, chosen = B.autotune("fp64", reps=3)
    print("fp64 tile timings (ms):", ms, "chosen", chosen)
    assert chosen in ms and set(ms) == {16, 32}


def test_batch_block_jacobi_iterates(batch):
    """Block-Jacobi preconditioned LSQR per pair (factors of G_bb + 1e-6 trace/K I, accurate to
    ~1e-10) equals the oracle's preconditioned LSQR after 1 and 5 steps."""
    B, oracle = batch
    torch = torch_mod()
    shift = 1e-6
    assert B.precondition(shift) == 0
    for k in (1, 5):
        coef = torch.empty(R * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
        infos = B.solve(coef, iter_lim=k, atol=0.0, btol=0.0, check_every=5, precond=True)
        cs = _coefs(B, coef, oracle)
        worst = 0.0
        for i, (s, bl, h) in enumerate(oracle):
            n = len(bl) * s.K
            facs = linalg.block_jacobi_factors(bl, shift)
            for j in range(R):
                x_ref, res = linalg.preconditioned_lsqr(
                    lambda v: asm.matvec(bl, v, s.n_rows), lambda u: asm.rmatvec(bl, u, n), bl,
                    facs, h[j], n, atol=0, btol=0, iter_lim=k)
                err = np.linalg.norm(cs[i][j] - x_ref) / np.linalg.norm(x_ref)
                worst = max(worst, err)
                assert infos[i * R + j]["iters"] == k
                assert abs(infos[i * R + j]["rnorm"] - res.rnorm) <= 1e-8 * res.rnorm
        print(f"bj-lsqr k={k}: worst coefficient rel diff {worst:.2e}")
        assert worst <= 1e-8


def test_batch_block_jacobi_beats_plain(batch):
    """With the production shift 1e-12, 200 preconditioned steps leave a smaller residual than
    200 plain steps on every pair that has not converged, and the oracle confirms the residual
    of the returned coefficients."""
    B, oracle = batch
    torch = torch_mod()
    B.precondition(1e-12)
    coef = torch.empty(R * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
    pre = B.solve(coef, iter_lim=200, atol=0.0, btol=0.0, check_every=50, precond=True)
    cs = _coefs(B, coef, oracle)
    plain = B.solve(torch.empty_like(coef), iter_lim=200, atol=0.0, btol=0.0, check_every=50)
    for i, (s, bl, h) in enumerate(oracle):
        for j in range(R):
            p, q = pre[i * R + j], plain[i * R + j]
            r = np.linalg.norm(asm.matvec(bl, cs[i][j], s.n_rows) - h[j])
            print(f"instance {i} rhs {j}: ||r|| plain {q['rnorm']:.3e}, bj {p['rnorm']:.3e}, "
                  f"oracle residual of bj coefficients {r:.3e}")
            assert abs(r - p["rnorm"]) <= 1e-6 * np.linalg.norm(h[j]) + 1e-3 * r
            assert p["rnorm"] <= q["rnorm"] * 1.01


def test_batch_mixed_refinement_matches_oracle(batch32):
    """FP64 refinement around inner LSQR on the FP32 copy of the block-Jacobi preconditioned
    matrix M R^{-1} (formed in FP64, rounded to nearest even): after 1 and 2 outer steps of 5
    inner steps every pair equals the oracle's refinement on its folded blocks, mapped back by
    R^{-1}.  The FP32 copies come from FP64 products summed in different orders, so an entry
    next to a rounding boundary may round differently: tolerance 1e-7."""
    _mixed_vs_oracle(*batch32, lowprec.to_f32)


def test_batch_mixed_refinement_fp16_matches_oracle():
    """The same refinement on the IEEE binary16 rounding of the folded M R^{-1}; refinement on
    the unfolded FP16 copy is refused.  An FP16 entry that rounds differently moves the
    coefficients by 1e-6 to 1e-4 (measured on the oracle), so the shift is 1e-3, which leaves few
    entries within fold_tolerance of a boundary, and the device result must match the oracle's
    refinement on one of the admissible roundings.  small2d (many such entries) is left out."""
    B, oracle = _make("fp16", [s for s in _batch_specs() if s.name != "small2d"])
    torch = torch_mod()
    coef = torch.empty(R * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
    with pytest.raises(Exception, match="FP16"):
        B.solve(coef, method="mixed_ir", inner_iters=5, outer_lim=1, precond=False, atol=0.0,
                btol=0.0)
    _mixed_vs_oracle(B, oracle, lowprec.to_fp16, shift=1e-3)
    B.destroy()


def _mixed_vs_oracle(B, oracle, rounding, shift=1e-6):
    """After 1 and 2 outer steps of 5 inner steps every pair equals the oracle's refinement on
    its folded blocks (for FP16: on one of the admissible roundings, rounded_variants), mapped
    back by R^{-1}, to 1e-7 in the coefficients."""
    torch = torch_mod()
    B.precondition(shift)
    inner = 5
    for outer in (1, 2):
        coef = torch.empty(R * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
        infos = B.solve(coef, method="mixed_ir", inner_iters=inner, outer_lim=outer, check_every=5,
                        precond=True, atol=0.0, btol=0.0)
        cs = _coefs(B, coef, oracle)
        worst = 0.0
        for i, (s, bl, h) in enumerate(oracle):
            wi = 0.0
            n = len(bl) * s.K
            facs = linalg.block_jacobi_factors(bl, shift)
            fb = linalg.fold_blocks(bl, facs)
            if rounding is lowprec.to_fp16:
                variants = rounded_variants(fb, rounding, s.K, shift)
            else:
                variants = [[rounding(blk.M) for blk in fb]]
            los = [[asm.Block(blk.sd, blk.rows, Mv) for blk, Mv in zip(fb, Ms)] for Ms in variants]
            for j in range(R):
                info = infos[i * R + j]
                assert info["outer_iters"] == outer and info["iters"] == outer * inner
                best = np.inf
                for lo in los:
                    cy, hist = linalg.refine_lsqr(
                        lambda v: asm.matvec(fb, v, s.n_rows), lambda u: asm.rmatvec(fb, u, n),
                        lambda v: asm.matvec(lo, v, s.n_rows), lambda u: asm.rmatvec(lo, u, n),
                        h[j], n, outer, inner)
                    c = linalg.block_apply(bl, facs, cy)
                    best = min(best, np.linalg.norm(cs[i][j] - c) / np.linalg.norm(c))
                wi = max(wi, best)
                r = np.linalg.norm(asm.matvec(bl, cs[i][j], s.n_rows) - h[j])
                assert abs(info["rnorm"] - r) <= 1e-9 * np.linalg.norm(h[j])
            print(f"  instance {i} ({s.name}): coefficient rel diff {wi:.2e} "
                  f"({len(los)} admissible roundings)")
            worst = max(worst, wi)
        print(f"mixed outer={outer}: worst coefficient rel diff {worst:.2e}")
        assert worst <= 1e-7


@pytest.mark.parametrize("store", ["fp32", "fp16"])
def test_batch_folded_copies_match_oracle(store):
    """elmfb_batch_precondition forms M_b R_b^{-1} for every block of every instance: the FP64
    folded blocks equal the oracle's within the sensitivity of the shifted Cholesky factor
    (fold_tolerance) and the low-precision copy is their rounding to nearest even (entries within
    that distance of a boundary may round either way); the copy of M in that precision is no
    longer held."""
    B, oracle = _make(store)
    _check_folded(B, oracle, store, 1e-4)
    B.destroy()


def test_batch_timing_keeps_tables_intact():
    """The tuner and the kernel timer write the row gather's output into a row-sized vector: on a
    batch with more rows than columns (6,712 against 2,924) they leave every other table intact,
    so the fold that follows them still matches the oracle."""
    B, oracle = _make("fp32")
    assert B.sizes["n_rows"] > B.sizes["n_phi"]
    B.tune("fp32", reps=1, use_cache=False)
    B.time_kernels("fp32", reps=2)
    B.time_kernels("fp64", reps=2)
    _check_folded(B, oracle, "fp32", 1e-4)
    B.destroy()


def _check_folded(B, oracle, store, shift):
    torch = torch_mod()
    B.precondition(shift)
    nnz = B.sizes["nnz"]
    b64 = torch.empty(nnz, dtype=torch.float64, device="cuda")
    blo = torch.empty(nnz, dtype={"fp32": torch.float32, "fp16": torch.float16}[store],
                      device="cuda")
    table = B.copy_blocks(b64, "fp64", folded=True)
    B.copy_blocks(blo, store, folded=True)
    with pytest.raises(Exception):
        B.copy_blocks(blo, store, folded=False)
    torch.cuda.synchronize()
    h64, hlo = b64.cpu().numpy(), blo.double().cpu().numpy()
    rounding = lowprec.to_f32 if store == "fp32" else lowprec.to_fp16
    k, worst, nm, na = 0, 0.0, 0, 0
    for i, (s, bl, _) in enumerate(oracle):
        fb = linalg.fold_blocks(bl, linalg.block_jacobi_factors(bl, shift))
        for blk in fb:
            inst, lvl, ix0, nx, iy0, ny, K, off = (int(v) for v in table[k])
            k += 1
            npt = nx * ny
            assert inst == i and K == s.K and npt == blk.M.shape[0]
            A64 = h64[off:off + K * npt].reshape(K, npt).T
            Alo = hlo[off:off + K * npt].reshape(K, npt).T
            tol = fold_tolerance(blk.M, K, shift)
            err = np.abs(A64 - blk.M).max()
            worst = max(worst, err / tol)
            assert err <= tol
            m, a = check_rounded_fold(Alo, blk.M, rounding, tol)
            nm += m
            na += a
    assert k == len(table)
    print(f"batch {store}: FP64 fold worst {worst:.2f} of its tolerance; rounded copy {nm} entries "
          f"off the oracle's rounding, {na} within tolerance of a boundary")


def test_batch_mixed_solve_to_tolerance(batch32):
    """Mixed refinement with the production shift stops each pair on its FP64 tests: pairs
    reporting istop 1 satisfy ||h - M c|| <= btol ||h|| by the oracle's matvec; pairs reporting
    istop 2 (least-squares optimality, ||M^T r|| <= atol ||M|| ||r||) have the optimal residual of
    the oracle's dense QR solution (their systems are inconsistent)."""
    B, oracle = batch32
    torch = torch_mod()
    B.precondition(1e-12)
    btol = 1e-6
    coef = torch.empty(R * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
    infos = B.solve(coef, method="mixed_ir", inner_iters=2000, outer_lim=6, check_every=50,
                    precond=True, atol=btol, btol=btol)
    cs = _coefs(B, coef, oracle)
    n_conv = n_opt = 0
    for i, (s, bl, h) in enumerate(oracle):
        for j in range(R):
            info = infos[i * R + j]
            r = np.linalg.norm(asm.matvec(bl, cs[i][j], s.n_rows) - h[j]) / np.linalg.norm(h[j])
            print(f"instance {i} rhs {j}: istop {info['istop']}, outer {info['outer_iters']}, "
                  f"inner {info['iters']}, rel residual {r:.2e}")
            if info["istop"] == 1:
                n_conv += 1
                assert r <= btol * (1 + 1e-2)
            elif info["istop"] == 2:
                n_opt += 1
                n = len(bl) * s.K
                M = asm.dense_from_blocks(bl, s.n_rows, n)
                x = linalg.householder_lstsq(M, h[j])
                r_opt = np.linalg.norm(M @ x - h[j]) / np.linalg.norm(h[j])
                print(f"    optimal rel residual {r_opt:.6e}")
                assert r <= r_opt * (1 + 1e-3)
            else:
                assert info["istop"] == 7 and info["outer_iters"] == 6
    assert n_conv >= 1 and n_opt >= 1


def test_batch_warm_start(batch32):
    """Warm starts: preconditioned LSQR from x0 equals the oracle's preconditioned LSQR from x0
    after 5 steps (x = x0 + R^{-1} y, y for h - M x0), and refinement from a nearly converged x0
    stops at once while meeting the same ||h - M c|| <= btol ||h|| target (oracle residual)."""
    B, oracle = batch32
    torch = torch_mod()
    shift = 1e-6
    B.precondition(shift)
    rng = np.random.default_rng(21)
    X0 = [rng.standard_normal((R, len(bl) * s.K)) for s, bl, _ in oracle]
    x0 = dev(np.concatenate([x.ravel() for x in X0]))
    coef = torch.empty(R * B.sizes["n_phi"], dtype=torch.float64, device="cuda")
    B.solve(coef, iter_lim=5, atol=0.0, btol=0.0, check_every=5, precond=True, x0=x0)
    cs = _coefs(B, coef, oracle)
    worst = 0.0
    for i, (s, bl, h) in enumerate(oracle):
        n = len(bl) * s.K
        facs = linalg.block_jacobi_factors(bl, shift)
        for j in range(R):
            x_ref, _ = linalg.preconditioned_lsqr(
                lambda v: asm.matvec(bl, v, s.n_rows), lambda u: asm.rmatvec(bl, u, n), bl, facs,
                h[j], n, x0=X0[i][j], atol=0, btol=0, iter_lim=5)
            worst = max(worst, np.linalg.norm(cs[i][j] - x_ref) / np.linalg.norm(x_ref))
    print(f"warm bj-lsqr k=5: worst coefficient rel diff {worst:.2e}")
    assert worst <= 1e-8
    # refinement: cold to btol, then warm from the cold result
    btol = 1e-4
    cold = B.solve(coef, method="mixed_ir", inner_iters=2000, outer_lim=4, check_every=50,
                   precond=True, atol=0.0, btol=btol)
    warm_coef = torch.empty_like(coef)
    warm = B.solve(warm_coef, method="mixed_ir", inner_iters=2000, outer_lim=4, check_every=50,
                   precond=True, atol=0.0, btol=btol, x0=coef)
    cs = _coefs(B, warm_coef, oracle)
    for i, (s, bl, h) in enumerate(oracle):
        for j in range(R):
            c, w = cold[i * R + j], warm[i * R + j]
            r = np.linalg.norm(asm.matvec(bl, cs[i][j], s.n_rows) - h[j]) / np.linalg.norm(h[j])
            print(f"instance {i} rhs {j}: cold istop {c['istop']} after {c['iters']}, warm istop "
                  f"{w['istop']} after {w['iters']}, rel residual {r:.2e}")
            if c["istop"] == 1:
                assert w["istop"] == 1 and w["iters"] == 0 and w["outer_iters"] == 0
                assert r <= btol * (1 + 1e-2)


@pytest.mark.parametrize("ahead,rows", [(4, 1), (16, 2), (8, 2)])
def test_batch_shapes_products_and_iterates(batch, ahead, rows):
    """Every launch shape the tuner can choose for the M V look-ahead and the row gather: products
    per instance and right-hand side to 1e-12 and 5 LSQR steps to 1e-9 against the oracle (the
    shape is restored afterwards)."""
    B, oracle = batch
    torch = torch_mod()
    B.set_shape("fp64", rmvb_tile=32, mvb_ahead=ahead, gather_rows=rows)
    try:
        test_batch_products(batch)
        test_batch_lsqr_iterates(batch)
    finally:
        B.set_shape("fp64", rmvb_tile=32, mvb_ahead=8, gather_rows=1)


def test_batch_tuner_and_its_cache(batch32):
    """The tuner times every candidate of the three passes and keeps the fastest of each; the
    same batch class then takes the cached choice without timing; a shape outside the candidates
    is refused."""
    from paper_2409_01949_amd import elmfb
    B, oracle = batch32
    t = B.tune("fp32", reps=2, use_cache=False)
    print(t)
    assert not t["from_cache"]
    assert set(t["ms_rmvb"]) == {16, 32, 64} and set(t["ms_mvb"]) == {4, 8, 16}
    assert set(t["ms_gather"]) == {1, 2}
    assert t["rmvb_tile"] == min(t["ms_rmvb"], key=t["ms_rmvb"].get)
    assert t["mvb_ahead"] == min(t["ms_mvb"], key=t["ms_mvb"].get)
    assert t["gather_rows"] == min(t["ms_gather"], key=t["ms_gather"].get)
    c = B.tune("fp32", reps=2, use_cache=True)
    assert c["from_cache"] and all(c[k] == t[k] for k in ("rmvb_tile", "mvb_ahead", "gather_rows"))
    with pytest.raises(elmfb.ElmfbError):
        B.set_shape("fp64", rmvb_tile=64)
    with pytest.raises(elmfb.ElmfbError):
        B.set_shape("fp32", mvb_ahead=5)
