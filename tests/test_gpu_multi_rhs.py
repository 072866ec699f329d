"""Several right-hand sides on one single-problem handle (one matrix, n_rhs forcing terms),
through the C ABI: the assembled right-hand sides, solves and evaluations against the oracle
and against one-at-a-time solves; the info fields acond and ms_assemble; and the per-instance
sizes of a batch against the oracle's geometry."""
import dataclasses

import numpy as np
import pytest

from inputs import configs, feature_params
from inputs.problems import grid_points
from oracle import assemble as asm
from oracle import evaluate as ev
from oracle import geometry as geo
from oracle import linalg

from gpu_util import dev, torch_mod

pytestmark = pytest.mark.gpu

R = 8


def _forcings(spec):
    """8 forcing terms of the multiscale family with seeded amplitudes (the workload's data
    shape: one matrix, several right-hand sides)."""
    rng = np.random.default_rng(21)
    pts = grid_points(spec)
    out = []
    for r in range(R):
        amps = tuple(rng.standard_normal(len(spec.meta["freqs"])))
        out.append(configs.forcing(
            dataclasses.replace(spec, meta={**spec.meta, "amps": amps}), pts))
    return np.stack(out)


@pytest.fixture(scope="module")
def case():
    from paper_2409_01949_amd import Problem
    spec = configs.medium2d()
    W, b = feature_params(spec)
    P = Problem.from_spec(spec, W, b, "fp64")
    F = _forcings(spec)
    P.assemble(dev(F))
    blocks = asm.assemble_blocks(spec, W, b)
    N, n = spec.n_rows, len(blocks) * spec.K
    H = np.stack([asm.rhs(spec, f) for f in F])
    yield spec, P, W, b, F, blocks, H, N, n
    P.destroy()


def test_right_hand_sides(case):
    """The 8 assembled right-hand sides are the oracle's h_r = f_r / sqrt(N_I), exactly."""
    spec, P, W, b, F, blocks, H, N, n = case
    torch = torch_mod()
    hd = torch.empty(R * N, dtype=torch.float64, device="cuda")
    P.copy_rhs(hd)
    assert np.array_equal(hd.cpu().numpy().reshape(R, N), H)


def test_solves_match_the_oracle_and_single_solves(case):
    """5 LSQR steps for all 8 right-hand sides in one call: each within max(1e-10, 50x the
    oracle's spread under row permutations) of the oracle's LSQR on that right-hand side in u,
    and bit-identical to a solve of that right-hand side assembled alone; the evaluation of all 8
    coefficient vectors in one call equals the one-by-one evaluation."""
    from paper_2409_01949_amd import Problem
    spec, P, W, b, F, blocks, H, N, n = case
    torch = torch_mod()
    k = 5
    coef = torch.empty(R * n, dtype=torch.float64, device="cuda")
    infos = P.solve(coef, iter_lim=k, atol=0.0, btol=0.0, check_every=k, n_rhs=R)
    assert len(infos) == R and all(i["iters"] == k for i in infos)
    C = coef.cpu().numpy().reshape(R, n)
    xt = grid_points(spec, (40, 40))
    M = asm.dense_from_blocks(blocks, N, n)
    for r in (0, 3, 7):
        ref = linalg.lsqr(lambda v: M @ v, lambda u: M.T @ u, H[r], n, atol=0, btol=0,
                          iter_lim=k)
        uref = ev.evaluate(spec, W, b, ref.x, xt)
        spread = 0.0
        for seed in range(3):
            perm = np.random.default_rng(seed).permutation(N)
            rp = linalg.lsqr(lambda v: M[perm] @ v, lambda u: M[perm].T @ u, H[r][perm], n,
                             atol=0, btol=0, iter_lim=k)
            spread = max(spread, ev.rel_l2(ev.evaluate(spec, W, b, rp.x, xt), uref))
        du = ev.rel_l2(ev.evaluate(spec, W, b, C[r], xt), uref)
        print(f"rhs {r}: u {du:.2e} (tol {max(1e-10, 50 * spread):.1e})")
        assert du <= max(1e-10, 50 * spread)
    single = Problem.from_spec(spec, W, b, "fp64")
    try:
        for r in (1, 6):
            single.assemble(dev(F[r]))
            c1 = torch.empty(n, dtype=torch.float64, device="cuda")
            single.solve(c1, iter_lim=k, atol=0.0, btol=0.0, check_every=k)
            assert np.array_equal(c1.cpu().numpy(), C[r])
    finally:
        single.destroy()
    pts = dev(xt)
    U = torch.empty(R * xt.shape[0], dtype=torch.float64, device="cuda")
    P.evaluate(coef, pts, U)
    U = U.cpu().numpy().reshape(R, -1)
    for r in (0, 5):
        u1 = torch.empty(xt.shape[0], dtype=torch.float64, device="cuda")
        P.evaluate(coef[r * n:(r + 1) * n], pts, u1)
        assert np.array_equal(u1.cpu().numpy(), U[r])


def test_info_fields(case):
    """ms_assemble is the last assembly's wall time (> 0); acond, when asked for, equals
    sigma_max / sigma_min of the recorded bidiagonal (elmfb_condition_estimate) and is -1
    otherwise; asking for more right-hand sides than assembled is refused."""
    from paper_2409_01949_amd import elmfb
    spec, P, W, b, F, blocks, H, N, n = case
    torch = torch_mod()
    coef = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    infos = P.solve(coef, iter_lim=12, atol=0.0, btol=0.0, check_every=12, n_rhs=2,
                    estimate_cond=True)
    smax, smin, kk = P.condition_estimate()
    assert kk == 12
    assert infos[1]["acond"] == pytest.approx(smax / smin, rel=1e-14)
    assert all(i["ms_assemble"] > 0 for i in infos)
    i0 = P.solve(coef[:n], iter_lim=3, atol=0.0, btol=0.0, check_every=3)
    assert i0["acond"] == -1.0
    with pytest.raises(elmfb.ElmfbError):
        P.solve(torch.empty(9 * n, dtype=torch.float64, device="cuda"), iter_lim=1, n_rhs=9)


def test_batch_instance_sizes():
    """elmfb_batch_query_instances: rows, columns, stored entries, blocks and block points of
    every instance equal the oracle's geometry of that instance; they sum to the totals."""
    from paper_2409_01949_amd import Batch
    specs, _ = configs.batch_instances(n=5, seed=11, n_rhs=2, J_range=(3, 6), K_range=(12, 30),
                                       p_range=(10.0, 30.0))
    specs = specs + [configs.small2d()]
    feats = [feature_params(s) for s in specs]
    B = Batch(specs, [w for w, _ in feats], [b for _, b in feats], 2)
    try:
        per = B.query_instances()
        for s, z in zip(specs, per):
            rows = geo.support_rows(s)
            assert z["n_rows"] == s.n_rows == z["n_interior"]
            assert z["n_phi"] == len(rows) * s.K
            assert z["n_blocks"] == len(rows)
            assert z["n_block_points"] == sum(len(r) for r in rows)
            assert z["nnz"] == sum(len(r) for r in rows) * s.K
        for key in ("n_rows", "n_phi", "nnz", "n_blocks", "n_block_points"):
            assert sum(z[key] for z in per) == B.sizes[key]
    finally:
        B.destroy()
