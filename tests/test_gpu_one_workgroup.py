"""LSQR in one workgroup (systems whose vectors fit in LDS: the damped oscillator of Sec. 4.2, the
small 1D problems and a small 2D one) against the multi-workgroup LSQR on the same system
(ELMFB_PERSISTENT=0) and against the oracle's LSQR.  Every call goes through the C ABI."""
import dataclasses

import numpy as np
import pytest

from inputs import configs
from oracle import assemble as asm
from oracle import evaluate as ev
from oracle import linalg

from gpu_util import OracleSpread, build, torch_mod

pytestmark = pytest.mark.gpu

SPECS = [configs.oscillator(), configs.oscillator(omega0=30.0, J=6, K=5, n=120, levels=((1,), (6,))),
         configs.small1d_multilevel(), configs.tiny1d(),
         # a 2D system small enough for one workgroup: rows covered along both axes
         dataclasses.replace(configs.small2d(), name="tiny2d", n_points=(15, 13),
                             levels=((1, 1), (2, 3)), K=6)]


def _test_points(spec):
    if spec.dim == 1:
        return np.linspace(spec.lo[0], spec.hi[0], 1000)[:, None]
    return np.random.default_rng(5).uniform(spec.lo, spec.hi, (1000, 2))


@pytest.fixture(scope="module", params=SPECS, ids=lambda s: s.name + f"_L{len(s.levels)}")
def case(request):
    spec = request.param
    P, W, b, f = build(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    N, n = spec.n_rows, len(blocks) * spec.K
    M = asm.dense_from_blocks(blocks, N, n)
    h = asm.rhs(spec, f)
    M = np.vstack([M, asm.bc_rows(spec, W, b)])   # no rows when there are no conditions
    yield spec, P, W, b, M, h
    P.destroy()


def _solve(P, n, multi, monkeypatch, **kw):
    torch = torch_mod()
    if multi:
        monkeypatch.setenv("ELMFB_PERSISTENT", "0")
    else:
        monkeypatch.delenv("ELMFB_PERSISTENT", raising=False)
    coef = torch.empty(n, dtype=torch.float64, device="cuda")
    info = P.solve(coef, method="lsqr", **kw)
    return coef.cpu().numpy(), info


def test_chunking_and_repeat_are_bit_identical(case, monkeypatch):
    """40 steps in launches of 3, 7 or all 40 steps, and a repeat: the same step count, stop
    reason and bits (the state and vectors go through global memory unchanged between launches,
    every sum has a fixed order)."""
    spec, P, W, b, M, h = case
    n = M.shape[1]
    runs = [_solve(P, n, False, monkeypatch, iter_lim=40, atol=0.0, btol=0.0, check_every=ce)
            for ce in (40, 3, 7, 40)]
    for c, info in runs:
        # 40 steps, or fewer where a 12-column system meets the tests on x and A^T r first
        assert info["iters"] == runs[0][1]["iters"] <= 40
        assert info["istop"] == runs[0][1]["istop"]
        assert np.array_equal(c, runs[0][0])
        assert info["rnorm"] == runs[0][1]["rnorm"]


@pytest.mark.parametrize("k", [1, 6, 25])
def test_iterates_match_the_multi_workgroup_path_and_the_oracle(case, monkeypatch, k):
    """The k-th iterate of the one-workgroup LSQR and of the multi-workgroup LSQR both equal the
    oracle's in u on 1,000 test points within max(1e-10, 50x the oracle's own spread under row
    permutations); both report the step count and the oracle's ||r|| within max(1e-9, 50x the
    oracle's spread of ||r||) (the oscillator's bidiagonal loses orthogonality within a few
    dozen steps, and row order alone then moves ||r|| by ~1e-3)."""
    spec, P, W, b, M, h = case
    n = M.shape[1]
    xt = _test_points(spec)
    ref = linalg.lsqr(lambda vv: M @ vv, lambda uu: M.T @ uu, h, n, atol=0, btol=0, iter_lim=k)
    uref = ev.evaluate(spec, W, b, ref.x, xt)
    spread = rspread = 0.0
    for seed in range(3):
        perm = np.random.default_rng(seed).permutation(M.shape[0])
        Mp, hp = M[perm], h[perm]
        rp = linalg.lsqr(lambda vv: Mp @ vv, lambda uu: Mp.T @ uu, hp, n, atol=0, btol=0,
                         iter_lim=k)
        spread = max(spread, ev.rel_l2(ev.evaluate(spec, W, b, rp.x, xt), uref))
        rspread = max(rspread, abs(rp.rnorm - ref.rnorm) / max(ref.rnorm, 1e-300))
    tol = max(1e-10, 50 * spread)
    rtol = max(1e-9, 50 * rspread)
    one, i1 = _solve(P, n, False, monkeypatch, iter_lim=k, atol=0.0, btol=0.0, check_every=5)
    multi, i2 = _solve(P, n, True, monkeypatch, iter_lim=k, atol=0.0, btol=0.0, check_every=5)
    d1 = ev.rel_l2(ev.evaluate(spec, W, b, one, xt), uref)
    d2 = ev.rel_l2(ev.evaluate(spec, W, b, multi, xt), uref)
    print(f"{spec.name} k={k}: one-wg {d1:.2e}, multi-wg {d2:.2e} (tol {tol:.1e})")
    assert i1["iters"] == i2["iters"] == k
    assert d1 <= tol and d2 <= tol
    for info in (i1, i2):
        assert abs(info["rnorm"] - ref.rnorm) <= rtol * max(ref.rnorm, 1e-300)


def test_bidiagonal_and_stopping_test(case, monkeypatch):
    """LSQR to its stopping test (atol = btol = 1e-8) on both paths, against the oracle's LSQR to
    the same test on the system and on three row-permuted copies of it (OracleSpread): both
    paths stop on the residual tests with the reported ||r|| equal to ||h - M c|| of the returned
    coefficients to 1e-6; the step count within 3x the oracle's step-count spread plus 2 steps;
    u on the test points, ||r||, sigma_max and sigma_min of the recorded bidiagonal each within
    50x the oracle's spread of that quantity (floor 1e-10), for each path against the oracle and
    between the two paths."""
    spec, P, W, b, M, h = case
    n = M.shape[1]
    xt = _test_points(spec)
    sp = OracleSpread(M, h, n, lambda x: ev.evaluate(spec, W, b, x, xt), atol=1e-8, btol=1e-8,
                      iter_lim=20000)
    out = {}
    for multi in (False, True):
        c, info = _solve(P, n, multi, monkeypatch, iter_lim=20000, atol=1e-8, btol=1e-8,
                         check_every=100)
        smax, smin, kk = P.condition_estimate()
        out[multi] = (c, info, smax, smin)
        r = np.linalg.norm(h - M @ c)
        assert info["istop"] in (1, 2)
        assert abs(info["rnorm"] - r) <= 1e-6 * max(r, 1e-300)
        assert kk == info["iters"]
    print(f"{spec.name}: {sp.describe()}")
    smax_ref, smin_ref = sp.sigma_ref
    for multi, (c, info, smax, smin) in out.items():
        du = ev.rel_l2(ev.evaluate(spec, W, b, c, xt), sp.u_ref)
        dr = abs(info["rnorm"] - sp.ref.rnorm) / sp.ref.rnorm
        print(f"  {'multi' if multi else 'one'}-wg: {info['iters']} steps (tol "
              f"{sp.count_tol():.0f}), u {du:.2e} (tol {sp.tol(sp.u):.1e}), ||r|| {dr:.2e} "
              f"(tol {sp.tol(sp.rnorm):.1e}), sigma_max {smax:.6e} vs {smax_ref:.6e}, sigma_min "
              f"{smin:.4e} vs {smin_ref:.4e} (tol {sp.tol(sp.sigma_min):.1e})")
        assert abs(info["iters"] - sp.ref.itn) <= sp.count_tol()
        assert du <= sp.tol(sp.u)
        assert dr <= sp.tol(sp.rnorm)
        assert abs(smax - smax_ref) <= sp.tol(sp.sigma_max) * smax_ref
        assert abs(smin - smin_ref) <= sp.tol(sp.sigma_min) * smin_ref
    (c1, i1, a1, b1), (c2, i2, a2, b2) = out[False], out[True]
    assert abs(a1 - a2) <= sp.tol(sp.sigma_max) * smax_ref
    assert abs(b1 - b2) <= sp.tol(sp.sigma_min) * smin_ref
    assert abs(i1["iters"] - i2["iters"]) <= sp.count_tol()
