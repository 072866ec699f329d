"""Pins of the oracle's L-shaped Helmholtz problem (Sec. 4.4): counts the paper states, the
manufactured solution against finite differences, the partition of unity over the kept
subdomains (the windows of discarded subdomains are gone from the normalisation), the
(Lap + k^2) rows against finite differences of psi = omega_j phi_q, the least-squares <-> loss
identity with the boundary term, and a weak calibration against the paper's baseline table."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from inputs import configs, feature_params
from oracle import assemble as asm
from oracle import basis
from oracle import evaluate as ev
from oracle import geometry as geo
from oracle import linalg

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_helmholtz_baseline.json")))

SMALL = configs.helmholtz(omega=2.0, levels=((1, 1), (4, 4), (6, 6)), K=6, n=30)
BASE = configs.helmholtz()
MULTI = configs.helmholtz(levels=((1, 1), (8, 8), (16, 16)))


def _fd_lap(fun, x, h):
    out = -4.0 * fun(x)
    for a in range(2):
        e = np.zeros(2)
        e[a] = h
        out = out + fun(x + e) + fun(x - e)
    return out / (h * h)


def _params(spec):
    return geo.kept_parameters(spec, *feature_params(spec))


def test_counts_as_in_the_paper():
    """80 x 80 grid points less the 40 x 40 in the removed quarter, 80 + 40 + 40 + 40 + 40 + 80
    boundary points, 16 x 16 - 8 x 8 = 192 and 8 x 8 - 4 x 4 = 48 kept subdomains, 1 x 1 kept."""
    c = GOLD["counts"]
    assert geo.points(BASE).shape[0] == c["interior_points"]
    xb = configs.boundary_points(BASE)
    assert xb.shape[0] == c["boundary_points"]
    subs = geo.subdomains(MULTI)
    assert [sum(1 for s in subs if s.level == l) for l in range(3)] == \
        [c["kept_subdomains_1"], c["kept_subdomains_8"], c["kept_subdomains_16"]]
    assert len(geo.subdomains(BASE)) == c["kept_subdomains_16"]
    # boundary points lie on the boundary of the L, none twice
    x, y = xb[:, 0], xb[:, 1]
    on = (np.isclose(y, 0) | np.isclose(x, 0) | (np.isclose(x, 1) & (y <= 0.5)) |
          (np.isclose(y, 0.5) & (x >= 0.5)) | (np.isclose(x, 0.5) & (y >= 0.5)) |
          (np.isclose(y, 1) & (x <= 0.5)))
    assert on.all() and len(np.unique(np.round(xb, 12), axis=0)) == xb.shape[0]


def test_manufactured_solution():
    """f of eq. helmholtz_f equals Lap u + k^2 u of eq. helmholtz_exact by central second
    differences, with the error falling ~4x when the step halves."""
    rng = np.random.default_rng(0)
    x = rng.uniform(0.05, 0.95, size=(200, 2))
    for omega in (1.0, 8.0):
        spec = configs.helmholtz(omega=omega)
        u = lambda z: configs.exact(spec, z)
        f = configs.forcing(spec, x)
        k2 = spec.meta["k"] ** 2
        e1 = np.abs(_fd_lap(u, x, 2e-4) + k2 * u(x) - f).max()
        e2 = np.abs(_fd_lap(u, x, 1e-4) + k2 * u(x) - f).max()
        assert e2 <= 1e-5 * np.abs(f).max()
        assert 3.0 < e1 / e2 < 5.0


@pytest.mark.parametrize("spec", [SMALL, MULTI], ids=["small", "multilevel"])
def test_partition_of_unity_over_kept_subdomains(spec):
    """sum over the kept subdomains of omega_j = 1, of grad omega_j = 0 and of Lap omega_j = 0
    at every interior and boundary collocation point of every level."""
    x = np.vstack([geo.points(spec), configs.boundary_points(spec)])
    subs = geo.subdomains(spec)
    for l in range(len(spec.levels)):
        lev = [s for s in subs if s.level == l]
        sums = basis.level_sum(x, lev)
        assert np.all(sums[0] > 0)
        tot, gt, lt = np.zeros(x.shape[0]), np.zeros_like(x), np.zeros(x.shape[0])
        gs = ls = 1.0
        for sd in lev:
            m = geo.in_support(x, sd)
            w, g, lap = basis.window(x[m], sd, tuple(s[m] for s in sums))
            tot[m] += w
            gt[m] += g
            lt[m] += lap
            gs, ls = max(gs, np.abs(g).max()), max(ls, np.abs(lap).max())
        assert np.abs(tot - 1).max() < 1e-14
        assert np.abs(gt).max() < 1e-13 * gs
        assert np.abs(lt).max() < 1e-12 * ls


def test_rows_against_finite_differences():
    """Entries of M times sqrt(N_I) L equal (Lap + k^2)(omega_j phi_q) by finite differences of
    psi, the window renormalised over the kept subdomains at the shifted points."""
    spec = SMALL
    W, b = _params(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    x = geo.points(spec)
    N, L = x.shape[0], len(spec.levels)
    k2 = spec.meta["k"] ** 2
    subs = geo.subdomains(spec)
    for bi in (0, 5, len(blocks) - 3):
        blk = blocks[bi]
        lev = [s for s in subs if s.level == blk.sd.level]
        q = slice(blk.sd.q0, blk.sd.q0 + spec.K)

        def psi(z):
            return basis.localized_function(z, spec, blk.sd, W[q], b[q],
                                            basis.level_sum(z, lev))[0]

        pick = blk.rows[:: max(1, len(blk.rows) // 20)]
        sel = np.searchsorted(blk.rows, pick)
        fd = _fd_lap(psi, x[pick], 1e-4) + k2 * psi(x[pick])
        got = blk.M[sel] * np.sqrt(N) * L
        assert np.abs(fd - got).max() <= 1e-5 * np.abs(got).max()


def test_loss_identity_with_boundary_rows():
    """For random coefficients a: ||[N; B] a - [h; h_B]||^2 = (1/N_I) sum_i (Lap u + k^2 u -
    f)^2(x_i) + lambda_bc (1/N_B) sum_b (u(x_b) - g_b)^2, with u evaluated by the oracle's
    evaluate function and Lap u by finite differences (interior term checked row by row on
    points whose stencil stays in the L), the boundary term exactly."""
    spec = SMALL
    W, b = _params(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    x = geo.points(spec)
    N = x.shape[0]
    n = len(blocks) * spec.K
    xb = configs.boundary_points(spec)
    g = configs.exact(spec, xb)
    B = asm.dirichlet_rows(spec, W, b, xb)
    f = configs.forcing(spec, x)
    h = asm.rhs(spec, f, g)
    a = np.random.default_rng(3).standard_normal(n)
    r = np.concatenate([asm.matvec(blocks, a, N), B @ a]) - h
    hh = 1e-4
    inner = (np.all((x > 3 * hh) & (x < 1 - 3 * hh), axis=1) &
             ~((x[:, 0] > 0.5 - 3 * hh) & (x[:, 1] > 0.5 - 3 * hh)))
    u = lambda z: ev.evaluate(spec, W, b, a, z)
    op = _fd_lap(u, x[inner], hh) + spec.meta["k"] ** 2 * u(x[inner])
    assert np.allclose(r[:N][inner] * np.sqrt(N), op - f[inner], rtol=0,
                       atol=1e-5 * np.abs(op).max())
    lam, nb = spec.meta["lambda_bc"], xb.shape[0]
    bterm = lam / nb * np.sum((u(xb) - g) ** 2)
    assert np.isclose(np.sum(r[N:] ** 2), bterm, rtol=1e-12)


@pytest.mark.slow
def test_baseline_against_the_paper():
    """The paper's baseline (omega = 8, 192 subdomains, K = 16) after the full 15,000-step LSQR
    budget: e_L1 on the 96 x 96 test points inside the L and kappa(M) within 10x of the printed
    1.3e-2 and 3.7e8 (seeds, generator and precision differ)."""
    spec = BASE
    W, b = _params(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    x = geo.points(spec)
    N, n = x.shape[0], len(blocks) * spec.K
    xb = configs.boundary_points(spec)
    M = np.vstack([asm.dense_from_blocks(blocks, N, n), asm.dirichlet_rows(spec, W, b, xb)])
    S = sp.csr_matrix(M)
    h = asm.rhs(spec, configs.forcing(spec, x), configs.exact(spec, xb))
    res = linalg.lsqr(lambda v: S @ v, lambda u: S.T @ u, h, n, atol=0, btol=0, iter_lim=15000)
    xt = geo.points(spec, spec.meta["n_test"])
    e = ev.e_l1(ev.evaluate(spec, W, b, res.x, xt), configs.exact(spec, xt))
    s = np.linalg.svd(M, compute_uv=False)
    g = GOLD["baseline"]
    print(f"helmholtz baseline: e_L1 {e:.3e} (paper {g['e_L1']}), kappa {s[0] / s[-1]:.2e} "
          f"(paper {g['cond_M']})")
    assert g["e_L1"] / 10 <= e <= g["e_L1"] * 10
    assert g["cond_M"] / 10 <= s[0] / s[-1] <= g["cond_M"] * 10
