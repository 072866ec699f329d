"""Pins of the oracle's windows, features, ansatz and operator rows against what the
mathematics fixes: partition of unity, complex-step and finite-difference derivatives,
the single-subdomain special case and the loss <-> least-squares identity."""
import numpy as np
import pytest

from inputs import configs, feature_params
from oracle import assemble as asm
from oracle import basis
from oracle import evaluate as ev
from oracle import geometry as geo

H_CS = 1e-30


def _level_subs(spec, l):
    return [sd for sd in geo.subdomains(spec) if sd.level == l]


@pytest.mark.parametrize("spec", [configs.small1d_multilevel(), configs.small2d()],
                         ids=lambda s: s.name)
def test_partition_of_unity(spec):
    """sum_j omega_j = 1, sum_j grad omega_j = 0, sum_j Lap omega_j = 0 at every point of every
    level (Sec. 3: the windows form a partition of unity on each level)."""
    x = geo.points(spec)
    for l in range(len(spec.levels)):
        subs = _level_subs(spec, l)
        sums = basis.level_sum(x, subs)
        tot = np.zeros(x.shape[0])
        gtot = np.zeros_like(x)
        ltot = np.zeros(x.shape[0])
        gscale = lscale = 1.0
        for sd in subs:
            w, g, lap = basis.window(x, sd, sums)
            tot += w
            gtot += g
            ltot += lap
            gscale = max(gscale, np.abs(g).max())
            lscale = max(lscale, np.abs(lap).max())
        assert np.abs(tot - 1.0).max() < 1e-14
        assert np.abs(gtot).max() < 1e-13 * gscale
        assert np.abs(ltot).max() < 1e-12 * lscale


def test_window_support_and_values():
    """Window is zero outside |x - mu| < sigma and (1+cos(pi t))^2 inside; at the centre 4."""
    sd = geo.Subdomain(0, 0, (0,), np.array([0.3]), np.array([0.2]), 0, False)
    x = np.array([[0.3], [0.1], [0.5], [0.0], [0.4]])
    v, _, _ = basis.window_hat(x, sd)
    assert v[0] == 4.0
    assert v[1] == 0.0 and v[2] == 0.0 and v[3] == 0.0
    assert abs(v[4] - (1 + np.cos(np.pi * 0.5)) ** 2) < 1e-15


def _cs_grad(fun, x, a):
    """Complex-step derivative d fun / d x_a (Squire & Trapp 1998)."""
    xc = x.astype(complex)
    xc[:, a] += 1j * H_CS
    return np.imag(fun(xc)) / H_CS


@pytest.mark.parametrize("spec", [configs.small1d_multilevel(), configs.small2d()],
                         ids=lambda s: s.name)
def test_complex_step_first_derivatives(spec):
    """Analytic gradients of the raw window, the features and the ansatz equal complex-step
    derivatives to ~1e-15 relative."""
    rng = np.random.default_rng(0)
    W, b = feature_params(spec)
    subs = geo.subdomains(spec)
    sd = [s for s in subs if not s.single][len(subs) // 3]
    x = sd.mu[None, :] + (rng.uniform(-0.95, 0.95, size=(40, spec.dim)) * sd.sigma[None, :])
    _, g, _ = basis.window_hat(x, sd)
    q = slice(sd.q0, sd.q0 + spec.K)
    _, gphi, _ = basis.features(x, sd, W[q], b[q])
    _, gC, _ = basis.ansatz(x, spec)
    for a in range(spec.dim):
        cs = _cs_grad(lambda z: basis.window_hat(z, sd)[0], x, a)
        assert np.abs(cs - g[:, a]).max() <= 1e-13 * max(1.0, np.abs(g).max())
        cs = _cs_grad(lambda z: basis.features(z, sd, W[q], b[q])[0], x, a)
        assert np.abs(cs - gphi[:, :, a]).max() <= 1e-13 * max(1.0, np.abs(gphi).max())
        cs = _cs_grad(lambda z: basis.ansatz(z, spec)[0], x, a)
        assert np.abs(cs - gC[:, a]).max() <= 1e-13 * max(1.0, np.abs(gC).max())


def _fd_lap(fun, x, h):
    d = x.shape[1]
    out = -2.0 * d * fun(x)
    for a in range(d):
        e = np.zeros(d)
        e[a] = h
        out = out + fun(x + e) + fun(x - e)
    return out / (h * h)


def test_second_derivatives_fd_order():
    """Laplacians of window, features and ansatz against central second differences: the error
    falls by ~4 when the step halves (second-order agreement)."""
    spec = configs.small2d()
    W, b = feature_params(spec)
    subs = geo.subdomains(spec)
    sd = [s for s in subs if s.level == 2][7]
    rng = np.random.default_rng(1)
    x = sd.mu[None, :] + rng.uniform(-0.8, 0.8, size=(30, 2)) * sd.sigma[None, :]
    q = slice(sd.q0, sd.q0 + spec.K)
    cases = [
        (lambda z: basis.window_hat(z, sd)[0], basis.window_hat(x, sd)[2]),
        (lambda z: basis.features(z, sd, W[q], b[q])[0], basis.features(x, sd, W[q], b[q])[2]),
        (lambda z: basis.ansatz(z, spec)[0], basis.ansatz(x, spec)[2]),
    ]
    for fun, lap in cases:
        e1 = np.abs(_fd_lap(fun, x, 4e-4) - lap).max()
        e2 = np.abs(_fd_lap(fun, x, 2e-4) - lap).max()
        ratio = e1 / e2
        assert 3.3 < ratio < 4.7, ratio
        assert e2 < 1e-5 * max(1.0, np.abs(lap).max())


def _psi_value(spec, sd, W, b, z):
    """psi_q = C omega_j phi_q at points z, with the level normalisation recomputed at z."""
    subs = [s for s in geo.subdomains(spec) if s.level == sd.level]
    sums = basis.level_sum(z, subs)
    q = slice(sd.q0, sd.q0 + spec.K)
    return basis.localized_function(z, spec, sd, W[q], b[q], sums)[0]


def test_operator_rows_fd_2d():
    """Entries of M times sqrt(N) L equal -Lap(C omega_j phi_q) by finite differences of the
    scalar function psi (Sec. 3 "Definition of the system matrices")."""
    spec = configs.small2d()
    W, b = feature_params(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    x = geo.points(spec)
    N, L = x.shape[0], len(spec.levels)
    for bi in (3, 17, len(blocks) - 2):
        blk = blocks[bi]
        pick = blk.rows[:: max(1, len(blk.rows) // 25)]
        sel = np.searchsorted(blk.rows, pick)
        fd = -_fd_lap(lambda z: _psi_value(spec, blk.sd, W, b, z), x[pick], 1e-4)
        got = blk.M[sel] * np.sqrt(N) * L
        assert np.abs(fd - got).max() <= 1e-5 * np.abs(got).max()


def test_operator_rows_complex_step_1d():
    """1D d/dx rows against the complex-step derivative of psi."""
    spec = configs.small1d_multilevel()
    W, b = feature_params(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    x = geo.points(spec)
    N, L = x.shape[0], len(spec.levels)
    for blk in blocks[::3]:
        cs = _cs_grad(lambda z: _psi_value(spec, blk.sd, W, b, z), x[blk.rows], 0)
        got = blk.M * np.sqrt(N) * L
        assert np.abs(cs - got).max() <= 1e-12 * max(1.0, np.abs(got).max())


def test_single_subdomain_special_case():
    """L = 1, J = 1: the window is 1 and the rows are d/dx[tanh(w x) tanh(W xbar + b)]/sqrt(N),
    here differentiated by complex step from the plain product of tanh factors."""
    spec = configs.tiny1d(K=5, J=1, n=40)
    W, b = feature_params(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    assert len(blocks) == 1 and len(blocks[0].rows) == 40
    x = geo.points(spec)[:, 0]
    mu, sig = 0.0, 1.0                                 # [-1, 1]: midpoint 0, half-width 1
    w = spec.ansatz_omega
    xc = x.astype(complex) + 1j * H_CS
    vals = np.tanh(w * xc)[:, None] * np.tanh(np.outer((xc - mu) / sig, W[:, 0]) + b[None, :])
    ref = np.imag(vals) / H_CS / np.sqrt(40.0)
    assert np.abs(blocks[0].M - ref).max() <= 1e-15 * 40


@pytest.mark.parametrize("spec", [configs.small1d_multilevel(), configs.small2d()],
                         ids=lambda s: s.name)
def test_loss_identity(spec):
    """||M a - h||^2 = (1/N_I) sum_n (Op[u_tilde](x_n) - f(x_n))^2 for random a, with Op[u_tilde]
    by finite differences of the evaluated solution (Sec. 3 eq. multilevel_loss vs
    eq. multilevel_ls with the 1/sqrt(N_I) and 1/L scalings)."""
    W, b = feature_params(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    x = geo.points(spec)
    N = x.shape[0]
    n = len(blocks) * spec.K
    rng = np.random.default_rng(7)
    a = rng.standard_normal(n)
    f = configs.forcing(spec)
    h = asm.rhs(spec, f)
    lhs = np.sum((asm.matvec(blocks, a, N) - h) ** 2)
    # keep FD stencils inside the domain: use interior points only for both sides
    if spec.dim == 1:
        hh = 1e-5
        interior = (x[:, 0] > spec.lo[0] + 2 * hh) & (x[:, 0] < spec.hi[0] - 2 * hh)
        xi = x[interior]
        du = (ev.evaluate(spec, W, b, a, xi + hh) - ev.evaluate(spec, W, b, a, xi - hh)) / (2 * hh)
        op = du
    else:
        hh = 1e-4
        interior = np.all((x > np.array(spec.lo) + 2 * hh) & (x < np.array(spec.hi) - 2 * hh), axis=1)
        xi = x[interior]
        op = -_fd_lap(lambda z: ev.evaluate(spec, W, b, a, z), xi, hh)
    Ma = asm.matvec(blocks, a, N)
    # the identity row by row on interior points, then the full sum with the exact rows
    lhs_rows = (Ma[interior] - h[interior]) ** 2
    rhs_rows = (op - f[interior]) ** 2 / N
    assert np.abs(lhs_rows.sum() - rhs_rows.sum()) <= 1e-5 * rhs_rows.sum()
    assert np.allclose(Ma[interior] * np.sqrt(N), op, rtol=0, atol=1e-5 * np.abs(op).max())
    assert lhs >= lhs_rows.sum()


@pytest.mark.parametrize("spec", [configs.small1d_multilevel(), configs.small2d()],
                         ids=lambda s: s.name)
def test_structure_and_block_decomposition(spec):
    """M_{r,q} != 0 exactly where omega_j(x_r) != 0, and sum_j V_j^T M_j W_j equals the matrix
    built point by point (Sec. 3 eq. multilevel_domain_decomp)."""
    W, b = feature_params(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    x = geo.points(spec)
    N = spec.n_rows
    n = len(blocks) * spec.K
    Mb = asm.dense_from_blocks(blocks, N, n)
    Md = asm.assemble_dense(spec, W, b)
    assert np.array_equal(Mb, Md)
    x = geo.points(spec)
    for blk in blocks:
        sub = Md[:, blk.sd.q0:blk.sd.q0 + spec.K]
        nz_rows = np.nonzero(np.any(sub != 0, axis=1))[0]
        # rows of I_j whose entries all round to zero lie on the support edge (a tie in exact
        # arithmetic that the floating-point test |x - mu| < sigma puts inside)
        assert np.all(np.isin(nz_rows, blk.rows))
        zero_rows = np.setdiff1d(blk.rows, nz_rows)
        # (or are rows the operator annihilates for every column: the domain corners, where the
        # hard-constraint factor and its derivatives all vanish)
        if zero_rows.size:
            t = np.abs(x[zero_rows] - blk.sd.mu[None, :]) / blk.sd.sigma[None, :]
            edge = np.max(t, axis=1) > 1.0 - 1e-12
            dead = ~np.any(Md[zero_rows] != 0, axis=1)
            assert np.all(edge | dead)
        if not blk.sd.single:
            sums = basis.level_sum(x, [s for s in geo.subdomains(spec) if s.level == blk.sd.level])
            w, _, _ = basis.window(x, blk.sd, tuple(np.where(s == 0, 1.0, s) if i == 0 else s
                                                    for i, s in enumerate(sums)))
            assert np.all(np.isin(np.nonzero(w != 0)[0], blk.rows))


def test_hard_constraint_and_identity_operator():
    """u_tilde vanishes on the boundary (Sec. 4.3 hard constraint) and, with the identity
    operator, M a sqrt(N) equals the evaluated solution at the grid points."""
    spec = configs.small2d()
    W, b = feature_params(spec)
    rng = np.random.default_rng(3)
    n = spec.n_subdomains() * spec.K
    a = rng.standard_normal(n)
    x = geo.points(spec)
    onb = (x[:, 0] == spec.lo[0]) | (x[:, 0] == spec.hi[0]) | (x[:, 1] == spec.lo[1]) | \
          (x[:, 1] == spec.hi[1])
    u = ev.evaluate(spec, W, b, a, x)
    assert np.all(u[onb] == 0.0)
    import dataclasses
    ident = dataclasses.replace(spec, op="identity")
    blocks = asm.assemble_blocks(ident, W, b)
    Mu = asm.matvec(blocks, a, x.shape[0]) * np.sqrt(x.shape[0])
    assert np.abs(Mu - u).max() <= 1e-13 * np.abs(u).max()


def test_grid_definition_matches_inputs():
    """The oracle's grid and the input generator's grid are the same doubles."""
    from inputs import grid_points
    for spec in (configs.ode1d(), configs.small2d(), configs.poisson3l()):
        assert np.array_equal(geo.points(spec), grid_points(spec))


def test_oscillator_exact_solution():
    """The damped oscillator's closed form (Sec. 4.2 eq. harm_u_exact) solves
    m u'' + mu u' + k u = 0 (complex step for u', central second differences for u'') and meets
    u(0) = 1, u'(0) = 0."""
    spec = configs.oscillator(omega0=80.0)
    m, mu, k = spec.meta["osc"]
    t = np.linspace(0.05, 0.95, 181)
    u = configs.exact(spec, t[:, None])
    du = np.imag(configs.exact(spec, (t + 1j * H_CS)[:, None])) / H_CS
    hh = 1e-4
    d2u = (configs.exact(spec, (t + hh)[:, None]) - 2 * u + configs.exact(spec, (t - hh)[:, None])) \
        / hh ** 2
    res = m * d2u + mu * du + k * u
    assert np.abs(res).max() <= 1e-4 * k * np.abs(u).max()
    assert configs.exact(spec, np.array([[0.0]]))[0] == pytest.approx(1.0, abs=1e-14)
    du0 = np.imag(configs.exact(spec, np.array([[1j * H_CS]]))) / H_CS
    assert abs(du0[0]) <= 1e-10 * spec.meta["omega0"]


def test_oscillator_rows_and_constraint_rows():
    """Operator rows of m u'' + mu u' + k u: entries times sqrt(N) L equal m FD2(psi) +
    mu CS(psi) + k psi of the scalar function psi = omega_j phi_q; the two soft-constraint rows
    are sqrt(lambda) (1/L) psi(0) and sqrt(lambda) (1/L) psi'(0) (complex step), nonzero only on
    the subdomains whose support holds t = 0."""
    spec = configs.oscillator(omega0=30.0, J=6, K=5, n=120, levels=((1,), (6,)))
    m, mu, k = spec.meta["osc"]
    W, b = feature_params(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    x = geo.points(spec)
    N, L = x.shape[0], len(spec.levels)
    hh = 1e-4
    for blk in blocks:
        inner = (x[blk.rows, 0] > 2 * hh) & (x[blk.rows, 0] < 1 - 2 * hh)
        z = x[blk.rows][inner]
        psi = lambda y: _psi_value(spec, blk.sd, W, b, y)
        ref = m * (psi(z + hh) - 2 * psi(z) + psi(z - hh)) / hh ** 2 + \
            mu * _cs_grad(psi, z, 0) + k * psi(z)
        got = blk.M[inner] * np.sqrt(N) * L
        assert np.abs(ref - got).max() <= 1e-5 * np.abs(got).max()
    B = asm.bc_rows(spec, W, b)
    assert B.shape == (2, len(blocks) * spec.K)
    z0 = np.zeros((1, 1))
    for blk in blocks:
        q = slice(blk.sd.q0, blk.sd.q0 + spec.K)
        if not geo.in_support(z0, blk.sd)[0]:
            assert not np.any(B[:, q])
            continue
        psi = lambda y: _psi_value(spec, blk.sd, W, b, y)
        assert np.allclose(B[0, q], k / L * psi(z0)[0], rtol=1e-14, atol=0)
        assert np.allclose(B[1, q], 30.0 / L * _cs_grad(psi, z0, 0)[0], rtol=1e-12, atol=0)
    h = asm.rhs(spec, configs.forcing(spec))
    assert h.shape == (N + 2,) and h[N] == k and h[N + 1] == 0.0


def test_oscillator_least_squares_solution_tracks_the_exact_solution():
    """The paper's baseline (omega0 = 80, J = 20, K = 12, delta = 2.9, 260 points): the dense QR
    least-squares solution of [N; B] a = h reproduces the exact solution on 1,000 test points
    (rel-L2 below 1e-4; measured 4.8e-6), and without the constraint rows it does not (the
    homogeneous equation alone is solved by a = 0)."""
    spec = configs.oscillator()
    W, b = feature_params(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    N, n = spec.n_rows, len(blocks) * spec.K
    M = np.vstack([asm.dense_from_blocks(blocks, N, n), asm.bc_rows(spec, W, b)])
    h = asm.rhs(spec, configs.forcing(spec))
    from oracle import linalg
    c = linalg.householder_lstsq(M, h)
    xt = np.linspace(0.0, 1.0, 1000)[:, None]
    ue = configs.exact(spec, xt)
    err = np.linalg.norm(ev.evaluate(spec, W, b, c, xt) - ue) / np.linalg.norm(ue)
    assert err <= 1e-4
    c0 = linalg.householder_lstsq(M[:N], h[:N])
    assert np.linalg.norm(c0) <= 1e-12
