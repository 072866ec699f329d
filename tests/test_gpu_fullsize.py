"""Parity at the full sizes of the multilevel 2D workloads (400^2 points, levels 1/4/16, K=96;
1024^2 points, levels 1/8/16/32/64, K=256) in the configuration the benchmark times (FP64 matrix
plus FP32 copy, block-Jacobi, FP64 refinement).  The oracle cannot assemble these systems whole,
so it evaluates the same definitions at a sample of grid points: rows of M v and the M^T u
contribution of those rows are compared element by element; solver results are checked through
properties that hold at any size."""
import numpy as np
import pytest

from inputs import configs, feature_params, grid_points
from oracle import assemble as asm

from gpu_util import dev, torch_mod

pytestmark = pytest.mark.gpu

N_SAMPLE = 1500


@pytest.fixture(scope="module", params=["poisson3l", "poisson5l"])
def full(request):
    from paper_2409_01949_amd import Problem
    spec = getattr(configs, request.param)()
    W, b = feature_params(spec)
    print(f"# {spec.name}: define + assemble", flush=True)
    P = Problem.from_spec(spec, W, b, "fp32")
    f = configs.forcing(spec)
    P.assemble(dev(f))
    N = spec.n_rows
    rng = np.random.default_rng(0)
    nx, ny = spec.n_points
    corners = [0, ny - 1, (nx - 1) * ny, N - 1]
    rows = np.unique(np.concatenate([rng.choice(N, N_SAMPLE, replace=False), corners]))
    x = grid_points(spec)[rows]
    # the oracle's blocks at the sampled points; its 1/sqrt(N) scale refers to the sample size
    blocks = asm.assemble_blocks(spec, W, b, x)
    fix = np.sqrt(len(rows)) / np.sqrt(N)
    for blk in blocks:
        blk.M = blk.M * fix
    yield spec, P, f, rows, blocks
    P.destroy()


def test_full_points_and_rhs(full):
    spec, P, f, rows, _ = full
    torch = torch_mod()
    xy_d = torch.empty((spec.n_rows, spec.dim), dtype=torch.float64, device="cuda")
    P.points(xy_d)
    xy = xy_d.cpu().numpy()
    assert np.array_equal(xy[rows], grid_points(spec)[rows])
    h = torch.empty(spec.n_rows, dtype=torch.float64, device="cuda")
    P.copy_rhs(h)
    hr = h.cpu().numpy()[rows]
    assert np.abs(hr - f[rows] / np.sqrt(spec.n_rows)).max() <= 1e-15 * np.abs(hr).max()


def test_full_matvec_rows(full):
    spec, P, _, rows, blocks = full
    torch = torch_mod()
    n = P.sizes["n_phi"]
    v = np.random.default_rng(1).standard_normal(n)
    y = torch.empty(spec.n_rows, dtype=torch.float64, device="cuda")
    P.matvec(dev(v), y)
    ys = y.cpu().numpy()[rows]
    ref = asm.matvec(blocks, v, len(rows))
    err = np.abs(ys - ref).max() / np.abs(ref).max()
    print(f"{spec.name}: sampled rows of M v, max rel err {err:.2e}")
    assert err <= 1e-12


def test_full_rmatvec_of_sampled_rows(full):
    """u nonzero only on the sampled rows: M^T u is the oracle's sampled blocks transposed."""
    spec, P, _, rows, blocks = full
    torch = torch_mod()
    n = P.sizes["n_phi"]
    us = np.random.default_rng(2).standard_normal(len(rows))
    u = np.zeros(spec.n_rows)
    u[rows] = us
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    P.rmatvec(dev(u), x)
    ref = asm.rmatvec(blocks, us, n)
    err = np.abs(x.cpu().numpy() - ref).max() / np.abs(ref).max()
    print(f"{spec.name}: M^T u on sampled rows, max rel err {err:.2e}")
    assert err <= 1e-12


def test_full_refinement_reports_true_residual(full):
    """Preconditioned FP64 refinement around FP32 inner LSQR: the residual it reports is
    ||h - M c|| recomputed by the FP64 products, and it does not grow between outer steps."""
    spec, P, _, _, _ = full
    torch = torch_mod()
    n = P.sizes["n_phi"]
    P.precondition(1e-12)
    h = torch.empty(spec.n_rows, dtype=torch.float64, device="cuda")
    P.copy_rhs(h)
    prev = None
    for outer in (1, 2):
        c = torch.empty(n, dtype=torch.float64, device="cuda")
        info = P.solve(c, method="mixed_ir", inner_iters=100, outer_lim=outer, atol=0.0, btol=0.0,
                       check_every=50, precond=True)
        y = torch.empty(spec.n_rows, dtype=torch.float64, device="cuda")
        P.matvec(c, y)
        r = float(torch.linalg.vector_norm(h - y))
        print(f"{spec.name} outer={outer}: reported {info['rnorm']:.6e}, recomputed {r:.6e}")
        assert abs(info["rnorm"] - r) <= 1e-9 * float(torch.linalg.vector_norm(h))
        if prev is not None:
            assert info["rnorm"] <= prev * (1 + 1e-12)
        prev = info["rnorm"]
