"""GPU parity of the descriptor's parameter and input options: W and b drawn by the library from a
seed (no caller arrays) assemble the oracle's matrix for the oracle's draw of the same stream,
in single problems and batches; global feature inputs (xbar = x) give the oracle's entries,
constraint rows, Dirichlet rows and evaluations.  Every call goes through the C ABI."""
import dataclasses

import numpy as np
import pytest

from inputs import configs
from inputs.problems import grid_points
from oracle import assemble as asm
from oracle import evaluate as ev
from oracle import rng

from gpu_util import dev, device_blocks, torch_mod

pytestmark = pytest.mark.gpu


def _blocks_err(P, spec, blocks):
    got = device_blocks(P, spec.K, "fp64")
    assert len(got) == len(blocks)
    return max(np.abs(Mg - blk.M).max() / max(np.abs(blk.M).max(), 1e-300)
               for (_, Mg), blk in zip(got, blocks))


def _oracle_params(spec):
    return rng.feature_params(spec.n_subdomains() * spec.K, spec.dim, spec.seed, spec.w_range,
                              spec.b_range)


@pytest.mark.parametrize("spec", [dataclasses.replace(configs.small2d(), seed=11),
                                  dataclasses.replace(configs.ode1d(), seed=(1 << 63) + 3)],
                         ids=lambda s: s.name)
def test_library_drawn_parameters(spec):
    """Entries to 1e-12 of each block's largest entry and evaluations to 1e-12, against the
    oracle assembled from its own draw of the stream."""
    from paper_2409_01949_amd import Problem
    torch = torch_mod()
    W, b = _oracle_params(spec)
    P = Problem.from_spec(spec, None, None)
    try:
        P.assemble(dev(configs.forcing(spec)))
        err = _blocks_err(P, spec, asm.assemble_blocks(spec, W, b))
        coef = np.random.default_rng(2).standard_normal(P.sizes["n_phi"])
        xt = grid_points(spec, spec.meta["n_test"])
        u = torch.empty(xt.shape[0], dtype=torch.float64, device="cuda")
        P.evaluate(dev(coef), dev(xt), u)
        ref = ev.evaluate(spec, W, b, coef, xt)
        eu = np.abs(u.cpu().numpy() - ref).max() / np.abs(ref).max()
        print(f"{spec.name}: drawn parameters, entries {err:.2e}, evaluation {eu:.2e}")
        assert err <= 1e-12 and eu <= 1e-12
    finally:
        P.destroy()


def test_batch_with_library_drawn_parameters():
    """A batch whose instances pass no parameters: products against the oracle's blocks for the
    oracle's draws, to 1e-12."""
    from paper_2409_01949_amd import Batch
    torch = torch_mod()
    specs, _ = configs.batch_instances(n=3, seed=4, n_rhs=2, J_range=(3, 5), K_range=(12, 20),
                                       p_range=(10.0, 20.0))
    specs = [dataclasses.replace(s, seed=100 + i) for i, s in enumerate(specs)]
    B = Batch(specs, [None] * 3, [None] * 3, 2)
    try:
        f = np.concatenate([configs.batch_forcing(s)[:2].ravel() for s in specs])
        B.assemble(dev(f))
        blocks = [asm.assemble_blocks(s, *_oracle_params(s)) for s in specs]
        r = np.random.default_rng(5)
        V = [r.standard_normal((2, len(bl) * s.K)) for s, bl in zip(specs, blocks)]
        y = torch.empty(2 * B.sizes["n_rows"], dtype=torch.float64, device="cuda")
        B.matvec(dev(np.concatenate([v.ravel() for v in V])), y)
        yh = y.cpu().numpy()
        for i, (s, bl) in enumerate(zip(specs, blocks)):
            r0 = B.offsets[i][0]
            yi = yh[2 * r0:2 * (r0 + s.n_rows)].reshape(2, s.n_rows)
            for j in range(2):
                yo = asm.matvec(bl, V[i][j], s.n_rows)
                assert np.linalg.norm(yi[j] - yo) <= 1e-12 * np.linalg.norm(yo)
    finally:
        B.destroy()


GLOBAL = [dataclasses.replace(configs.small2d(), input_norm="global"),
          dataclasses.replace(configs.small1d_multilevel(), input_norm="global")]


@pytest.mark.parametrize("spec", GLOBAL, ids=lambda s: s.name)
def test_global_inputs_entries_and_evaluation(spec):
    from paper_2409_01949_amd import Problem
    from inputs import feature_params
    torch = torch_mod()
    W, b = feature_params(spec)
    P = Problem.from_spec(spec, W, b)
    try:
        P.assemble(dev(configs.forcing(spec)))
        err = _blocks_err(P, spec, asm.assemble_blocks(spec, W, b))
        coef = np.random.default_rng(3).standard_normal(P.sizes["n_phi"])
        xt = grid_points(spec, spec.meta["n_test"])
        u = torch.empty(xt.shape[0], dtype=torch.float64, device="cuda")
        P.evaluate(dev(coef), dev(xt), u)
        ref = ev.evaluate(spec, W, b, coef, xt)
        eu = np.abs(u.cpu().numpy() - ref).max() / np.abs(ref).max()
        print(f"{spec.name}: global inputs, entries {err:.2e}, evaluation {eu:.2e}")
        assert err <= 1e-12 and eu <= 1e-12
    finally:
        P.destroy()


def test_global_inputs_constraint_rows():
    """The oscillator's initial-condition rows (value and derivative) with global inputs."""
    from paper_2409_01949_amd import Problem
    from inputs import feature_params
    torch = torch_mod()
    spec = dataclasses.replace(configs.oscillator(omega0=30.0, J=6, K=5, n=120,
                                                  levels=((1,), (6,))), input_norm="global")
    W, b = feature_params(spec)
    P = Problem.from_spec(spec, W, b)
    try:
        P.assemble(dev(configs.forcing(spec)))
        Bo = asm.bc_rows(spec, W, b)
        Bd = torch.empty(Bo.size, dtype=torch.float64, device="cuda")
        P.copy_bc(Bd)
        Bg = Bd.cpu().numpy().reshape(Bo.shape)
        err = _blocks_err(P, spec, asm.assemble_blocks(spec, W, b))
        print(f"oscillator, global inputs: entries {err:.2e}, constraint rows "
              f"{np.abs(Bg - Bo).max() / np.abs(Bo).max():.2e}")
        assert err <= 1e-12
        for r in range(Bo.shape[0]):
            assert np.abs(Bg[r] - Bo[r]).max() <= 1e-12 * np.abs(Bo[r]).max()
    finally:
        P.destroy()


def test_global_inputs_dirichlet_rows():
    """The L-shaped Helmholtz problem's Dirichlet rows at points with global inputs."""
    from paper_2409_01949_amd import Problem
    from inputs import feature_params
    from oracle import geometry as geo
    torch = torch_mod()
    spec = dataclasses.replace(configs.helmholtz(levels=((4, 4),), n=24), input_norm="global")
    Wf, bf = feature_params(spec)                 # every subdomain of the full grids
    xb = configs.boundary_points(spec)
    wgt = asm.dirichlet_weight(spec, xb.shape[0])
    g = np.zeros(xb.shape[0])
    P = Problem.from_spec(spec, Wf, bf, bc_pts=xb, bc_vals=g, bc_weight=wgt)
    try:
        P.assemble(dev(configs.forcing(spec)))
        W, b = geo.kept_parameters(spec, Wf, bf)
        Do = asm.dirichlet_rows(spec, W, b, xb)
        Dd = torch.empty(Do.size, dtype=torch.float64, device="cuda")
        P.copy_bc(Dd)
        Dg = Dd.cpu().numpy().reshape(Do.shape)
        e = np.abs(Dg - Do).max() / np.abs(Do).max()
        print(f"helmholtz, global inputs: Dirichlet rows {e:.2e}")
        assert e <= 1e-12
    finally:
        P.destroy()
