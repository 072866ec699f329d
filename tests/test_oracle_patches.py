"""Pins of the oracle's block-Jacobi preconditioner over patches of neighbouring subdomains:
P = 1 is the per-subdomain preconditioner exactly; patch blocks are the members' blocks placed
on the union of their rows (checked against the dense assembly); one patch over a whole level
gives the Cholesky factor of the whole shifted Gram matrix, whose folded matrix has the Gram
matrix I - lambda R^{-T} R^{-1} and lets LSQR finish a consistent system in a few steps; the
preconditioned minimiser maps back to the minimiser of M."""
import dataclasses

import numpy as np
import pytest

from inputs import configs, feature_params
from oracle import assemble as asm
from oracle import linalg


def _case(J=5, K=8, n=22, dim=2, seed=3):
    if dim == 2:
        spec = dataclasses.replace(configs.small2d(), levels=((J, J),), K=K, n_points=(n, n),
                                   seed=seed)
    else:
        spec = dataclasses.replace(configs.tiny1d(), levels=((J,),), K=K, n_points=(n,),
                                   delta=1.9, seed=seed)
    W, b = feature_params(spec)
    blocks = asm.assemble_blocks(spec, W, b)
    M = asm.dense_from_blocks(blocks, spec.n_rows, len(blocks) * spec.K)
    return spec, blocks, M


def test_patch_one_is_the_subdomain_preconditioner():
    spec, blocks, M = _case()
    pb = linalg.patch_blocks(blocks, 1)
    assert len(pb) == len(blocks)
    np.testing.assert_array_equal(linalg.patch_order(pb), np.arange(M.shape[1]))
    for p, blk in zip(pb, blocks):
        np.testing.assert_array_equal(p.rows, blk.rows)
        np.testing.assert_array_equal(p.M, blk.M)
    fp = linalg.block_jacobi_factors(pb, 1e-10)
    fb = linalg.block_jacobi_factors(blocks, 1e-10)
    for a, c in zip(fp, fb):
        np.testing.assert_array_equal(a, c)


@pytest.mark.parametrize("J,P,dim", [(5, 2, 2), (6, 3, 2), (7, 2, 1)])
def test_patch_blocks_against_the_dense_matrix(J, P, dim):
    """Patch counts, member order, rows = union of the members' rows, and products of the patch
    system equal those of the dense M with its columns permuted into patch order."""
    spec, blocks, M = _case(J=J, dim=dim, n=22 if dim == 2 else 60)
    pb = linalg.patch_blocks(blocks, P)
    npa = -(-J // P)
    assert len(pb) == npa ** dim
    sizes = sorted({len(p.members) for p in pb})
    assert sizes[-1] == P ** dim
    for p in pb:
        jj = [tuple(m.sd.jj) for m in p.members]
        assert jj == sorted(jj)
        assert all(tuple(j // P for j in t) == p.index for t in jj)
        np.testing.assert_array_equal(p.rows, np.unique(np.concatenate([m.rows for m in p.members])))
        c = 0
        for m in p.members:
            inside = np.isin(p.rows, m.rows)
            np.testing.assert_array_equal(p.M[inside, c:c + spec.K], m.M)
            assert not np.any(p.M[~inside, c:c + spec.K])
            c += spec.K
    perm = linalg.patch_order(pb)
    np.testing.assert_array_equal(np.sort(perm), np.arange(M.shape[1]))
    rng = np.random.default_rng(1)
    y = rng.standard_normal(M.shape[1])
    u = rng.standard_normal(M.shape[0])
    Mp = M[:, perm]
    np.testing.assert_allclose(linalg.patch_matvec(pb, y, M.shape[0]), Mp @ y, rtol=0,
                               atol=1e-13 * np.abs(Mp).sum(axis=1).max() * np.abs(y).max())
    np.testing.assert_allclose(linalg.patch_rmatvec(pb, u), Mp.T @ u, rtol=0,
                               atol=1e-13 * np.abs(Mp).sum(axis=0).max() * np.abs(u).max())


def test_one_patch_over_the_level_is_the_global_cholesky():
    """P >= J: a single patch; R^T R = M^T M + lambda I, the folded matrix Q = M R^{-1} has
    Q^T Q = I - lambda R^{-T} R^{-1}, and R^{-1} y maps products of Q to products of M."""
    spec, blocks, M = _case(J=4, K=6, n=18)
    pb = linalg.patch_blocks(blocks, 4)
    assert len(pb) == 1
    (R,) = linalg.block_jacobi_factors(pb, 1e-8)
    perm = linalg.patch_order(pb)
    Mp = M[:, perm]
    G = Mp.T @ Mp
    lam = 1e-8 * np.trace(G) / G.shape[0]
    np.testing.assert_allclose(R.T @ R, G + lam * np.eye(G.shape[0]), rtol=0,
                               atol=1e-12 * np.abs(G).max())
    (Q,) = [p.M for p in linalg.fold_blocks(pb, [R])]
    Ri = np.linalg.inv(R)
    np.testing.assert_allclose(Q.T @ Q, np.eye(Q.shape[1]) - lam * Ri.T @ Ri, rtol=0, atol=1e-9)
    rng = np.random.default_rng(2)
    y = rng.standard_normal(Q.shape[1])
    folded = linalg.fold_blocks(pb, [R])
    x = linalg.patch_recover(pb, [R], y)
    np.testing.assert_allclose(M @ x, linalg.patch_matvec(folded, y, M.shape[0]), rtol=0,
                               atol=1e-9 * np.linalg.norm(M @ x))


def test_whole_level_patch_makes_lsqr_finish_quickly():
    """With the whole level orthonormalised, LSQR on a consistent right-hand side h = M x
    reaches ||r|| <= 1e-8 ||h|| within a few steps (M has full column rank here, so Q has
    orthonormal columns up to lambda and one step suffices); per-subdomain blocks need many more."""
    spec, blocks, M = _case(J=4, K=6, n=18)
    x_true = np.random.default_rng(4).standard_normal(M.shape[1])
    h = M @ x_true
    its = {}
    for P in (1, 4):
        pb = linalg.patch_blocks(blocks, P)
        folded = linalg.fold_blocks(pb, linalg.block_jacobi_factors(pb, 1e-12))
        res = linalg.lsqr(lambda y: linalg.patch_matvec(folded, y, M.shape[0]),
                          lambda u: linalg.patch_rmatvec(folded, u), h, M.shape[1],
                          atol=0.0, btol=1e-8, iter_lim=5000)
        assert res.istop == 1
        its[P] = res.itn
    assert its[4] <= 3
    assert its[1] >= 3 * its[4]


def test_patch_preconditioning_keeps_the_minimiser():
    """An overdetermined full-rank case: lstsq on the folded patch system, mapped back with
    R^{-1}, is the least-squares solution of M."""
    spec, blocks, M = _case(J=3, K=3, n=40, dim=1)
    assert M.shape[0] > M.shape[1] and np.linalg.matrix_rank(M) == M.shape[1]
    h = np.random.default_rng(5).standard_normal(M.shape[0])
    pb = linalg.patch_blocks(blocks, 2)
    F = linalg.block_jacobi_factors(pb, 1e-14)
    folded = linalg.fold_blocks(pb, F)
    Q = np.zeros((M.shape[0], M.shape[1]))
    o = 0
    for p in folded:
        Q[p.rows, o:o + p.M.shape[1]] = p.M
        o += p.M.shape[1]
    y = np.linalg.lstsq(Q, h, rcond=None)[0]
    x = linalg.patch_recover(pb, F, y)
    ref = np.linalg.lstsq(M, h, rcond=None)[0]
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-8 * np.abs(ref).max())
