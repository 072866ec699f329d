"""Pin of the oracle's global feature inputs (xbar = x): with one draw of W, b shared by every
subdomain of a level, the partition of unity makes a level's columns of feature k sum to the
operator applied to C tanh(W_k . x + b_k) (identity: the function itself; -Laplacian: checked by
second differences of that closed form), divided by sqrt(N) L.  Subdomain-local inputs give
each subdomain a different function, so they fail the same identity."""
import dataclasses

import numpy as np

from inputs import configs
from oracle import assemble as asm
from oracle import basis
from oracle import geometry as geo


def _spec(op, input_norm):
    s = configs.small2d()
    return dataclasses.replace(s, op=op, input_norm=input_norm, levels=((1, 1), (2, 3), (4, 3)))


def _shared(spec, seed=3):
    rng = np.random.default_rng(seed)
    subs = geo.subdomains(spec)
    K = spec.K
    Wl = {l: rng.uniform(-1, 1, (K, spec.dim)) for l in range(spec.n_levels)}
    bl = {l: rng.uniform(-1, 1, K) for l in range(spec.n_levels)}
    W = np.concatenate([Wl[sd.level] for sd in subs])
    b = np.concatenate([bl[sd.level] for sd in subs])
    return W, b, Wl, bl


def _level_sums(spec, M):
    subs = geo.subdomains(spec)
    K = spec.K
    out = {}
    for l in range(spec.n_levels):
        cols = [sd.q0 for sd in subs if sd.level == l]
        out[l] = sum(M[:, q:q + K] for q in cols)
    return out


def _closed(spec, x, W, b):
    C, _, _ = basis.ansatz(x, spec)
    return C[:, None] * np.tanh(x @ W.T + b[None, :])


def test_global_inputs_partition_of_unity_identity():
    spec = _spec("identity", "global")
    W, b, Wl, bl = _shared(spec)
    M = asm.assemble_dense(spec, W, b)
    x = geo.points(spec)
    scale = np.sqrt(spec.n_rows) * spec.n_levels
    for l, S in _level_sums(spec, M).items():
        ref = _closed(spec, x, Wl[l], bl[l]) / scale
        assert np.abs(S - ref).max() <= 1e-13 * np.abs(ref).max()
    # the local reading fails it
    ML = asm.assemble_dense(_spec("identity", "local"), W, b)
    S = _level_sums(spec, ML)[2]
    ref = _closed(spec, x, Wl[2], bl[2]) / scale
    assert np.abs(S - ref).max() > 1e-2 * np.abs(ref).max()


def test_global_inputs_laplacian_rows():
    spec = _spec("neg_laplace", "global")
    W, b, Wl, bl = _shared(spec)
    M = asm.assemble_dense(spec, W, b)
    x = geo.points(spec)
    inner = np.all((x > 0.05) & (x < np.asarray(spec.hi) - 0.05), axis=1)
    scale = np.sqrt(spec.n_rows) * spec.n_levels
    h = 1e-3
    for l, S in _level_sums(spec, M).items():
        f = lambda y: _closed(spec, y, Wl[l], bl[l])
        lap = np.zeros((x.shape[0], spec.K))
        for a in range(2):
            e = np.zeros(2)
            e[a] = h
            lap += (f(x + e) - 2.0 * f(x) + f(x - e)) / h ** 2
        ref = -lap / scale
        err = np.abs(S[inner] - ref[inner]).max() / np.abs(ref[inner]).max()
        assert err < 1e-4, (l, err)
