"""Pins of the oracle's counter-based parameter draws (SplitMix64 in counter mode): the published
outputs of the generator, counter mode against the sequential generator, the uniform mapping's
range and moments, and the parameter layout."""
import json
import os

import numpy as np

from oracle import rng

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.json")))


def test_published_outputs():
    want = [int(h, 16) for h in GOLD["outputs_hex"]]
    assert rng.sequential(GOLD["seed"], len(want)) == want


def test_counter_mode_is_the_sequential_stream():
    for seed in (0, 1, 12345, (1 << 64) - 1):
        seq = rng.sequential(seed, 200)
        got = [int(v) for v in rng.at(seed, np.arange(200))]
        assert got == seq


def test_uniform_range_and_moments():
    n = 200_000
    u = rng.uniform_at(3, np.arange(n), -2.0, 2.0)
    assert u.min() >= -2.0 and u.max() < 2.0
    # mean 0 and variance 4/3 of U[-2, 2], within 5 standard errors
    assert abs(u.mean()) < 5 * np.sqrt(4.0 / 3.0 / n)
    assert abs(u.var() - 4.0 / 3.0) < 5 * np.sqrt((16.0 / 5.0 - 16.0 / 9.0) / n)
    # neighbouring indices are uncorrelated and the histogram is flat
    assert abs(np.corrcoef(u[:-1], u[1:])[0, 1]) < 5 / np.sqrt(n)
    h, _ = np.histogram(u, bins=20, range=(-2.0, 2.0))
    chi2 = np.sum((h - n / 20) ** 2 / (n / 20))
    assert chi2 < 60.0          # 19 degrees of freedom: p < 1e-5 above this


def test_parameter_layout():
    W, b = rng.feature_params(50, 2, 9, (-1.0, 1.0), (-0.5, 0.5))
    assert W.shape == (50, 2) and b.shape == (50,)
    q = 17
    assert W[q, 1] == rng.uniform_at(9, [4 * q + 1], -1.0, 1.0)[0]
    assert b[q] == rng.uniform_at(9, [4 * q + 3], -0.5, 0.5)[0]
    W2, b2 = rng.feature_params(50, 2, 10, (-1.0, 1.0), (-0.5, 0.5))
    assert not np.any(W2 == W) and not np.any(b2 == b)
