"""Counter-based draws of the random-feature parameters (the method fixes W and b at random,
Sec. 3; their generator is not stated, so this is a reading of the paper: SplitMix64 of Steele,
Lea and Flood 2014, in counter mode).  Test infrastructure: the library's own implementation is
checked against this one bit for bit.

SplitMix64 steps its state by the odd constant gamma = 0x9e3779b97f4a7c15 and returns the state
passed through a 64-bit finaliser (two xor-shift-multiply rounds with the constants of the
published generator, then a final xor-shift).  In counter mode the value with index c of stream
`seed` is the finaliser of seed + (c + 1) gamma (mod 2^64): the (c + 1)-th output of the
sequential generator started at `seed`.  A uniform on [lo, hi) is lo + (hi - lo) u with
u = (z >> 11) 2^-53 (the top 53 bits, exact in FP64), each operation rounded on its own.

Parameter q of the full per-level subdomain grids (level, then subdomain in x-major order, then
feature k; the order of the caller-supplied arrays) draws W[q][a] at index 4 q + a and b[q] at
index 4 q + 3.
"""
from __future__ import annotations

import numpy as np

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
MUL1 = 0xBF58476D1CE4E5B9
MUL2 = 0x94D049BB133111EB


def finalise(z: int) -> int:
    """The SplitMix64 output function on one 64-bit integer (plain Python integers)."""
    z &= MASK
    z = ((z ^ (z >> 30)) * MUL1) & MASK
    z = ((z ^ (z >> 27)) * MUL2) & MASK
    return z ^ (z >> 31)


def sequential(seed: int, n: int):
    """The first n outputs of the sequential generator started at state `seed`."""
    x = seed & MASK
    out = []
    for _ in range(n):
        x = (x + GAMMA) & MASK
        out.append(finalise(x))
    return out


def at(seed: int, index) -> np.ndarray:
    """Counter-mode values for an array of indices (numpy uint64, arithmetic mod 2^64)."""
    c = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK) + (c + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MUL1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MUL2)
    return z ^ (z >> np.uint64(31))


def uniform_at(seed: int, index, lo: float, hi: float) -> np.ndarray:
    u = (at(seed, index) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    span = np.float64(hi) - np.float64(lo)
    t = span * u
    return np.float64(lo) + t


def feature_params(n_params: int, dim: int, seed: int, w_range, b_range):
    """W [n_params, dim] and b [n_params] of the full per-level subdomain grids."""
    q = np.arange(n_params, dtype=np.uint64)
    W = np.stack([uniform_at(seed, 4 * q + a, w_range[0], w_range[1]) for a in range(dim)],
                 axis=1)
    b = uniform_at(seed, 4 * q + 3, b_range[0], b_range[1])
    return np.ascontiguousarray(W), np.ascontiguousarray(b)
