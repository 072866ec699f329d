"""Round-to-nearest-even from float64 to float32 and to bfloat16 (8 exponent bits, 7 stored
mantissa bits), written from the IEEE-754 definition: scale by the power of two that puts the
last kept bit at the units place, round half to even, scale back."""
from __future__ import annotations

import numpy as np


def to_f32(x):
    """float64 -> float32 with round-to-nearest-even (returned as float64 values)."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def to_bf16(x):
    """float64 -> bfloat16 with round-to-nearest-even (returned as float64 values).

    Normal range: 8 significant bits; below 2^-126 the spacing is fixed at 2^-133 (subnormals);
    magnitudes that round above the largest finite bfloat16 become infinities."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = (x != 0) & np.isfinite(x)
    ax = np.abs(x[nz])
    e = np.floor(np.log2(ax))
    # guard against log2 rounding across a power of two
    e = np.where(2.0 ** e > ax, e - 1, e)
    e = np.where(2.0 ** (e + 1) <= ax, e + 1, e)
    e = np.maximum(e, -126.0)
    ulp = 2.0 ** (e - 7)
    r = np.rint(ax / ulp) * ulp           # np.rint rounds half to even
    maxbf = (2.0 - 2.0 ** -7) * 2.0 ** 127
    r = np.where(r > maxbf, np.inf, r)
    out[nz] = np.sign(x[nz]) * r
    out[~np.isfinite(x)] = x[~np.isfinite(x)]
    return out
