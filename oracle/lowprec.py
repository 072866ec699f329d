"""Round-to-nearest-even from float64 to float32, to bfloat16 (8 exponent bits, 7 stored
mantissa bits) and to IEEE binary16 (5 exponent bits, 10 stored mantissa bits), written from the
IEEE-754 definition: scale by the power of two that puts the last kept bit at the units place,
round half to even, scale back.  Test infrastructure, not part of the product path."""
from __future__ import annotations

import numpy as np


def to_f32(x):
    """float64 -> float32 with round-to-nearest-even (returned as float64 values)."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def _to_small(x, mant_bits, exp_bits):
    """float64 -> a format with mant_bits stored mantissa bits and exp_bits exponent bits
    (bias 2^(exp_bits-1) - 1), round-to-nearest-even in one step, as float64 values.

    Normal range: mant_bits + 1 significant bits; below 2^emin the spacing is fixed at
    2^(emin - mant_bits) (subnormals); magnitudes that round above the largest finite value
    become infinities."""
    emax = 2 ** (exp_bits - 1) - 1
    emin = 1 - emax
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = (x != 0) & np.isfinite(x)
    ax = np.abs(x[nz])
    e = np.floor(np.log2(ax))
    # guard against log2 rounding across a power of two
    e = np.where(2.0 ** e > ax, e - 1, e)
    e = np.where(2.0 ** (e + 1) <= ax, e + 1, e)
    e = np.maximum(e, float(emin))
    ulp = 2.0 ** (e - mant_bits)
    r = np.rint(ax / ulp) * ulp           # np.rint rounds half to even
    largest = (2.0 - 2.0 ** -mant_bits) * 2.0 ** emax
    r = np.where(r > largest, np.inf, r)
    out[nz] = np.sign(x[nz]) * r
    out[~np.isfinite(x)] = x[~np.isfinite(x)]
    return out


def to_bf16(x):
    """float64 -> bfloat16 with round-to-nearest-even (returned as float64 values): 8 significant
    bits, spacing 2^-133 below 2^-126, infinities above the largest finite value."""
    return _to_small(x, 7, 8)


def to_fp16(x):
    """float64 -> IEEE binary16 with round-to-nearest-even (returned as float64 values): 11
    significant bits, spacing 2^-24 below 2^-14, infinities above 65504."""
    return _to_small(x, 10, 5)
