"""Rounding of FP64 values to the narrow operand formats of the Gaussian sketch.

* bfloat16: 8 significant bits, FP32 exponent range, round to nearest even.
* FP8 E4M3 (OCP "fn" variant): 4 significant bits for |x| >= 2**-6, fixed quantum 2**-9
  below that, largest finite value 448; round to nearest even, saturating at 448.

Pinned by: exhaustive comparison with torch's own bfloat16 / float8_e4m3fn casts on
representable neighbourhoods (tests), which are independent library routines.
"""
from __future__ import annotations

import numpy as np


def _round_sig(x: np.ndarray, bits: int) -> np.ndarray:
    """Round to ``bits`` significant bits, ties to even (no exponent limits)."""
    x = np.asarray(x, dtype=np.float64)
    mant, expo = np.frexp(x)                  # x = mant * 2**expo, |mant| in [0.5, 1)
    scaled = np.ldexp(mant, bits)             # |scaled| in [2**(bits-1), 2**bits)
    return np.ldexp(np.rint(scaled), expo - bits)


def round_bf16(x) -> np.ndarray:
    return _round_sig(x, 8)


def round_e4m3(x) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    normal = _round_sig(x, 4)
    sub = np.rint(x * 2.0 ** 9) * 2.0 ** -9
    out = np.where(np.abs(x) < 2.0 ** -6, sub, normal)
    return np.clip(out, -448.0, 448.0)


def round_to(x, dtype: str) -> np.ndarray:
    if dtype == "bf16":
        return round_bf16(x)
    if dtype == "e4m3":
        return round_e4m3(x)
    if dtype == "f32":
        return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    if dtype == "f64":
        return np.asarray(x, dtype=np.float64)
    raise ValueError(dtype)
