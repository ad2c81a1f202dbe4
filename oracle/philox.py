"""Philox4x32-10, written from the published description (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11).

Pinned by: the generator's published known-answer vectors (a fixture in the tests), bit
equality with rocRAND's independent ``philox4x32_10_engine`` (a library routine compiled from
its source header in the tests), plus uniformity statistics.

A block maps a 128-bit counter ``(c0, c1, c2, c3)`` and a 64-bit key ``(k0, k1)`` to four
32-bit words.  One round multiplies ``c0`` and ``c2`` by the two Philox multipliers, keeps
the high and low halves of the 64-bit products and mixes them with ``c1``, ``c3`` and the
key; between rounds the key is advanced by the two Weyl constants.
"""
from __future__ import annotations

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
_MULT0 = np.uint64(0xD2511F53)
_MULT1 = np.uint64(0xCD9E8D57)
_WEYL0 = np.uint64(0x9E3779B9)
_WEYL1 = np.uint64(0xBB67AE85)
ROUNDS = 10


def philox4x32(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  Arguments are integers or integer arrays (values < 2**32).

    Returns a tuple of four ``uint64`` arrays holding the 32-bit output words.
    """
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & MASK32 for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    shift = np.uint64(32)
    for r in range(ROUNDS):
        if r:
            k0 = (k0 + _WEYL0) & MASK32
            k1 = (k1 + _WEYL1) & MASK32
        p0 = _MULT0 * c0          # exact: both factors < 2**32
        p1 = _MULT1 * c2
        hi0, lo0 = p0 >> shift, p0 & MASK32
        hi1, lo1 = p1 >> shift, p1 & MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def key_of(seed: int):
    """Philox key from a 64-bit seed: low and high 32-bit halves."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def block(seed: int, idx, sub, stream: int):
    """Counter layout used for every draw: ``(lo32(idx), hi32(idx), sub, stream)``."""
    idx = np.asarray(idx, dtype=np.uint64)
    k0, k1 = key_of(seed)
    return philox4x32(idx & MASK32, idx >> np.uint64(32), sub, stream, k0, k1)
