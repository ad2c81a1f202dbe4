"""Random draws that define a sketch realisation, regenerated from ``(seed, counters)``.

Every draw comes from one Philox4x32-10 block with counter ``(lo32(idx), hi32(idx), sub,
stream)`` and key ``seed``.  Streams:

====== ================== ===============================================================
stream object             counter and bits
====== ================== ===============================================================
1      sign diagonal D    ``idx = j >> 7``; bit ``j & 31`` of word ``(j >> 5) & 3``; set = -1
2      SRHT rows R        draw ``t``: ``idx = t``; words 0,1 form a 64-bit uniform
3      sparse rows        column ``j``, draw ``t``: ``idx = j``, ``sub = t >> 2``, word ``t & 3``
4      sparse signs       column ``j``: ``idx = j >> 2``, word ``j & 3``, bit ``t``; set = -1
5      Gaussian entries   ``G[i, j]``: ``idx = j``, ``sub = i >> 2``; words (0,1) give rows
                          ``4q, 4q+1`` and words (2,3) rows ``4q+2, 4q+3`` by Box-Muller
====== ================== ===============================================================

Sampling without replacement uses Floyd's algorithm: to pick ``c`` distinct values from
``[0, P)``, for ``t = 0..c-1`` let ``i = P - c + t``, draw ``x`` uniform on ``[0, i]`` and
take ``x`` unless it was already taken, in which case take ``i``.  The uniform integer is
``floor(u * (i + 1) / 2**b)`` for a ``b``-bit uniform ``u`` (b = 64 for SRHT rows, 32 for
sparse rows).

Pinned by: Philox bit equality (see ``philox``), exact distinctness, exact sign/row counts
and chi-square uniformity tests; the SRHT row set also pins through the orthogonality of
the full-size transform (``s = m_p``).
"""
from __future__ import annotations

import math

import numpy as np

from .philox import block

STREAM_SIGNS = 1
STREAM_ROWS = 2
STREAM_SPARSE_ROWS = 3
STREAM_SPARSE_SIGNS = 4
STREAM_GAUSS = 5


def next_pow2(m: int) -> int:
    return 1 << max(0, (int(m) - 1).bit_length())


def signs(seed: int, m: int) -> np.ndarray:
    """Diagonal of D as an int8 array of +-1 (length m)."""
    j = np.arange(m, dtype=np.uint64)
    words = block(seed, j >> np.uint64(7), 0, STREAM_SIGNS)
    words = np.stack(words)                                  # 4 x m
    w = words[(j >> np.uint64(5)) & np.uint64(3), np.arange(m)]
    bit = (w >> (j & np.uint64(31))) & np.uint64(1)
    return (1 - 2 * bit.astype(np.int64)).astype(np.int8)


def srht_rows(seed: int, pool: int, s: int) -> np.ndarray:
    """``s`` distinct rows of ``[0, pool)`` by Floyd sampling, sorted ascending (int64)."""
    if not (0 < s <= pool):
        raise ValueError("need 0 < s <= pool")
    t = np.arange(s, dtype=np.uint64)
    w0, w1, _, _ = block(seed, t, 0, STREAM_ROWS)
    chosen = set()
    out = []
    for tt in range(s):
        u = int(w0[tt]) | (int(w1[tt]) << 32)
        i = pool - s + tt
        x = (u * (i + 1)) >> 64
        if x in chosen:
            x = i
        chosen.add(x)
        out.append(x)
    return np.sort(np.asarray(out, dtype=np.int64))


def sparse(seed: int, m: int, s: int, zeta: int):
    """Sparse-sign supports and signs: ``rows[j, t]`` (int32) and ``sgn[j, t]`` (int8 +-1).

    Column ``j`` of S has ``zeta`` distinct nonzero rows ``rows[j, :]`` (in draw order) with
    values ``sgn[j, t] / sqrt(zeta)``.
    """
    if not (1 <= zeta <= s) or zeta > 32:
        raise ValueError("need 1 <= zeta <= min(s, 32)")
    j = np.arange(m, dtype=np.uint64)
    rows = np.empty((m, zeta), dtype=np.int64)
    cache = {}
    for t in range(zeta):
        sub = t >> 2
        if sub not in cache:
            cache[sub] = block(seed, j, sub, STREAM_SPARSE_ROWS)
        w = cache[sub][t & 3]
        i = s - zeta + t
        x = ((w * np.uint64(i + 1)) >> np.uint64(32)).astype(np.int64)
        if t:
            dup = (rows[:, :t] == x[:, None]).any(axis=1)
            x = np.where(dup, i, x)
        rows[:, t] = x
    sw = np.stack(block(seed, j >> np.uint64(2), 0, STREAM_SPARSE_SIGNS))
    w = sw[(j & np.uint64(3)).astype(np.int64), np.arange(m)]
    bits = (w[:, None] >> np.arange(zeta, dtype=np.uint64)[None, :]) & np.uint64(1)
    sgn = (1 - 2 * bits.astype(np.int64)).astype(np.int8)
    return rows.astype(np.int32), sgn


def gaussian_block(seed: int, s: int, j0: int, j1: int) -> np.ndarray:
    """Standard normal entries ``G[0:s, j0:j1]`` in FP64 (Box-Muller from 32-bit words).

    For a word pair ``(a, b)``: ``u = (a + 1) / 2**32`` in (0, 1], ``v = b / 2**32``,
    ``r = sqrt(-2 ln u)``, and the two entries are ``r cos(2 pi v)`` and ``r sin(2 pi v)``.
    """
    q = (s + 3) // 4
    cols = np.arange(j0, j1, dtype=np.uint64)
    out = np.empty((4 * q, j1 - j0))
    two32 = 2.0 ** 32
    for qq in range(q):
        w = block(seed, cols, qq, STREAM_GAUSS)
        for h in range(2):
            a = w[2 * h].astype(np.float64)
            b = w[2 * h + 1].astype(np.float64)
            u = (a + 1.0) / two32
            v = b / two32
            r = np.sqrt(-2.0 * np.log(u))
            out[4 * qq + 2 * h] = r * np.cos(2.0 * math.pi * v)
            out[4 * qq + 2 * h + 1] = r * np.sin(2.0 * math.pi * v)
    return out[:s]
