"""Explicit sketching matrices S (s x m) and the plain product SA = S A, all in FP64.

Sketch kinds (Section 2):

* ``srht``   -- subsampled randomized trigonometric transform with the Walsh-Hadamard
  transform as the trig transform: ``S = sqrt(m_p / s) R (H / sqrt(m_p)) D`` restricted to
  the first ``m`` columns, ``m_p = 2**ceil(log2 m)`` (``A`` is zero-padded to ``m_p`` rows).
  Entry ``(i, j)`` is ``d_j (-1)**popcount(r_i & j) / sqrt(s)``: the SRFT definition
  ``Omega^* = sqrt(m/s) R F^* D`` of Section 2 with F the normalised Hadamard matrix.
* ``sparse`` -- sparse sign: each column of S has ``zeta`` distinct nonzero rows with
  values ``+-1/sqrt(zeta)`` (the CountSketch family mentioned in Section 2).
* ``gauss``  -- ``S = G_hat / sqrt(s)`` with ``G_hat`` the i.i.d. N(0,1) matrix G of Section 2
  rounded to the operand format (bf16 or e4m3); rounding happens before use, so
  ``G_hat`` itself is the sketch (FP64 holds bf16/e4m3 values exactly).
* ``srdct``  -- the SRFT of Section 2 with the orthonormal DCT-II as trig transform, the
  choice Section 4 makes for real data: ``S = sqrt(m_p / s) R C D`` on ``A`` zero-padded to
  ``m_p = max(1024, 2**ceil(log2 m))`` rows, with the same ``D`` and the same row sampler as
  the Hadamard kind (rows drawn from ``[0, m_p)``).  ``C[k, j] = c_k cos(pi k (2j+1) / (2 m_p))``
  with ``c_0 = sqrt(1/m_p)`` and ``c_k = sqrt(2/m_p)`` otherwise, so entry ``(i, j)`` of S is
  ``d_j w_i cos(pi r_i (2j+1) / (2 m_p))`` with ``w_i = sqrt(1/s)`` for ``r_i = 0`` and
  ``sqrt(2/s)`` otherwise.  The cosine's argument is reduced exactly, in integers, modulo one
  period before the cosine is taken.

* ``hrht``   -- hashed randomized Hadamard transform (the H-RHT of Section 2): the SRFT's row
  sample R replaced by a 1-hashing matrix Phi (s x m_p, one entry +-1 per column at a uniformly
  drawn row), ``S = Phi (H / sqrt(m_p)) D`` on ``A`` zero-padded to ``m_p = 2**ceil(log2 m)``
  rows, with the Hadamard kind's D.  Phi is the sparse-sign kind's draw with zeta = 1 over the
  m_p columns (Floyd with one draw is a uniform row; the sign bit as for sparse sign).

Pinned by: the special case ``s = m = m_p`` where the SRHT and the DCT kind are orthogonal
(SVD of ``SA`` equals SVD of ``A``), unit column norms, ``S S^T`` structure, the DCT kind
against SciPy's orthonormal DCT-II of the signed, padded ``A`` (a library transform), and
the Gaussian embedding envelope of Theorem 2.1.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import draws
from .precision import round_to


def srht_columns(seed: int, m: int, s: int, j0: int, j1: int, rows=None, d=None) -> np.ndarray:
    """Columns ``j0:j1`` of the SRHT sketching matrix (s x (j1 - j0))."""
    m_p = draws.next_pow2(m)
    if rows is None:
        rows = draws.srht_rows(seed, m_p, s)
    if d is None:
        d = draws.signs(seed, m)
    j = np.arange(j0, j1, dtype=np.int64)
    parity = np.bitwise_count(rows[:, None] & j[None, :]) & 1
    had = 1.0 - 2.0 * parity
    return had * d[j0:j1].astype(np.float64)[None, :] / math.sqrt(s)


def dct_pool(m: int) -> int:
    """Padded length ``m_p`` of the DCT kind: the next power of two, and at least 1024."""
    return max(1024, draws.next_pow2(m))


def srdct_columns(seed: int, m: int, s: int, j0: int, j1: int, rows=None, d=None) -> np.ndarray:
    """Columns ``j0:j1`` of the subsampled randomized DCT-II sketching matrix."""
    m_p = dct_pool(m)
    if rows is None:
        rows = draws.srht_rows(seed, m_p, s)
    if d is None:
        d = draws.signs(seed, m)
    j = np.arange(j0, j1, dtype=np.int64)
    num = (rows[:, None] * (2 * j[None, :] + 1)) % (4 * m_p)   # angle = pi num / (2 m_p)
    cosv = np.cos(np.pi * num.astype(np.float64) / (2.0 * m_p))
    w = np.where(rows == 0, math.sqrt(1.0 / s), math.sqrt(2.0 / s))
    return cosv * w[:, None] * d[j0:j1].astype(np.float64)[None, :]


def fwht(x: np.ndarray) -> np.ndarray:
    """Unnormalised Walsh-Hadamard transform along axis 0 (length a power of two): the plain
    radix-2 butterflies, entry (i, j) of the matrix being (-1)^popcount(i & j)."""
    y = np.array(x, dtype=np.float64, copy=True)
    n = y.shape[0]
    h = 1
    while h < n:
        y = y.reshape(n // (2 * h), 2, h, *y.shape[1:])
        a, b = y[:, 0].copy(), y[:, 1].copy()
        y[:, 0], y[:, 1] = a + b, a - b
        y = y.reshape(n, *y.shape[3:])
        h *= 2
    return y


def hrht_matrix(seed: int, m: int, s: int) -> np.ndarray:
    """The whole H-RHT sketching matrix (s x m, small cases only)."""
    m_p = draws.next_pow2(m)
    phi = sparse_matrix(seed, m_p, s, 1).toarray()
    j = np.arange(m)
    had = 1.0 - 2.0 * (np.bitwise_count(np.arange(m_p)[:, None] & j[None, :]) & 1)
    return phi @ had * draws.signs(seed, m).astype(np.float64)[None, :] / math.sqrt(m_p)


def sparse_matrix(seed: int, m: int, s: int, zeta: int) -> sp.csc_matrix:
    """Sparse-sign sketching matrix as a SciPy CSC matrix (s x m)."""
    rows, sgn = draws.sparse(seed, m, s, zeta)
    cols = np.repeat(np.arange(m), zeta)
    vals = sgn.reshape(-1).astype(np.float64) / math.sqrt(zeta)
    return sp.csc_matrix((vals, (rows.reshape(-1), cols)), shape=(s, m))


def gaussian_columns(seed: int, s: int, j0: int, j1: int, dtype: str) -> np.ndarray:
    """Columns ``j0:j1`` of ``G_hat / sqrt(s)`` with ``G_hat`` rounded to ``dtype``."""
    g = draws.gaussian_block(seed, s, j0, j1)
    return round_to(g, dtype) / math.sqrt(s)


def explicit(kind: str, seed: int, m: int, s: int, zeta: int = 8, gauss_dtype: str = "bf16"):
    """The whole S as a dense FP64 array (small cases only)."""
    if kind == "srht":
        return srht_columns(seed, m, s, 0, m)
    if kind == "srdct":
        return srdct_columns(seed, m, s, 0, m)
    if kind == "hrht":
        return hrht_matrix(seed, m, s)
    if kind == "sparse":
        return sparse_matrix(seed, m, s, zeta).toarray()
    if kind == "gauss":
        return gaussian_columns(seed, s, 0, m, gauss_dtype)
    raise ValueError(kind)


def sketch(a: np.ndarray, kind: str, s: int, seed: int, zeta: int = 8,
           gauss_dtype: str = "bf16", block: int = 8192) -> np.ndarray:
    """``SA`` in FP64 for an m x N matrix ``a`` (any real dtype; cast exactly to FP64)."""
    m, n = a.shape
    if kind == "hrht":
        m_p = draws.next_pow2(m)
        x = np.zeros((m_p, n))
        x[:m] = draws.signs(seed, m).astype(np.float64)[:, None] * np.asarray(a, dtype=np.float64)
        return sparse_matrix(seed, m_p, s, 1) @ (fwht(x) / math.sqrt(m_p))
    if kind == "sparse":
        S = sparse_matrix(seed, m, s, zeta)
        out = np.zeros((s, n))
        for j0 in range(0, m, 1 << 18):
            j1 = min(m, j0 + (1 << 18))
            out += S[:, j0:j1] @ np.asarray(a[j0:j1], dtype=np.float64)
        return out
    out = np.zeros((s, n))
    if kind == "srht":
        rows = draws.srht_rows(seed, draws.next_pow2(m), s)
        d = draws.signs(seed, m)
    if kind == "srdct":
        rows = draws.srht_rows(seed, dct_pool(m), s)
        d = draws.signs(seed, m)
    for j0 in range(0, m, block):
        j1 = min(m, j0 + block)
        if kind == "srht":
            cols = srht_columns(seed, m, s, j0, j1, rows=rows, d=d)
        elif kind == "srdct":
            cols = srdct_columns(seed, m, s, j0, j1, rows=rows, d=d)
        elif kind == "gauss":
            cols = gaussian_columns(seed, s, j0, j1, gauss_dtype)
        else:
            raise ValueError(kind)
        out += cols @ np.asarray(a[j0:j1], dtype=np.float64)
    return out
