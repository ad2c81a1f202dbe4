"""Row and column updates of a sketch (Section 5), in FP64.  TEST INFRASTRUCTURE ONLY (see the
package header).

A column added to ``A`` adds its sketch ``S a`` as a column of ``SA``; a removed column is
dropped from ``SA`` (Section 5, opening remarks).  Rows change ``SA`` by rank-one terms with
one column of the updated sketching matrix ``S_r``:

* row downdate (Algorithm 3): removing row ``j`` gives ``SA - S(:, j) A(j, :)``;
* row update (Algorithm 2): appending a row ``a`` gives ``SA + g a / sqrt(s)`` with ``g`` a
  standard Gaussian column independent of ``S``.  For the Gaussian kind ``g / sqrt(s)`` is the
  next column of ``G_hat / sqrt(s)`` (the same as sketching the longer matrix from scratch);
  for the other kinds an appended Gaussian column is what Section 5.3 prescribes.

Column ``j`` of ``S_r`` is therefore the kind's column of ``S`` for an original row ``j < m``
and, for a row appended at index ``j >= m``, the Gaussian column ``G[:, j] / sqrt(s)`` drawn
with the Gaussian kind's counters (Box-Muller in FP64; rounded to the operand format for the
Gaussian kind itself).

Pinned by: a downdate equals the from-scratch sketch of ``A`` with that row removed (the
product of the pinned explicit ``S`` with the smaller matrix); a Gaussian-kind update equals
the from-scratch sketch of the longer matrix; a non-Gaussian update equals the explicit
``[S | g / sqrt(s)]`` times the longer matrix; a downdate undoes the matching update.
"""
from __future__ import annotations

import math

import numpy as np

from . import draws, operators


def sketch_column(kind: str, seed: int, m: int, s: int, j: int, zeta: int = 8,
                  gauss_dtype: str = "bf16") -> np.ndarray:
    """Column ``j`` of the updated sketching matrix ``S_r`` (length ``s``)."""
    if kind == "gauss":
        return operators.gaussian_columns(seed, s, j, j + 1, gauss_dtype)[:, 0]
    if j >= m:
        return draws.gaussian_block(seed, s, j, j + 1)[:, 0] / math.sqrt(s)
    if kind == "srht":
        return operators.srht_columns(seed, m, s, j, j + 1)[:, 0]
    if kind == "srdct":
        return operators.srdct_columns(seed, m, s, j, j + 1)[:, 0]
    if kind == "sparse":
        rows, sgn = draws.sparse(seed, j + 1, s, zeta)
        col = np.zeros(s)
        col[rows[j].astype(np.int64)] = sgn[j].astype(np.float64) / math.sqrt(zeta)
        return col
    raise ValueError(kind)


def update_rows(sa: np.ndarray, kind: str, seed: int, m: int, rows, values: np.ndarray, ops,
                zeta: int = 8, gauss_dtype: str = "bf16") -> np.ndarray:
    """``SA + sum_t ops[t] S_r(:, rows[t]) values[t, :]``: ``ops`` +1 adds row ``rows[t]`` with
    values ``values[t]`` (update), -1 removes it (downdate)."""
    s = sa.shape[0]
    out = np.array(sa, dtype=np.float64, copy=True)
    vals = np.asarray(values, dtype=np.float64)
    for t, (j, op) in enumerate(zip(rows, ops)):
        col = sketch_column(kind, seed, m, s, int(j), zeta, gauss_dtype)
        out += float(op) * np.outer(col, vals[t])
    return out
