"""AAA rational approximation with a reused sketch (Section 6), in FP64, real sample points.
TEST INFRASTRUCTURE ONLY (see the package header).

AAA (Section 6.1): with support points z_{i_1..i_k}, the barycentric approximant is
``r(z) = sum_j w_j f_{i_j} / (z - z_{i_j}) / sum_j w_j / (z - z_{i_j})``; the next support point
is the sample point where ``|f - r|`` is largest (the first one on ties; ``r`` is the mean of
``f`` before any support point is chosen), and the weights are the trailing right singular
vector of the Loewner matrix ``L[i, j] = (f_i - f_{i_j}) / (z_i - z_{i_j})`` over the sample
points that are not support points.  The loop stops once the largest error is at most
``tol * max|f|`` or ``n_max`` support points are taken.

Sketch reuse (Section 6.2): the s x k sketch of the Loewner matrix is kept; choosing support
point j removes its row (``- S(:, j) L(j, :)``, Algorithm 3) and adds the column of the new
support point (the sketch of that column, zero at every support point).  The weights are then
the trailing right singular vector of the s x k sketch.  ``plain`` solves the same loop with
the SVD of the Loewner matrix itself.

Pinned by: with ``s = m = m_p`` the Hadamard sketch is orthogonal, so the sketched loop takes
the support points of the plain loop, whose weights come from LAPACK's SVD; the approximant
interpolates f at the support points; for tanh(50 z) on [-1, 1] the error falls below the
tolerance well before the degree cap.
"""
from __future__ import annotations

import numpy as np

from . import operators, updates
from .svd import jacobi_svd


def barycentric(z, f, sup, w):
    """``r`` at every sample point (``f`` itself at the support points)."""
    mask = np.zeros(len(z), dtype=bool)
    mask[sup] = True
    r = np.array(f, dtype=np.float64, copy=True)
    zi = z[~mask]
    C = 1.0 / (zi[:, None] - z[sup][None, :])
    r[~mask] = (C @ (w * f[sup])) / (C @ w)
    return r


def _trailing(mat):
    _, v, _, _ = jacobi_svd(mat)
    w = v[:, -1]
    return w if w[np.argmax(np.abs(w))] > 0 else -w


def aaa(z, f, n_max, tol, kind="srht", s=None, seed=0, zeta=8, plain=False):
    """``(support indices, weights, max error before each step)``."""
    z = np.asarray(z, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    m = len(z)
    fmax = float(np.max(np.abs(f)))
    mask = np.zeros(m, dtype=bool)
    sup, hist = [], []
    w = np.zeros(0)
    SA = None if plain else np.zeros((s, n_max))
    r = np.full(m, np.mean(f))
    for k in range(n_max + 1):
        err = np.abs(f - r)
        err[mask] = -1.0
        j = int(np.argmax(err))
        hist.append(float(err[j]))
        if err[j] <= tol * fmax or k == n_max:
            break
        if not plain and k > 0:
            row = (f[j] - f[sup]) / (z[j] - z[sup])
            SA[:, :k] = updates.update_rows(SA[:, :k], kind, seed, m, [j], row[None, :], [-1], zeta=zeta)
        mask[j] = True
        sup.append(j)
        if plain:
            L = (f[~mask][:, None] - f[sup][None, :]) / (z[~mask][:, None] - z[sup][None, :])
            _, _, vt = np.linalg.svd(L, full_matrices=False)
            w = vt[-1]
            w = w if w[np.argmax(np.abs(w))] > 0 else -w
        else:
            col = np.zeros(m)
            col[~mask] = (f[~mask] - f[j]) / (z[~mask] - z[j])
            SA[:, k] = operators.sketch(col[:, None], kind, s, seed, zeta=zeta)[:, 0]
            w = _trailing(SA[:, :k + 1])
        r = barycentric(z, f, sup, w)
    return sup, w, hist
