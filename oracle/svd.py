"""Plain one-sided (Hestenes) Jacobi SVD in FP64, applied to the sketch itself (no QR).

Line 3 of Algorithm 1 takes the SVD of ``SA``.  One-sided Jacobi orthogonalises the
columns of ``X = SA`` by plane rotations ``X <- X J`` accumulated in ``V``: for a column
pair ``(p, q)`` with ``alpha = |x_p|^2``, ``beta = |x_q|^2``, ``gamma = x_p . x_q``, the
rotation with ``zeta = (beta - alpha) / (2 gamma)``, ``t = sign(zeta) / (|zeta| +
sqrt(1 + zeta^2))``, ``c = 1 / sqrt(1 + t^2)``, ``s = c t`` makes the pair orthogonal.
Pairs are visited in round-robin (tournament) order, each round holding disjoint pairs; a
pair is skipped when ``|gamma| <= tol sqrt(alpha beta)`` with ``tol = N * u``.  At
convergence the singular values are the column norms, sorted non-increasing; ``V`` is
permuted to match and each column is sign-normalised so that its entry of largest
magnitude (lowest index on ties) is positive.

Pinned by: LAPACK singular values of the same matrix, reconstruction and orthogonality
residuals, and exact null vectors.
"""
from __future__ import annotations

import numpy as np

U64 = np.finfo(np.float64).eps / 2


def round_robin(n: int):
    """Rounds of disjoint pairs covering every pair of ``range(n)`` once (circle method)."""
    n_even = n + (n & 1)
    others = list(range(1, n_even))
    rounds = []
    for r in range(n_even - 1):
        arr = [0] + others[r:] + others[:r]
        ps, qs = [], []
        for i in range(n_even // 2):
            a, b = arr[i], arr[n_even - 1 - i]
            if a < n and b < n:
                ps.append(min(a, b))
                qs.append(max(a, b))
        rounds.append((np.asarray(ps, dtype=np.int64), np.asarray(qs, dtype=np.int64)))
    return rounds


def sign_normalise(v: np.ndarray) -> np.ndarray:
    """Flip each column so that its largest-magnitude entry (lowest index on ties) is positive."""
    v = np.array(v, dtype=np.float64, copy=True)
    idx = np.argmax(np.abs(v), axis=0)
    flip = v[idx, np.arange(v.shape[1])] < 0
    v[:, flip] *= -1.0
    return v


def jacobi_svd(x: np.ndarray, tol: float | None = None, max_sweeps: int = 60):
    """One-sided Jacobi SVD of ``x`` (rows >= cols).

    Returns ``(sigma, V, U, sweeps)`` with ``sigma`` non-increasing, ``x = U diag(sigma) V^T``
    (columns of ``U`` for zero singular values are zero), ``V`` sign-normalised.
    """
    x = np.array(x, dtype=np.float64, copy=True)
    rows, n = x.shape
    if tol is None:
        tol = n * U64
    v = np.eye(n)
    schedule = round_robin(n)
    sweeps = 0
    for sweep in range(max_sweeps):
        rotated = 0
        for ps, qs in schedule:
            if ps.size == 0:
                continue
            xp, xq = x[:, ps], x[:, qs]
            alpha = np.einsum("ij,ij->j", xp, xp)
            beta = np.einsum("ij,ij->j", xq, xq)
            gamma = np.einsum("ij,ij->j", xp, xq)
            act = np.abs(gamma) > tol * np.sqrt(alpha * beta)
            if not act.any():
                continue
            rotated += int(act.sum())
            ps, qs = ps[act], qs[act]
            alpha, beta, gamma = alpha[act], beta[act], gamma[act]
            zeta = (beta - alpha) / (2.0 * gamma)
            t = np.where(zeta >= 0, 1.0, -1.0) / (np.abs(zeta) + np.sqrt(1.0 + zeta * zeta))
            c = 1.0 / np.sqrt(1.0 + t * t)
            s = c * t
            xp, xq = x[:, ps], x[:, qs]
            x[:, ps] = c * xp - s * xq
            x[:, qs] = s * xp + c * xq
            vp, vq = v[:, ps], v[:, qs]
            v[:, ps] = c * vp - s * vq
            v[:, qs] = s * vp + c * vq
        sweeps = sweep + 1
        if rotated == 0:
            break
    else:
        raise RuntimeError("one-sided Jacobi did not converge")
    sigma = np.linalg.norm(x, axis=0)
    order = np.argsort(-sigma, kind="stable")
    sigma = sigma[order]
    v = v[:, order]
    u = x[:, order]
    nz = sigma > 0
    u[:, nz] /= sigma[nz]
    u[:, ~nz] = 0.0
    flip = np.sign(v[np.argmax(np.abs(v), axis=0), np.arange(n)])
    flip[flip == 0] = 1.0
    return sigma, v * flip, u * flip, sweeps
