"""Quality measures and bounds of Sections 2-4, in FP64.

* ``sin_theta``        -- largest canonical-angle sine between two orthonormal bases
                          (Definition 3.1 and its remark: the sines are the singular values
                          of ``U_perp^* V``), computed as ``|W2 - W1 (W1^T W2)|_2``.
* ``residual_ratio``   -- ``|A W~|_F / |A W|_F`` with ``W`` the exact trailing right singular
                          vectors (Problem 2.1; the TLS column of Table 1).  The denominator
                          is floored at ``sqrt(k) u |A|_F`` when the optimum is at rounding level.
* ``chi``              -- relative gap ``|a - b| / sqrt(|ab|)`` (Section 3.1).
* ``ostrowski_ratio``  -- ``sigma_max(S U_A) / sigma_min(S U_A)``: the deterministic bound on
                          the residual ratio for the realised S (proof of Theorem 2.3).
* ``thm32_bound``      -- ``|R - R^{-*}|_2 / chi(alpha^2, (alpha + delta)^2)`` of Theorem 3.2
                          with ``S U = QR`` for the realised S.
* ``thm34_bounds``     -- Theorem 3.4 for subspaces of different dimensions (l < k): the
                          bounds on ``sin Theta([V_2, V_3], V~_3)`` and on
                          ``sin Theta(V_3, [V~_2, V~_3])``, each infinite where its gap
                          condition fails.
* ``expected_rho``     -- first-order mean residual ratio for a Gaussian sketch,
                          ``sqrt(1 + (N - k) / (s - N + k - 1))`` (inverse-Wishart mean;
                          derived from the sketch's distribution, not printed in the paper).

Pinned by: closed forms (orthogonal rotations of known angle), Table 1's printed residual
ratios, and the inequalities themselves on realised sketches.
"""
from __future__ import annotations

import math

import numpy as np

U64 = np.finfo(np.float64).eps / 2


def sin_theta(w1: np.ndarray, w2: np.ndarray) -> float:
    w1 = np.asarray(w1, dtype=np.float64).reshape(w1.shape[0], -1)
    w2 = np.asarray(w2, dtype=np.float64).reshape(w2.shape[0], -1)
    return float(np.linalg.norm(w2 - w1 @ (w1.T @ w2), 2))


def trailing_exact(a: np.ndarray, k: int):
    """Exact trailing k right singular vectors and singular values of ``a`` (LAPACK, FP64)."""
    _, sig, vt = np.linalg.svd(np.asarray(a, dtype=np.float64), full_matrices=False)
    return vt[-k:].T, sig[-k:], sig


def residual(a: np.ndarray, w: np.ndarray) -> float:
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) @ w))


def residual_ratio(a: np.ndarray, w_tilde: np.ndarray, w_opt: np.ndarray | None = None,
                   unit_roundoff: float = U64) -> float:
    a = np.asarray(a, dtype=np.float64)
    k = w_tilde.shape[1] if w_tilde.ndim == 2 else 1
    w_tilde = w_tilde.reshape(a.shape[1], k)
    if w_opt is None:
        w_opt, _, _ = trailing_exact(a, k)
    num = np.linalg.norm(a @ w_tilde)
    den = max(np.linalg.norm(a @ w_opt), math.sqrt(k) * unit_roundoff * np.linalg.norm(a))
    return float(num / den)


def chi(a: float, b: float) -> float:
    if a == b:
        return 0.0
    if a * b == 0:
        return math.inf
    return abs(a - b) / math.sqrt(abs(a * b))


def _left_basis(a: np.ndarray) -> np.ndarray:
    u, _, _ = np.linalg.svd(np.asarray(a, dtype=np.float64), full_matrices=False)
    return u


def ostrowski_ratio(S: np.ndarray, a: np.ndarray) -> float:
    sv = np.linalg.svd(S @ _left_basis(a), compute_uv=False)
    return float(sv[0] / sv[-1])


def embedding_range(S: np.ndarray, a: np.ndarray):
    """``(sigma_min, sigma_max)`` of ``S U_A``: the distortion of norms on range(A)."""
    sv = np.linalg.svd(S @ _left_basis(a), compute_uv=False)
    return float(sv[-1]), float(sv[0])


def thm32_bound(S: np.ndarray, a: np.ndarray, sa_sigma: np.ndarray, k: int) -> float:
    """Right-hand side of Theorem 3.2 in the 2-norm for the realised S.

    ``U`` are the left singular vectors of ``a``; ``S U = QR``; alpha and delta from either
    of the theorem's two conditions, whichever holds and gives the smaller bound.
    """
    u, sig, _ = np.linalg.svd(np.asarray(a, dtype=np.float64), full_matrices=False)
    n = sig.size
    _, r = np.linalg.qr(S @ u)
    m = r - np.linalg.inv(r).T
    num = np.linalg.norm(m, 2)
    best = math.inf
    # condition 1: min sigma_{1..n-k} >= alpha + delta, max sigma~_{n-k+1..n} <= alpha
    lo1, hi1 = sa_sigma[n - k], sig[n - k - 1]
    # condition 2: min sigma~_{1..n-k} >= alpha + delta, max sigma_{n-k+1..n} <= alpha
    lo2, hi2 = sig[n - k], sa_sigma[n - k - 1]
    for alpha, top in ((lo1, hi1), (lo2, hi2)):
        if top > alpha:
            c = chi(alpha ** 2, top ** 2)
            best = min(best, num / c if c > 0 else math.inf)
    return best


def thm34_bounds(S: np.ndarray, a: np.ndarray, sa_sigma: np.ndarray, k: int, l: int):
    """Right-hand sides of Theorem 3.4 in the 2-norm for the realised S, ``l < k < n``.

    First bound (on ``sin Theta([V_2, V_3], V~_3)``): alpha + delta = sigma_{n-k} (the smallest
    of the leading n - k singular values of A), alpha = sigma~_{n-l+1} (the largest of the
    trailing l of SA).  Second bound (on ``sin Theta(V_3, [V~_2, V~_3])``): alpha + delta =
    sigma~_{n-k}, alpha = sigma_{n-l+1}.  Both share ``|R - R^{-*}|_2`` with ``S U = QR``.
    """
    u, sig, _ = np.linalg.svd(np.asarray(a, dtype=np.float64), full_matrices=False)
    n = sig.size
    _, r = np.linalg.qr(S @ u)
    num = np.linalg.norm(r - np.linalg.inv(r).T, 2)
    out = []
    for top, alpha in ((sig[n - k - 1], sa_sigma[n - l]), (sa_sigma[n - k - 1], sig[n - l])):
        c = chi(alpha ** 2, top ** 2) if top > alpha else 0.0
        out.append(num / c if c > 0 else math.inf)
    return out[0], out[1]


def expected_rho(N: int, k: int, s: int) -> float:
    return math.sqrt(1.0 + (N - k) / (s - N + k - 1))
