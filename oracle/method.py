"""Algorithm 1 (sketch-and-solve for the null space problem), TLS and its gradient, in FP64.

* ``trailing_rsv``  -- Algorithm 1: draw S, form ``SA``, take its SVD, return the trailing
                       ``k`` right singular vectors ``W = V(:, n-k+1:n)`` and singular values.
* ``tls_solve``     -- Section 4 with one right-hand side: the trailing right singular vector
                       ``v`` of the sketched ``[A | b]`` gives ``x = -v(1:n) / v(n+1)``.
* ``tls_grad``      -- gradient of ``L = |x - x_target|^2`` with respect to ``[A | b]`` through
                       the sketch (the paper has no gradient; derivation below).
* ``tls_solve_multi`` -- Section 4 with k right-hand sides: ``X = -V12 V22^{-1}`` from the
                       trailing k right singular vectors of the sketched ``[A | B]``.
* ``null_space_eps`` -- the epsilon-tolerance version of Algorithm 1 (Section 2): every right
                       singular vector of ``SA`` whose singular value is below ``eps`` (times the
                       largest one when ``relative``); with ``eps = O(u)`` the numerical null space.

Gradient.  With ``M~ = S M`` (s x N), ``M~ = U~ Sigma V^T`` and ``v`` its last right singular
vector: ``g = 2 (x - x_target)``; ``dL/dv = -(1/v_N) [g; g^T x]``; first-order eigenvector
perturbation of ``M~^T M~`` gives ``w = sum_{j != N} v_j (v_j^T dL/dv) / (sigma_N^2 -
sigma_j^2)`` and ``dL/dM~ = (M~ v) w^T + (M~ w) v^T``; finally ``dL/dM = S^T dL/dM~``, applied
here with the explicit S.

Pinned by: planted exact null vectors and the full-size orthogonal sketch (``trailing_rsv``);
classical TLS by full SVD on tiny inputs (``tls_solve``); central finite differences of the
oracle's own loss (``tls_grad``).
"""
from __future__ import annotations

import numpy as np

from . import operators
from .svd import jacobi_svd


def trailing_rsv(a: np.ndarray, k: int, kind: str, s: int, seed: int, zeta: int = 8,
                 gauss_dtype: str = "bf16", return_all: bool = False):
    m, n = a.shape
    if not (n < s <= m) or not (1 <= k <= n):
        raise ValueError("need n < s <= m and 1 <= k <= n")
    sa = operators.sketch(a, kind, s, seed, zeta=zeta, gauss_dtype=gauss_dtype)
    sigma, v, _, sweeps = jacobi_svd(sa)
    out = (v[:, n - k:], sigma[n - k:])
    if return_all:
        return out + (sa, sigma, v, sweeps)
    return out


def null_space_eps(a: np.ndarray, eps: float, kind: str, s: int, seed: int, relative: bool = True,
                   zeta: int = 8):
    """``(W, sigma, count)``: all N right singular vectors of ``SA`` in non-increasing order of
    their singular values ``sigma``; the last ``count`` columns, those with ``sigma < eps``
    (``eps * sigma[0]`` when ``relative``), span the computed null space."""
    n = a.shape[1]
    _, _, _, sigma, v, _ = trailing_rsv(a, n, kind, s, seed, zeta=zeta, return_all=True)
    thr = eps * sigma[0] if relative else eps
    count = int(np.sum(sigma < thr))
    return v, sigma, count


def tls_solve_multi(mat: np.ndarray, nrhs: int, kind: str, s: int, seed: int, zeta: int = 8):
    """``(X, Vk, sigma_k)`` for ``mat = [A | B]`` with ``B`` the last ``nrhs`` columns."""
    N = mat.shape[1]
    vk, sk = trailing_rsv(mat, nrhs, kind, s, seed, zeta=zeta)
    n = N - nrhs
    X = -np.linalg.solve(vk[n:].T, vk[:n].T).T
    return X, vk, sk


def tls_from_v(v: np.ndarray) -> np.ndarray:
    """``x = -V_{k,1} V_{k,2}^{-1}`` for ``k = 1``: ``-v(1:n) / v(n+1)``."""
    return -v[:-1] / v[-1]


def tls_solve(mat: np.ndarray, kind: str, s: int, seed: int, zeta: int = 8):
    """Sketched TLS solution for ``mat = [A | b]``; returns ``(x, v, sigma, V, SA)``."""
    vk, _, sa, sigma, v, _ = trailing_rsv(mat, 1, kind, s, seed, zeta=zeta, return_all=True)
    return tls_from_v(vk[:, 0]), vk[:, 0], sigma, v, sa


def tls_loss(mat: np.ndarray, x_target: np.ndarray, kind: str, s: int, seed: int,
             zeta: int = 8) -> float:
    x = tls_solve(mat, kind, s, seed, zeta)[0]
    d = x - x_target
    return float(d @ d)


def tls_grad(mat: np.ndarray, x_target: np.ndarray, kind: str, s: int, seed: int,
             zeta: int = 8):
    """``(dL/dM, x, loss)`` with the explicit S of the same realisation."""
    m, nn = mat.shape
    x, vN, sigma, V, sa = tls_solve(mat, kind, s, seed, zeta)
    g = 2.0 * (x - x_target)
    gbar = -np.concatenate([g, [g @ x]]) / vN[-1]
    lam = sigma ** 2
    coef = (V.T @ gbar)[:-1] / (lam[-1] - lam[:-1])
    w = V[:, :-1] @ coef
    y_v = sa @ vN
    y_w = sa @ w
    if kind == "sparse":
        S = operators.sparse_matrix(seed, m, s, zeta)
        p = S.T @ y_v
        q = S.T @ y_w
    else:
        S = operators.explicit(kind, seed, m, s, zeta)
        p = S.T @ y_v
        q = S.T @ y_w
    grad = np.outer(p, w) + np.outer(q, vN)
    d = x - x_target
    return grad, x, float(d @ d)
