"""Seeded synthetic inputs for the five workloads of the sketch-and-solve null-space method.

This module only builds input matrices. It holds none of the sketching or
solving arithmetic: both the HIP library and the FP64 oracle receive the arrays
made here, and neither is imported by it.

Workloads (sizes as the method is evaluated on them):

* ``plain``   -- ``A = U diag(sigma) V^T`` in FP64, 2000 x 50, Haar ``U`` and ``V``,
  ``sigma_i = 10^(-8 (i-1)/48)`` for ``i = 1..49`` and ``sigma_50 = 0`` (one planted
  null vector, the last column of ``V``).  Same-dimension setting of Section 3.1.
* ``tls``     -- total least squares ``M = [A | b]``: ``A`` i.i.d. N(0,1) (m x n),
  ``x_true`` ~ N(0,1), ``b = A x_true + noise * N(0,1)``; built in FP64 from the FP32
  entries of ``A`` and stored in FP32 (Section 4 with one right-hand side).
* ``loewner`` -- AAA-shaped Loewner matrix for ``f = tanh(50 z)`` on ``m`` points
  uniform in [-1, 1], with ``n`` support points chosen greedily on ``|f - r|``
  (Section 6.1).  FP64.
* ``planted`` -- ``A = G (I - V_p V_p^T) + 1e-6 U_p V_p^T`` with Haar ``V_p`` (n x 4) and
  ``U_p`` (m x 4): N(0,1) entries with four near-null directions, stored in FP32.
* ``batched`` -- 512 instances with m uniform in [5000, 200000] and n uniform in
  [16, 256], each built as ``planted`` from the seed pair (4, i).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "haar", "plain_matrix", "tls_matrix", "tls_target", "loewner_aaa",
    "planted_matrix", "batched_sizes", "planted_matrix_torch", "coherent_matrix",
    "table1_tls_matrix",
]


def _rng(*seed):
    return np.random.Generator(np.random.PCG64(list(seed)))


def haar(rows: int, cols: int, rng: np.random.Generator) -> np.ndarray:
    """Orthonormal rows x cols matrix with Haar distribution (QR of a Gaussian, diag(R) > 0)."""
    g = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def plain_matrix(m: int = 2000, n: int = 50, seed: int = 1):
    """``A = U diag(sigma) V^T`` (FP64) with log-spaced sigma from 1 to 1e-8 and sigma_n = 0.

    Returns ``(A, sigma, V)``; ``V[:, -1]`` spans the exact null space of ``A``.
    """
    rng = _rng(1, seed)
    u = haar(m, n, rng)
    v = haar(n, n, rng)
    sigma = np.zeros(n)
    sigma[: n - 1] = 10.0 ** (-8.0 * np.arange(n - 1) / (n - 2))
    a = (u * sigma) @ v.T
    return a, sigma, v


def coherent_matrix(m: int = 1000, n: int = 100, sigma=None, seed: int = 11):
    """Coherent test matrix of Figure 1: left singular vectors ``[I_n; 0]``, Haar right ones."""
    rng = _rng(11, seed)
    v = haar(n, n, rng)
    if sigma is None:
        sigma = np.ones(n)
        sigma[-2] = 0.1
        sigma[-1] = 1e-6
    a = np.zeros((m, n))
    a[:n, :] = (np.asarray(sigma)[:, None] * v.T)
    return a, np.asarray(sigma), v


def tls_matrix(m: int = 1_000_000, n: int = 200, seed: int = 2, noise: float = 1e-3,
               dtype=np.float32):
    """``M = [A | b]`` (m x (n+1)) for total least squares with one right-hand side.

    ``A`` has i.i.d. N(0,1) entries rounded to ``dtype``; ``b = A x_true + noise * e`` is
    formed in FP64 from the rounded ``A`` and then rounded.  Returns ``(M, x_true)``.
    """
    rng = _rng(2, seed)
    m_out = np.empty((m, n + 1), dtype=dtype)
    x_true = rng.standard_normal(n)
    chunk = 1 << 16
    for r0 in range(0, m, chunk):
        r1 = min(m, r0 + chunk)
        a = rng.standard_normal((r1 - r0, n)).astype(dtype)
        e = rng.standard_normal(r1 - r0)
        b = a.astype(np.float64) @ x_true + noise * e
        m_out[r0:r1, :n] = a
        m_out[r0:r1, n] = b.astype(dtype)
    return m_out, x_true


def tls_target(n: int, seed: int = 5) -> np.ndarray:
    """Target vector ``x_target`` ~ N(0,1) of the differentiable TLS loss."""
    return _rng(5, seed).standard_normal(n)


def table1_tls_matrix(m: int = 1 << 14, n: int = 1000, k: int = 10, seed: int = 7,
                      trailing: float = 2.2e-8):
    """TLS input shaped like Table 1: ``[A | B]`` with A (m x n), B (m x k).

    ``A`` has Haar singular vectors and singular values decaying geometrically from 1 to
    1e-3; ``B = A X`` scaled to the Frobenius norm of ``A``, plus Gaussian noise scaled so
    that its Frobenius norm equals ``trailing`` (the printed TLS error of Table 1 is about
    2.2e-8; the paper does not state the noise normalisation).
    """
    rng = _rng(7, seed)
    u = haar(m, n, rng)
    v = haar(n, n, rng)
    sigma = 10.0 ** (-3.0 * np.arange(n) / (n - 1))
    a = (u * sigma) @ v.T
    x = rng.standard_normal((n, k))
    b = a @ x
    b *= np.linalg.norm(a) / np.linalg.norm(b)
    e = rng.standard_normal((m, k))
    b += e * (trailing / np.linalg.norm(e))
    return np.hstack([a, b])


def _aaa_eval(zs, fs, w, z):
    c = 1.0 / (z[:, None] - zs[None, :])
    return (c @ (w * fs)) / (c @ w)


def loewner_aaa(m: int = 100_000, n: int = 100, seed: int = 3):
    """Loewner matrix after ``n`` greedy AAA steps for ``f = tanh(50 z)``, z ~ U[-1, 1].

    Greedy start ``r = mean(f)``; each step adds the sample point where ``|f - r|`` is
    largest and recomputes the barycentric weights as the trailing right singular vector
    of the current Loewner matrix (LAPACK SVD in FP64).  Rows are the ``m - n`` non-support
    points, columns the ``n`` support points: ``L_ij = (f_i - f_j) / (z_i - z_j)``.

    Returns ``(L, z, f, support)`` with ``support`` the support indices in selection order.
    """
    rng = _rng(3, seed)
    z = rng.uniform(-1.0, 1.0, m)
    f = np.tanh(50.0 * z)
    mask = np.ones(m, dtype=bool)
    support = []
    r = np.full(m, f.mean())
    for _ in range(n):
        err = np.abs(f - r)
        err[~mask] = -1.0
        j = int(np.argmax(err))
        support.append(j)
        mask[j] = False
        zs, fs = z[support], f[support]
        zi, fi = z[mask], f[mask]
        loew = (fi[:, None] - fs[None, :]) / (zi[:, None] - zs[None, :])
        # weights of the current approximant: trailing right singular vector
        _, _, vt = np.linalg.svd(loew, full_matrices=False)
        w = vt[-1]
        r = np.empty(m)
        r[mask] = _aaa_eval(zs, fs, w, zi)
        r[~mask] = f[~mask]
    zs, fs = z[support], f[support]
    zi, fi = z[mask], f[mask]
    loew = (fi[:, None] - fs[None, :]) / (zi[:, None] - zs[None, :])
    return loew, z, f, np.asarray(support)


def planted_matrix(m: int, n: int, k: int = 4, level: float = 1e-6, seed=(4, 0),
                   dtype=np.float32):
    """``G (I - V_p V_p^T) + level * U_p V_p^T`` built in FP64, rounded to ``dtype``.

    Returns ``(A, V_p)``: ``V_p`` spans the planted near-null directions.
    """
    rng = _rng(*((seed,) if np.isscalar(seed) else tuple(seed)))
    g = rng.standard_normal((m, n))
    vp = haar(n, k, rng)
    up = haar(m, k, rng)
    a = g - (g @ vp) @ vp.T + level * (up @ vp.T)
    return a.astype(dtype), vp


def batched_sizes(count: int = 512, seed: int = 4, m_range=(5000, 200_000), n_range=(16, 256)):
    """Instance shapes ``(m_i, n_i)`` drawn uniformly (inclusive ranges)."""
    rng = _rng(4, seed, 999)
    ms = rng.integers(m_range[0], m_range[1] + 1, size=count)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=count)
    return [(int(a), int(b)) for a, b in zip(ms, ns)]


def planted_matrix_torch(m: int, n: int, index: int, device, k: int = 4, level: float = 1e-6,
                         seed: int = 4):
    """Device-side variant of :func:`planted_matrix` for large batches (torch RNG, FP32 result).

    Deterministic for a given (seed, index, device type); used where host generation of
    tens of GB would dominate.  Returns ``(A_fp32, V_p_fp64)``.
    """
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) * 1_000_003 + int(index))
    g = torch.randn((m, n), generator=gen, device=device, dtype=torch.float64)
    vp, rv = torch.linalg.qr(torch.randn((n, k), generator=gen, device=device, dtype=torch.float64))
    vp = vp * torch.sign(torch.diagonal(rv))
    up, ru = torch.linalg.qr(torch.randn((m, k), generator=gen, device=device, dtype=torch.float64))
    up = up * torch.sign(torch.diagonal(ru))
    a = g - (g @ vp) @ vp.T + level * (up @ vp.T)
    del g
    return a.to(torch.float32), vp


def seeds_for(name: str) -> int:
    """Default seed of each workload (its index in the list above, 1-based)."""
    return {"plain": 1, "tls": 2, "loewner": 3, "batched": 4, "tls_grad": 5}[name]

