"""Parity at the benchmarked size, in the launch configuration bench.py times.

The TLS workload [A | b] is 1,000,000 x 201 FP32 (two column blocks), sketched to s = 804.
The whole sparse-sign SA is compared with the oracle's sparse product, the solve with the
oracle's solve; for the SRHT and DCT-II kinds, sampled rows of SA are computed one by one by
the oracle (a row of the explicit S against all of A).  Tolerances as in the smaller parity
tests.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import draws, method, operators

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
DEV = "cuda:0"
M_ROWS, N_COLS, SEED_DATA, SEED_SKETCH = 1_000_000, 200, 2, 7
S = 4 * (N_COLS + 1)


@pytest.fixture(scope="module")
def workload():
    M, _ = W.tls_matrix(m=M_ROWS, n=N_COLS, seed=SEED_DATA)
    Mt = torch.from_numpy(M).to(DEV)
    return M, Mt


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def colrel(a, b):
    """Largest relative 2-norm error over the columns."""
    num = np.linalg.norm(a - b, axis=0)
    den = np.maximum(np.linalg.norm(b, axis=0), 1e-300)
    return float(np.max(num / den))


def oracle_rows(kind, M, s, seed, idx):
    """Rows idx of SA = S M from the explicit S, one sampled row of S at a time."""
    m = M.shape[0]
    pool = operators.dct_pool(m) if kind == "srdct" else draws.next_pow2(m)
    cols = operators.srdct_columns if kind == "srdct" else operators.srht_columns
    rows = draws.srht_rows(seed, pool, s)[idx]
    d = draws.signs(seed, m)
    out = np.zeros((len(idx), M.shape[1]))
    for j0 in range(0, m, 1 << 16):
        j1 = min(m, j0 + (1 << 16))
        out += cols(seed, m, s, j0, j1, rows=rows, d=d) @ M[j0:j1].astype(np.float64)
    return out


def test_sparse_sketch_and_solve_full_size(lib, workload):
    M, Mt = workload
    A, b = Mt[:, :N_COLS], Mt[:, N_COLS:]
    SA = lib.sketch([A, b], "sparse", S, SEED_SKETCH).cpu().numpy()
    ref = operators.sketch(M, "sparse", S, SEED_SKETCH)
    assert colrel(SA, ref) < 1e-12, colrel(SA, ref)
    x, _, info = lib.tls_solve(A, b, kind="sparse", s=S, seed=SEED_SKETCH, residual=True)
    torch.cuda.synchronize()
    x_ref, v_ref, sig, _, _ = method.tls_solve(M.astype(np.float64), "sparse", S, SEED_SKETCH)
    kappa = sig[0] / (sig[-2] - sig[-1])
    tol = max(1e-10, math.sqrt(N_COLS + 1) * U * kappa)      # on the trailing vector v
    # x = -v(1:n) / v(N): a perturbation eps of v moves x by at most eps (1 + |x|) / |v(N)|
    nx = np.linalg.norm(x_ref)
    assert rel(x.cpu().numpy(), x_ref) < tol * (1 + nx) * math.sqrt(1 + nx * nx) / nx
    res_ref = float(np.linalg.norm(M.astype(np.float64) @ v_ref))
    assert abs(lib.read_info(info).residual - res_ref) <= 1e-10 * res_ref


def test_hrht_sketch_columns_full_size(lib, workload):
    """Columns of SA are sketched independently: three whole columns of the 1e6 x 201 H-RHT
    sketch against the oracle's transform-and-hash of those columns."""
    M, Mt = workload
    SA = lib.sketch([Mt[:, :N_COLS], Mt[:, N_COLS:]], "hrht", S, SEED_SKETCH).cpu().numpy()
    cols = [0, 117, N_COLS]
    ref = operators.sketch(M[:, cols].astype(np.float64), "hrht", S, SEED_SKETCH)
    assert colrel(SA[:, cols], ref) < 1e-12, colrel(SA[:, cols], ref)


@pytest.mark.parametrize("kind", ["srht", "srdct"])
def test_trig_sketch_sampled_rows_full_size(lib, workload, kind):
    M, Mt = workload
    SA = lib.sketch([Mt[:, :N_COLS], Mt[:, N_COLS:]], kind, S, SEED_SKETCH).cpu().numpy()
    idx = np.array([0, 1, 401, 402, S - 1])
    ref = oracle_rows(kind, M, S, SEED_SKETCH, idx)
    assert colrel(SA[idx].T, ref.T) < 1e-12, colrel(SA[idx].T, ref.T)
    # every row: the sketch preserves the Frobenius norm to the embedding's accuracy
    ratio = np.linalg.norm(SA) / np.linalg.norm(M.astype(np.float64))
    assert abs(ratio - 1) < 0.1, ratio
