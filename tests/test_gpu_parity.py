"""Parity of the HIP path with the FP64 oracle, element by element, on seeded inputs.

Tolerances: sketches with FP64 accumulation agree with the oracle's FP64 product to
rounding (1e-12 relative); plain-FP32 and narrow-operand sketches to the FP32 bound (1e-4
relative: FP32 accumulation over the sketch's terms).  Sketches are compared column by
column (the largest relative error over the columns of SA).  Trailing vectors agree to
max(1e-10, sqrt(N) u kappa_gap) with kappa_gap = sigma_1 / (sigma_{N-k} - sigma_{N-k+1})
of the oracle's SA (the conditioning floor of a singular subspace under perturbations of
size u sigma_1), and residual ratios to 1e-10 (FP64 arithmetic) or 1e-4 (FP32 arithmetic).
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from conftest import BATCHED_FAULT
from oracle import draws, method, metrics, operators, updates
from oracle.precision import round_bf16, round_e4m3

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
DEV = "cuda:0"


def t(x, dtype=None):
    return torch.tensor(np.ascontiguousarray(x), device=DEV, dtype=dtype)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def colrel(a, b):
    """Largest relative 2-norm error over the columns (sketch comparisons: a few wrong entries
    of a small-norm column cannot hide behind the other columns)."""
    num = np.linalg.norm(a - b, axis=0)
    den = np.maximum(np.linalg.norm(b, axis=0), 1e-300)
    return float(np.max(num / den))


def assert_vectors(ref, got, tol):
    """got spans ref's subspace to tol (sin theta), with orthonormal columns: sin theta alone
    would accept a zero matrix."""
    gram = got.T @ got
    assert np.abs(gram - np.eye(gram.shape[0])).max() < 1e-9, gram
    err = metrics.sin_theta(ref, got)
    assert err <= tol, (err, tol)


def vec_tol(sigma, k, u=U):
    N = sigma.size
    kappa = sigma[0] / max(sigma[N - k - 1] - sigma[N - k], 1e-300)
    return max(1e-10, math.sqrt(N) * u * kappa)


# ---------------------------------------------------------------------------- draws
def test_device_signs_and_sparse_bit_exact(lib):
    d = lib.draw_signs_device(3, 100_003).cpu().numpy()
    assert np.array_equal(d, draws.signs(3, 100_003))
    for s, zeta in ((804, 8), (40, 3), (64, 32)):
        rows, sg = lib.draw_sparse_device(4, 20_001, s, zeta)
        r2, s2 = draws.sparse(4, 20_001, s, zeta)
        assert np.array_equal(rows.cpu().numpy(), r2) and np.array_equal(sg.cpu().numpy(), s2)


@pytest.mark.parametrize("m,s", [(2000, 200), (64, 64), (64, 1), (100, 100), (2048, 2048), (1 << 20, 804),
                                 (1 << 31, 2048), (3000, 2048), (5000, 1100), (700, 513)])
def test_device_row_sample_bit_exact(lib, m, s):
    """The device's parallel resolution of Floyd's rule returns the sequential rule's rows,
    including sample sizes equal to the pool (every draw collides or is forced) and near it."""
    for seed in (1, 7, 2 ** 40 + 3):
        got = lib.draw_srht_rows_device(seed, m, s).cpu().numpy().astype(np.int64)
        assert np.array_equal(got, lib.draw_srht_rows(seed, m, s))
        assert np.array_equal(got, draws.srht_rows(seed, draws.next_pow2(m), s))


@pytest.mark.parametrize("seed,s,j0,j1", [(5, 203, 17, 2017), (6, 200, 0, 100_000), (2 ** 33 + 1, 64, 10 ** 9, 10 ** 9 + 50_000)])
def test_device_gaussian_matches_oracle_box_muller(lib, seed, s, j0, j1):
    """FP32 Box-Muller values within their error bound; the rounded entries G_hat equal the
    oracle's rounding of its FP64 Box-Muller values exactly (the device settles every rounding
    decision its FP32 error bound leaves open in FP64)."""
    g = lib.draw_gaussian_device(seed, s, j0, j1, "f32").cpu().numpy().astype(np.float64)
    ref = draws.gaussian_block(seed, s, j0, j1)
    # the FP32 values lie within half the margin E = 2^-21 (|g| + r) the rounding check assumes
    # (r: the pair's radius; rows 2p and 2p + 1 form a pair)
    full = draws.gaussian_block(seed, 4 * ((s + 3) // 4), j0, j1)
    r = np.repeat(np.hypot(full[0::2], full[1::2]), 2, axis=0)[:s]
    assert np.all(np.abs(g - ref) <= 2.0 ** -22 * (np.abs(ref) + r)), np.max(np.abs(g - ref) / (np.abs(ref) + r))
    for fmt, rnd in (("bf16", round_bf16), ("e4m3", round_e4m3)):
        gq = lib.draw_gaussian_device(seed, s, j0, j1, fmt).cpu().numpy().astype(np.float64)
        rq = rnd(ref)
        assert np.array_equal(gq, rq), (fmt, int((gq != rq).sum()))


# ---------------------------------------------------------------------------- sketches
SRHT_CASES = [
    ("plain_fp64", 2000, 50, 200, np.float64),
    ("ragged_fp32", 5003, 37, 150, np.float32),
    ("tiny_m", 40, 9, 16, np.float64),            # m_p = 64: explicit-formula kernel
    ("short_m", 100, 13, 40, np.float32),         # m_p = 128 < transform block
    ("multi_block", 70_000, 21, 300, np.float32),
    ("wide", 9000, 129, 1100, np.float64),        # s > 1024
]


@pytest.mark.parametrize("name,m,n,s,dt", SRHT_CASES)
def test_srht_sketch_parity(lib, name, m, n, s, dt):
    a = np.random.default_rng(hash(name) % 2 ** 32).standard_normal((m, n)).astype(dt)
    SA = lib.sketch(t(a), "srht", s, 31).cpu().numpy()
    ref = operators.sketch(a.astype(np.float64), "srht", s, 31)
    assert colrel(SA, ref) < 1e-12, colrel(SA, ref)
    SA32 = lib.sketch(t(a), "srht", s, 31, acc="f32").cpu().numpy()
    assert colrel(SA32, ref) < 1e-4


SRDCT_CASES = [
    ("tiny_m", 40, 9, 16, np.float64),            # m_p = 1024: one block, 984 padding rows
    ("padded", 1000, 13, 100, np.float32),
    ("ragged", 5003, 37, 150, np.float32),        # 8 blocks
    ("multi_block", 70_000, 21, 300, np.float32),  # 128 blocks
    ("wide", 9000, 129, 1100, np.float64),        # s > 1024: 64 sampled rows a thread
    ("tls_shape", 20_000, 201, 804, np.float32),  # the TLS workload's N and s
]


@pytest.mark.parametrize("name,m,n,s,dt", SRDCT_CASES)
def test_srdct_sketch_parity(lib, name, m, n, s, dt):
    a = np.random.default_rng(len(name) + m).standard_normal((m, n)).astype(dt)
    SA = lib.sketch(t(a), "srdct", s, 41).cpu().numpy()
    ref = operators.sketch(a.astype(np.float64), "srdct", s, 41)
    assert colrel(SA, ref) < 1e-12, colrel(SA, ref)
    SA32 = lib.sketch(t(a), "srdct", s, 41, acc="f32").cpu().numpy()
    assert colrel(SA32, ref) < 1e-4, colrel(SA32, ref)


HRHT_CASES = [
    ("tiny_m", 40, 9, 16, np.float64),            # m_p = 64: one block, the first 64 rows kept
    ("ragged", 5003, 37, 150, np.float32),        # 8 blocks
    ("multi_block", 70_000, 21, 300, np.float32),  # 128 blocks
    ("wide", 9000, 129, 1100, np.float64),        # s > 1024
    ("tls_shape", 20_000, 201, 804, np.float32),
]


@pytest.mark.parametrize("name,m,n,s,dt", HRHT_CASES)
def test_hrht_sketch_parity(lib, name, m, n, s, dt):
    a = np.random.default_rng(len(name) * 7 + m).standard_normal((m, n)).astype(dt)
    SA = lib.sketch(t(a), "hrht", s, 43).cpu().numpy()
    ref = operators.sketch(a.astype(np.float64), "hrht", s, 43)
    assert colrel(SA, ref) < 1e-12, colrel(SA, ref)


def test_srdct_one_workgroup_per_column_tile(lib):
    """One row group: a workgroup runs all 128 blocks, its per-sample rotation recurrence taken
    exactly every 32 blocks."""
    m, n, s = 131_000, 19, 256
    a = np.random.default_rng(5).standard_normal((m, n)).astype(np.float32)
    ref = operators.sketch(a.astype(np.float64), "srdct", s, 9)
    SA = lib.sketch(t(a), "srdct", s, 9, row_groups=1).cpu().numpy()
    assert colrel(SA, ref) < 1e-12, colrel(SA, ref)
    SA32 = lib.sketch(t(a), "srdct", s, 9, acc="f32", row_groups=1).cpu().numpy()
    assert colrel(SA32, ref) < 1e-4, colrel(SA32, ref)


@pytest.mark.parametrize("m,n,s,zeta,dt", [(5003, 37, 150, 8, np.float32), (20_000, 201, 804, 8, np.float32),
                                           (3000, 30, 90, 3, np.float64), (4100, 17, 64, 16, np.float32),
                                           (12_001, 40, 1206, 8, np.float32), (9000, 33, 200, 24, np.float32)])
def test_sparse_sketch_parity(lib, m, n, s, zeta, dt):
    # tiles (sparse_tile): 16 columns with two chunks of staged draws, except s = 1206 (8 columns:
    # 16 do not fit at FP64 accumulation) and zeta = 24 at s = 200 (16 columns, one chunk staged)
    a = np.random.default_rng(m + n).standard_normal((m, n)).astype(dt)
    SA = lib.sketch(t(a), "sparse", s, 77, zeta=zeta).cpu().numpy()
    ref = operators.sketch(a.astype(np.float64), "sparse", s, 77, zeta=zeta)
    assert colrel(SA, ref) < 1e-12, colrel(SA, ref)
    SA32 = lib.sketch(t(a), "sparse", s, 77, zeta=zeta, acc="f32").cpu().numpy()
    assert colrel(SA32, ref) < 1e-4


def test_sketch_column_blocks_equal_concatenation(lib):
    M, _ = W.tls_matrix(m=9000, n=40)
    Mt = t(M)
    whole = lib.sketch(Mt, "sparse", 164, 3).cpu().numpy()
    split = lib.sketch([Mt[:, :40].contiguous(), Mt[:, 40:].contiguous()], "sparse", 164, 3).cpu().numpy()
    assert np.array_equal(whole, split)
    strided = lib.sketch([Mt[:, :40], Mt[:, 40:]], "srht", 164, 3).cpu().numpy()
    ref = operators.sketch(M.astype(np.float64), "srht", 164, 3)
    assert colrel(strided, ref) < 1e-12


@pytest.mark.parametrize("fix_cap", [None, "0", "1"])
@pytest.mark.parametrize("fmt", ["bf16", "e4m3"])
def test_gaussian_sketch_parity(lib, fmt, fix_cap, monkeypatch):
    """fix_cap None: uncertified entries corrected after the K loop (the common path); "0" and
    "1" (NSK_GAUSS_FIX_CAP): the record list overflows, so every workgroup with an uncertified
    entry redoes its sums with the entries redrawn in place."""
    if fix_cap is None:
        monkeypatch.delenv("NSK_GAUSS_FIX_CAP", raising=False)
    else:
        monkeypatch.setenv("NSK_GAUSS_FIX_CAP", fix_cap)
    m, n, s = 6000, 45, 96
    rng = np.random.default_rng(9)
    a = rng.standard_normal((m, n)) * np.exp(rng.uniform(-2, 2, n))[None, :]
    if fmt == "bf16":
        at = t(a, torch.float64).to(torch.bfloat16)
        stored = at.to(torch.float64).cpu().numpy()
        SA = lib.sketch(at, "gauss", s, 12).cpu().numpy()
    else:
        e = np.floor(np.log2(448.0 / np.abs(a).max(axis=0))).astype(np.int8)
        q = t(a * 2.0 ** e[None, :], torch.float64).to(torch.float8_e4m3fn)
        stored = q.to(torch.float64).cpu().numpy() * 2.0 ** (-e[None, :].astype(np.float64))
        SA = lib.sketch([(q, t(-e))], "gauss", s, 12).cpu().numpy()
    ref = operators.sketch(stored, "gauss", s, 12, gauss_dtype=fmt)
    assert colrel(SA, ref) < 1e-4, colrel(SA, ref)


# ---------------------------------------------------------------------------- epsilon null space
@pytest.mark.parametrize("kind,n,d", [("srht", 24, 3), ("sparse", 100, 5), ("srdct", 40, 1), ("sparse", 30, 0)])
def test_epsilon_null_space(lib, kind, n, d):
    rng = np.random.default_rng(n + d)
    u = np.linalg.qr(rng.standard_normal((5000, n)))[0]
    v = np.linalg.qr(rng.standard_normal((n, n)))[0]
    sig = np.concatenate([np.linspace(3, 1, n - d), np.zeros(d)])
    a = (u * sig) @ v.T
    eps = 64 * U * n
    V, sigma, count = lib.null_space(t(a), eps, kind=kind, s=4 * n, seed=5)
    torch.cuda.synchronize()
    W, sg_ref, c_ref = method.null_space_eps(a, eps, kind, 4 * n, 5)
    assert int(count.item()) == c_ref == d
    assert np.abs(sigma.cpu().numpy() - sg_ref).max() <= 1e-13 * sg_ref[0]
    V = V.cpu().numpy()
    assert np.abs(V.T @ V - np.eye(n)).max() < 1e-12
    if d:
        assert metrics.sin_theta(v[:, -d:], V[:, n - d:]) < 1e-12


# ---------------------------------------------------------------------------- sketch updates
@pytest.mark.parametrize("kind,dt", [("srht", np.float64), ("srdct", np.float32), ("sparse", np.float32),
                                     ("sparse", np.float64)])
def test_row_downdate_and_update_match_oracle(lib, kind, dt):
    m, n, s, seed = 6000, 23, 96, 21
    rng = np.random.default_rng(len(kind) + m)
    a = rng.standard_normal((m, n)).astype(dt)
    SA = lib.sketch(t(a), kind, s, seed)
    # Algorithm 3: removing rows equals the sketch of the matrix without them
    gone = [0, 5, m - 1, 4097]
    lib.sketch_rows(SA, t(a[gone]), gone, [-1] * len(gone), m, kind=kind, seed=seed)
    a0 = a.astype(np.float64)
    a0[gone] = 0.0
    ref = operators.sketch(a0, kind, s, seed)
    assert colrel(SA.cpu().numpy(), ref) < 1e-12, colrel(SA.cpu().numpy(), ref)
    # Algorithm 2 / Section 5.3: appended rows add Gaussian columns; a re-added original row its own
    before = SA.cpu().numpy()
    new = rng.standard_normal((3, n)).astype(dt)
    rows, ops = [m, m + 7, 5], [1, 1, 1]
    lib.sketch_rows(SA, t(new), rows, ops, m, kind=kind, seed=seed)
    ref = updates.update_rows(before, kind, seed, m, rows, new.astype(np.float64), ops)
    assert colrel(SA.cpu().numpy() - before, ref - before) < 1e-12


def test_gaussian_row_update_matches_oracle(lib):
    m, n, s, seed = 4000, 16, 64, 22
    rng = np.random.default_rng(8)
    at = t(rng.standard_normal((m + 2, n)), torch.float64).to(torch.bfloat16)
    stored = at.to(torch.float64).cpu().numpy()
    SA = lib.sketch(at[:m].contiguous(), "gauss", s, seed)
    before = SA.cpu().numpy()
    lib.sketch_rows(SA, at[m:].contiguous(), [m, m + 1], [1, 1], m, kind="gauss", seed=seed)
    delta = SA.cpu().numpy() - before
    ref = updates.update_rows(np.zeros_like(before), "gauss", seed, m, [m, m + 1], stored[m:], [1, 1],
                              gauss_dtype="bf16")
    # G_hat from FP32 Box-Muller on the device and FP64 on the host: rare one-step rounding flips
    close = np.abs(delta - ref) <= 1e-12 * np.abs(ref).max()
    assert close.mean() > 0.99, close.mean()
    assert rel(delta, ref) < 1e-2


@pytest.mark.parametrize("kind", ["srht", "srdct", "sparse"])
def test_column_update_writes_into_sketch_columns(lib, kind):
    m, n, s = 9000, 40, 164
    a = np.random.default_rng(9).standard_normal((m, n)).astype(np.float32)
    whole = lib.sketch(t(a), kind, s, 4).cpu().numpy()
    SA = torch.zeros((s, n), dtype=torch.float64, device=DEV)
    lib.sketch(t(a[:, :37]), kind, s, 4, out=SA[:, :37])
    lib.sketch(t(a[:, 37:]), kind, s, 4, out=SA[:, 37:])
    assert colrel(SA.cpu().numpy(), whole) < 1e-13


# ---------------------------------------------------------------------------- solves
def test_plain_workload_trailing_vector(lib):
    a, _, v = W.plain_matrix()
    Vk, sk, info = lib.trailing_rsv(t(a), 1, kind="srht", s=200, seed=1, residual=True)
    torch.cuda.synchronize()
    vk_ref, sk_ref, sa, sig, V, sweeps = method.trailing_rsv(a, 1, "srht", 200, 1, return_all=True)
    Vk = Vk.cpu().numpy()
    assert_vectors(vk_ref, Vk, vec_tol(sig, 1))
    assert abs(float(sk[0]) - sk_ref[0]) <= 1e-14 * sig[0]
    inf = lib.read_info(info)
    assert inf.converged and inf.sweeps <= 30
    assert abs(inf.sigma_max - sig[0]) <= 1e-13 * sig[0]
    assert abs(inf.residual - np.linalg.norm(a @ Vk)) <= 1e-15 * np.linalg.norm(a)
    # sign normalisation as the oracle: largest-magnitude entry positive
    assert Vk[np.argmax(np.abs(Vk[:, 0])), 0] > 0


@pytest.mark.parametrize("kind,dt,acc", [("sparse", np.float32, "f64"), ("srht", np.float32, "f64"),
                                         ("sparse", np.float32, "f32"), ("srht", np.float64, "f64"),
                                         ("srdct", np.float32, "f64"), ("srdct", np.float32, "f32"),
                                         ("hrht", np.float32, "f64")])
def test_tls_trailing_vector_and_residual_ratio(lib, kind, dt, acc):
    M, _ = W.tls_matrix(m=30_000, n=60, dtype=dt)
    s = 4 * 61
    Vk, sk, info = lib.trailing_rsv(t(M), 1, kind=kind, s=s, seed=8, acc=acc)
    torch.cuda.synchronize()
    M64 = M.astype(np.float64)
    vk_ref, sk_ref, sa, sig, V, _ = method.trailing_rsv(M64, 1, kind, s, 8, return_all=True)
    u = U if acc == "f64" else 2.0 ** -24
    assert_vectors(vk_ref, Vk.cpu().numpy(), max(vec_tol(sig, 1, u), 1e-10 if acc == "f64" else 1e-4))
    w_opt, _, _ = metrics.trailing_exact(M64, 1)
    r_gpu = metrics.residual_ratio(M64, Vk.cpu().numpy(), w_opt)
    r_ref = metrics.residual_ratio(M64, vk_ref, w_opt)
    assert abs(r_gpu - r_ref) <= (1e-10 if acc == "f64" else 1e-4)


def test_planted_near_null_subspace_k4(lib):
    a, vp = W.planted_matrix(20_000, 64, seed=(4, 1))
    Vk, sk, _ = lib.trailing_rsv(t(a), 4, kind="srht", s=256, seed=3)
    torch.cuda.synchronize()
    vk_ref, sk_ref, sa, sig, V, _ = method.trailing_rsv(a.astype(np.float64), 4, "srht", 256, 3, return_all=True)
    assert_vectors(vk_ref, Vk.cpu().numpy(), vec_tol(sig, 4))
    assert np.allclose(sk.cpu().numpy(), sk_ref, rtol=1e-9, atol=1e-13 * sig[0])


# Column counts that select each rows-per-lane variant of the Jacobi (N > 64 runs the
# multi-workgroup kernel) and k large enough to need several replay batches.
@pytest.mark.parametrize("m,N,k,kind", [(8000, 100, 3, "sparse"), (9000, 150, 5, "srht"),
                                        (12_000, 201, 2, "sparse"), (15_000, 300, 4, "sparse")])
def test_trailing_vectors_block_jacobi_shapes(lib, m, N, k, kind):
    a = W.planted_matrix(m, N, k=k, level=1e-4, seed=(8, N))[0].astype(np.float64)
    s = 4 * N
    Vk, sk, info = lib.trailing_rsv(t(a), k, kind=kind, s=s, seed=11)
    torch.cuda.synchronize()
    vk_ref, sk_ref, sa, sig, V, _ = method.trailing_rsv(a, k, kind, s, 11, return_all=True)
    assert_vectors(vk_ref, Vk.cpu().numpy(), vec_tol(sig, k))
    assert np.allclose(sk.cpu().numpy(), sk_ref, rtol=1e-10, atol=1e-14 * sig[0])
    assert lib.read_info(info).converged


@pytest.mark.parametrize("m,n,k,s,kind", [(64, 16, 16, 64, "srht"), (300, 1, 1, 8, "sparse"),
                                          (1000, 8, 3, 1000, "srht"), (513, 5, 2, 10, "sparse"),
                                          (1000, 8, 3, 1000, "srdct"), (64, 16, 16, 64, "srdct")])
def test_edge_shapes(lib, m, n, k, s, kind):
    a = np.random.default_rng(m).standard_normal((m, n))
    Vk, sk, _ = lib.trailing_rsv(t(a), k, kind=kind, s=s, seed=2)
    torch.cuda.synchronize()
    vk_ref, sk_ref, sa, sig, V, _ = method.trailing_rsv(a, k, kind, s, 2, return_all=True)
    if k < n:
        assert_vectors(vk_ref, Vk.cpu().numpy(), vec_tol(sig, k))
    else:
        assert np.abs(Vk.cpu().numpy().T @ Vk.cpu().numpy() - np.eye(n)).max() < 1e-13
    assert np.allclose(sk.cpu().numpy(), sk_ref, rtol=1e-10, atol=1e-14 * sig[0])


def test_nonconvergence_flag_and_nan_propagation(lib):
    M, _ = W.tls_matrix(m=5000, n=40, dtype=np.float64)
    _, _, info = lib.trailing_rsv(t(M), 1, kind="sparse", s=164, seed=1, max_sweeps=1)
    torch.cuda.synchronize()
    inf = lib.read_info(info)
    assert inf.sweeps == 1 and not inf.converged
    M[17, 3] = np.nan
    Vk, sk, _ = lib.trailing_rsv(t(M), 1, kind="sparse", s=164, seed=1)
    torch.cuda.synchronize()
    assert not np.isfinite(sk.cpu().numpy()).all() or not np.isfinite(Vk.cpu().numpy()).all()


def test_deterministic_bitwise(lib):
    M, _ = W.tls_matrix(m=40_000, n=100)
    Mt = t(M)
    a = lib.trailing_rsv(Mt, 1, kind="sparse", s=404, seed=5)
    b = lib.trailing_rsv(Mt, 1, kind="sparse", s=404, seed=5)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    c = lib.sketch(Mt, "srht", 404, 5)
    d = lib.sketch(Mt, "srht", 404, 5)
    assert torch.equal(c, d)
    e = lib.sketch(Mt, "srdct", 404, 5)
    f = lib.sketch(Mt, "srdct", 404, 5)
    assert torch.equal(e, f)


@pytest.mark.parametrize("m,N,k", [(12_000, 201, 2), (9000, 150, 3), (20_000, 320, 2)])
def test_coop_hand_over_forms_agree_bitwise(lib, m, N, k, monkeypatch):
    """The multi-workgroup QR and Jacobi hand columns between workgroups either within one
    XCD's L2 (the default where every worker shares an XCD) or with agent-scope release and
    acquire (NSK_COOP_LOCAL=0); the arithmetic is the same, so the results agree bit for bit,
    and both match the oracle."""
    a = W.planted_matrix(m, N, k=k, level=1e-4, seed=(9, N))[0].astype(np.float64)
    at = t(a)
    s = 4 * N
    monkeypatch.delenv("NSK_COOP_LOCAL", raising=False)
    v1, s1, i1 = lib.trailing_rsv(at, k, kind="sparse", s=s, seed=13)
    torch.cuda.synchronize()
    monkeypatch.setenv("NSK_COOP_LOCAL", "0")
    v0, s0, i0 = lib.trailing_rsv(at, k, kind="sparse", s=s, seed=13)
    torch.cuda.synchronize()
    assert torch.equal(v1, v0) and torch.equal(s1, s0)
    assert lib.read_info(i1).sweeps == lib.read_info(i0).sweeps and lib.read_info(i1).converged
    vk_ref, sk_ref, sa, sig, V, _ = method.trailing_rsv(a, k, "sparse", s, 13, return_all=True)
    assert_vectors(vk_ref, v1.cpu().numpy(), vec_tol(sig, k))


@pytest.mark.parametrize("m,N", [(40_003, 201), (5_001, 37), (777, 4), (9_999, 256), (3, 10)])
def test_residual_contiguous_rows(lib, m, N):
    # FP32 rows in one buffer, k = 1 (one 16-byte load per lane and row): as one block, as the
    # TLS split [A | b] of the same buffer, and as blocks of separate buffers (the general path)
    M = np.random.default_rng(m + N).standard_normal((m, N)).astype(np.float32)
    v = np.random.default_rng(N).standard_normal((N, 1))
    ref = np.linalg.norm(M.astype(np.float64) @ v)
    Mt = t(M)
    whole = float(lib.residual(Mt, t(v)))
    split = float(lib.residual([Mt[:, :N - 1], Mt[:, N - 1:]], t(v)))
    apart = float(lib.residual([Mt[:, :N - 1].contiguous(), Mt[:, N - 1:].contiguous()], t(v)))
    for r in (whole, split, apart):
        assert abs(r - ref) <= 1e-13 * ref, (r, ref)
    assert whole == split


def test_residual_entry_point(lib):
    a = np.random.default_rng(3).standard_normal((50_001, 33)).astype(np.float32)
    v = np.linalg.qr(np.random.default_rng(4).standard_normal((33, 3)))[0]
    r = float(lib.residual(t(a), t(v)))
    ref = np.linalg.norm(a.astype(np.float64) @ v)
    assert abs(r - ref) <= 1e-13 * ref


# ---------------------------------------------------------------------------- TLS + grad
def test_tls_solution_and_gradient(lib):
    m, n, s = 3000, 30, 124
    M, _ = W.tls_matrix(m=m, n=n, seed=21, dtype=np.float64)
    xt = W.tls_target(n)
    x, state, _ = lib.tls_solve(t(M[:, :n]), t(M[:, n]), kind="sparse", s=s, seed=6)
    grad, x_ref, _ = method.tls_grad(M, xt, "sparse", s, 6)
    torch.cuda.synchronize()
    assert rel(x.cpu().numpy(), x_ref) < 1e-10
    gx = 2.0 * (x - t(xt))
    dA, db = lib.tls_backward(state, m, n, gx, kind="sparse", s=s, seed=6, out_dtype=torch.float64)
    torch.cuda.synchronize()
    g_gpu = np.hstack([dA.cpu().numpy(), db.cpu().numpy()[:, None]])
    assert rel(g_gpu, grad) < 1e-10, rel(g_gpu, grad)


def test_tls_gradient_wide(lib):
    # N = 201: multi-workgroup Jacobi and a replay spread over three waves in the adjoint
    m, n, s = 5000, 200, 804
    M, _ = W.tls_matrix(m=m, n=n, seed=24, dtype=np.float64)
    xt = W.tls_target(n, seed=11)
    x, state, _ = lib.tls_solve(t(M[:, :n]), t(M[:, n]), kind="sparse", s=s, seed=12)
    grad, x_ref, _ = method.tls_grad(M, xt, "sparse", s, 12)
    gx = 2.0 * (x - t(xt))
    dA, db = lib.tls_backward(state, m, n, gx, kind="sparse", s=s, seed=12, out_dtype=torch.float64)
    torch.cuda.synchronize()
    g_gpu = np.hstack([dA.cpu().numpy(), db.cpu().numpy()[:, None]])
    assert rel(x.cpu().numpy(), x_ref) < 1e-10
    assert rel(g_gpu, grad) < 1e-9, rel(g_gpu, grad)


def test_tls_gradient_at_finite_difference_shape(lib):
    # the gradient workload's check shape: m = 5000, n = 256, s = 1024, FP64
    m, n, s = 5000, 256, 1024
    M, _ = W.tls_matrix(m=m, n=n, seed=5, dtype=np.float64)
    xt = W.tls_target(n)
    x, state, _ = lib.tls_solve(t(M[:, :n]), t(M[:, n]), kind="sparse", s=s, seed=5)
    grad, x_ref, _ = method.tls_grad(M, xt, "sparse", s, 5)
    gx = 2.0 * (x - t(xt))
    dA, db = lib.tls_backward(state, m, n, gx, kind="sparse", s=s, seed=5, out_dtype=torch.float64)
    torch.cuda.synchronize()
    g_gpu = np.hstack([dA.cpu().numpy(), db.cpu().numpy()[:, None]])
    assert rel(x.cpu().numpy(), x_ref) < 1e-10
    assert rel(g_gpu, grad) < 1e-9, rel(g_gpu, grad)


def test_tls_gradient_srht_kind(lib):
    m, n, s = 2000, 12, 52
    M, _ = W.tls_matrix(m=m, n=n, seed=22, dtype=np.float64)
    xt = W.tls_target(n, seed=9)
    x, state, _ = lib.tls_solve(t(M[:, :n]), t(M[:, n]), kind="srht", s=s, seed=7)
    grad, x_ref, _ = method.tls_grad(M, xt, "srht", s, 7)
    gx = 2.0 * (x - t(xt))
    dA, db = lib.tls_backward(state, m, n, gx, kind="srht", s=s, seed=7, out_dtype=torch.float64)
    torch.cuda.synchronize()
    g_gpu = np.hstack([dA.cpu().numpy(), db.cpu().numpy()[:, None]])
    assert rel(x.cpu().numpy(), x_ref) < 1e-10
    assert rel(g_gpu, grad) < 1e-10


def test_autograd_function(lib):
    m, n, s = 4000, 20, 84
    M, _ = W.tls_matrix(m=m, n=n, seed=23, dtype=np.float64)
    xt = W.tls_target(n, seed=4)
    A = t(M[:, :n]).requires_grad_(True)
    b = t(M[:, n]).requires_grad_(True)
    x = lib.TLSSketch.apply(A, b, s, 10, "sparse", 8)
    loss = ((x - t(xt)) ** 2).sum()
    loss.backward()
    grad, _, lref = method.tls_grad(M, xt, "sparse", s, 10)
    assert abs(float(loss.detach()) - lref) <= 1e-10 * lref
    g = np.hstack([A.grad.cpu().numpy(), b.grad.cpu().numpy()[:, None]])
    assert rel(g, grad) < 1e-10


# ---------------------------------------------------------------------------- batched
@pytest.mark.skip(reason=BATCHED_FAULT)
def test_batched_matches_single_instances(lib):
    shapes = [(5000, 16), (12_345, 40), (30_000, 100), (8192, 9), (20_001, 64), (7000, 33)]
    As = [W.planted_matrix(m, n, seed=(4, 100 + i))[0] for i, (m, n) in enumerate(shapes)]
    ks = [4 if n > 8 else 2 for _, n in shapes]
    ss = [4 * n for _, n in shapes]
    seeds = [1000 + i for i in range(len(shapes))]
    outs = lib.trailing_rsv_batched([t(a) for a in As], ks, ss, seeds)
    torch.cuda.synchronize()
    for a, (Vk, sk, info), k, s, seed in zip(As, outs, ks, ss, seeds):
        vk_ref, sk_ref, sa, sig, V, _ = method.trailing_rsv(a.astype(np.float64), k, "srht", s, seed,
                                                             return_all=True)
        assert_vectors(vk_ref, Vk.cpu().numpy(), vec_tol(sig, k))
        assert np.allclose(sk.cpu().numpy(), sk_ref, rtol=1e-9, atol=1e-13 * sig[0])
        assert lib.read_info(info).converged


# ---------------------------------------------------------------------------- AAA with sketch reuse
@pytest.mark.parametrize("kind", ["srht", "srdct", "sparse"])
def test_aaa_sketch_reuse_matches_oracle(lib, kind):
    """The GPU loop takes the oracle's support points while the errors are well above rounding
    (the argmax is decided by margins far larger than the two SVDs' differences); both reach the
    tolerance with the same or a neighbouring degree."""
    from oracle import aaa
    m, n_max, tol, s = 20_000, 40, 1e-10, 160
    z = np.sort(np.random.default_rng(11).uniform(-1, 1, m))
    f = np.tanh(50 * z)
    sup, w, hist = lib.aaa(t(z), t(f), n_max, tol, kind=kind, s=s, seed=6)
    sup_ref, w_ref, hist_ref = aaa.aaa(z, f, n_max, tol, kind=kind, s=s, seed=6)
    sure = next((i for i, h in enumerate(hist_ref) if h < 1e-6), len(hist_ref))
    assert sup[:sure] == sup_ref[:sure], (sup, sup_ref)
    assert np.allclose(hist[:sure], hist_ref[:sure], rtol=1e-6)
    assert hist[-1] <= tol and hist_ref[-1] <= tol
    assert abs(len(sup) - len(sup_ref)) <= 2
    if sup == sup_ref:
        assert metrics.sin_theta(w_ref[:, None], w.cpu().numpy()[:, None]) < 1e-6
    # the returned approximant's error at every sample point, recomputed on the host
    from oracle.aaa import barycentric
    r = barycentric(z, f, sup, w.cpu().numpy())
    assert np.abs(f - r).max() <= 1.01 * hist[-1] + 1e-15


# ---------------------------------------------------------------------------- large N, several right-hand sides
def test_large_path_trailing_vectors(lib):
    """N = 400 is past the register-blocked SVD: the multi-workgroup QR, then the large-N
    Jacobi on R."""
    m, N, k, s = 8192, 400, 3, 800
    a = W.planted_matrix(m, N, k=k, level=1e-4, seed=(8, N))[0].astype(np.float64)
    Vk, sk, info = lib.trailing_rsv(t(a), k, kind="srht", s=s, seed=12)
    torch.cuda.synchronize()
    vk_ref, sk_ref, sa, sig, V, _ = method.trailing_rsv(a, k, "srht", s, 12, return_all=True)
    assert_vectors(vk_ref, Vk.cpu().numpy(), vec_tol(sig, k))
    assert np.allclose(sk.cpu().numpy(), sk_ref, rtol=1e-10, atol=1e-14 * sig[0])
    inf = lib.read_info(info)
    assert inf.converged and abs(inf.sigma_max - sig[0]) <= 1e-12 * sig[0]


def test_large_path_streamed_columns(lib):
    """s = 4400 is past the multi-workgroup QR (s <= 4096), so the large-N Jacobi runs on SA
    itself, past its register chunks (s <= 2048): the column pairs of SA are streamed from
    memory, V's pair still held in registers.  A sparse-sign sketch this tall fits the LDS only
    with FP32 accumulation, so the tolerances are FP32 ones: sin theta to sqrt(N) u32 kappa_gap
    and the singular values to u32 sigma_1 (an FP32-rounded SA moves them by about that much).
    The expected vectors are LAPACK's SVD of the oracle's FP64 sketch."""
    m, N, k, s = 9000, 330, 3, 4400
    a = W.planted_matrix(m, N, k=k, level=1e-4, seed=(9, N))[0].astype(np.float64)
    Vk, sk, info = lib.trailing_rsv(t(a), k, kind="sparse", s=s, seed=13, acc="f32")
    torch.cuda.synchronize()
    sa = operators.sketch(a, "sparse", s, 13)
    _, sig, vt = np.linalg.svd(sa, full_matrices=False)
    vk_ref, sk_ref = vt[-k:].T, sig[-k:]
    u32 = 2.0 ** -24
    assert_vectors(vk_ref, Vk.cpu().numpy(), vec_tol(sig, k, u=u32))
    assert np.allclose(sk.cpu().numpy(), sk_ref, rtol=0, atol=8 * u32 * sig[0])
    inf = lib.read_info(info)
    assert inf.converged and abs(inf.sigma_max - sig[0]) <= 8 * u32 * sig[0]


def test_large_path_maximum_width(lib):
    """The largest accepted shape of the SVD: N = 1024 columns with s = 2048 (the Hadamard
    kind's largest sketch), planted k = 2.  Expected vectors: LAPACK's SVD of the oracle's
    sketch."""
    m, N, k, s = 4096, 1024, 2, 2048
    a = W.planted_matrix(m, N, k=k, level=1e-4, seed=(10, N))[0].astype(np.float64)
    Vk, sk, info = lib.trailing_rsv(t(a), k, kind="srht", s=s, seed=14)
    torch.cuda.synchronize()
    sa = operators.sketch(a, "srht", s, 14)
    _, sig, vt = np.linalg.svd(sa, full_matrices=False)
    assert_vectors(vt[-k:].T, Vk.cpu().numpy(), vec_tol(sig, k))
    assert np.allclose(sk.cpu().numpy(), sig[-k:], rtol=1e-10, atol=1e-14 * sig[0])
    inf = lib.read_info(info)
    assert inf.converged and abs(inf.sigma_max - sig[0]) <= 1e-12 * sig[0]


def test_multi_rhs_tls_matches_oracle(lib):
    m, n, k, s = 5000, 40, 3, 172
    rng = np.random.default_rng(15)
    a = rng.standard_normal((m, n))
    b = a @ rng.standard_normal((n, k)) + 1e-3 * rng.standard_normal((m, k))
    X, Vk, sk, _ = lib.tls_solve_multi(t(a), t(b), kind="sparse", s=s, seed=4)
    torch.cuda.synchronize()
    X_ref, vk_ref, sk_ref = method.tls_solve_multi(np.hstack([a, b]), k, "sparse", s, 4)
    assert rel(X.cpu().numpy(), X_ref) < 1e-10, rel(X.cpu().numpy(), X_ref)


def test_multi_rhs_tls_table1_shape(lib):
    """Table 1's shape: n = 1000, k = 10, s = 2(n + k) = 2020, DCT-II sketch, m = 2^14; A with
    singular values geometric from 1 to 1e-3, B in A's range plus noise.  The expected
    vectors are LAPACK's SVD of the oracle's sketch (the oracle's own Jacobi, pinned to LAPACK,
    would take minutes at N = 1010)."""
    m, n, k, s = 1 << 14, 1000, 10, 2020
    M = W.table1_tls_matrix(m, n, k, seed=16)
    a, b = M[:, :n], M[:, n:]
    X, Vk, sk, info = lib.tls_solve_multi(t(a), t(b), kind="srdct", s=s, seed=9)
    torch.cuda.synchronize()
    sa = operators.sketch(M, "srdct", s, 9)
    _, sig, vt = np.linalg.svd(sa, full_matrices=False)
    V = vt[-k:].T
    assert_vectors(V, Vk.cpu().numpy(), vec_tol(sig, k))
    X_ref = -np.linalg.solve(V[n:].T, V[:n].T).T
    gap_amp = np.linalg.norm(np.linalg.inv(V[n:]), 2)          # X's sensitivity to the vectors
    assert rel(X.cpu().numpy(), X_ref) <= 10 * vec_tol(sig, k) * gap_amp * (1 + np.linalg.norm(X_ref, 2))
    assert lib.read_info(info).converged
