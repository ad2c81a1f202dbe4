"""nsk_trailing_rsv_noalloc (the library's fixed device array as workspace) against
nsk_trailing_rsv with a caller workspace, through the C ABI: two calls in a row, the second
on a smaller input, each bitwise equal to the workspace entry point's result (same kernels,
same launch plan, deterministic reduction order)."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _call_noalloc(lib, M, k, kind, s, seed):
    raw = lib.load()
    ops, nb, m, N, dev, keep = lib._blocks(M)
    d = lib.make_desc(kind, s, seed, flags=lib.FLAG_RESIDUAL)
    Vk = torch.empty((N, k), dtype=torch.float64, device=DEV)
    sig = torch.empty(k, dtype=torch.float64, device=DEV)
    info = torch.zeros(lib.INFO_BYTES, dtype=torch.uint8, device=DEV)
    rc = raw.nsk_trailing_rsv_noalloc(ops, nb, m, k, ctypes.byref(d), Vk.data_ptr(), sig.data_ptr(),
                                      info.data_ptr(), lib._stream(dev))
    assert rc == 0, lib.STATUS.get(rc, rc)
    return Vk, sig, info


def test_noalloc_matches_workspace_entry_point(lib):
    cases = [(300_000, 150, "sparse", 604, 2, 21), (20_000, 40, "srht", 164, 3, 22)]   # second smaller
    for m, n, kind, s, k, seed in cases:
        M, _ = W.tls_matrix(m=m, n=n, seed=seed)
        Mt = torch.from_numpy(M).to(DEV)
        blocks = [Mt[:, :n], Mt[:, n:]]
        Vk, sig, info = _call_noalloc(lib, blocks, k, kind, s, seed)
        Vr, sr, ir = lib.trailing_rsv(blocks, k, kind=kind, s=s, seed=seed, residual=True)
        torch.cuda.synchronize()
        assert torch.equal(Vk, Vr) and torch.equal(sig, sr)
        a, b = lib.read_info(info), lib.read_info(ir)
        assert a.converged and a.sweeps == b.sweeps and a.residual == b.residual


def test_noalloc_rejects_oversized_workspace(lib):
    raw = lib.load()
    d = lib.make_desc("sparse", 804, 1)
    assert raw.nsk_workspace_bytes(20_000_000, 201, 1, ctypes.byref(d)) > raw.nsk_noalloc_scratch_bytes()
    A = torch.empty((16, 201), dtype=torch.float32, device=DEV)      # pointer only: rejected first
    ops = (lib.Operand * 1)(lib.Operand(A.data_ptr(), lib.F32, 0, 201, 201, None))
    rc = raw.nsk_trailing_rsv_noalloc(ops, 1, 20_000_000, 1, ctypes.byref(d), A.data_ptr(), A.data_ptr(),
                                      None, lib._stream(A.device))
    assert rc == 2   # NSK_EWORKSPACE
