"""The device entry points are stream-ordered: a call enqueues its work on the caller's stream
and returns while earlier work on that stream is still running, and its results are those of
the same call on an idle stream.

A long spin kernel (torch's ``_sleep``) is queued first; each call must return long before the
spin ends, and the stream must still be busy when the call has returned.
"""
import time

import numpy as np
import pytest
import torch

import workloads as W
from conftest import BATCHED_FAULT

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SPIN_MS = 400.0


def t(x):
    return torch.tensor(np.ascontiguousarray(x), device=DEV)


@pytest.fixture(scope="module")
def spin_cycles():
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda._sleep(1000)
    torch.cuda.synchronize()
    e0.record()
    torch.cuda._sleep(2_000_000)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    return int(2_000_000 * SPIN_MS / max(ms, 1e-3))


def _check_async(spin_cycles, call):
    ref = call()                      # warm-up: the allocator's blocks and the kernels' first load
    torch.cuda.synchronize()
    torch.cuda._sleep(spin_cycles)
    t0 = time.perf_counter()
    out = call()
    dt_ms = (time.perf_counter() - t0) * 1e3
    done = torch.cuda.Event()
    done.record()
    busy = not done.query()
    torch.cuda.synchronize()
    assert busy, "the spin kernel had finished before the call returned"
    assert dt_ms < SPIN_MS / 4, dt_ms
    for a, b in zip(ref, out):
        assert torch.equal(a, b)


@pytest.mark.parametrize("kind", ["srht", "srdct", "sparse"])
def test_sketch_and_solve_return_while_stream_busy(lib, spin_cycles, kind):
    M, _ = W.tls_matrix(m=60_000, n=40)
    Mt = t(M)
    _check_async(spin_cycles, lambda: (lib.sketch(Mt, kind, 164, 3),))
    _check_async(spin_cycles, lambda: lib.trailing_rsv(Mt, 1, kind=kind, s=164, seed=3)[:2])
    _check_async(spin_cycles, lambda: (lib.tls_solve(Mt[:, :40], Mt[:, 40:], kind=kind, s=164, seed=3)[0],))


def test_tls_backward_returns_while_stream_busy(lib, spin_cycles):
    M, _ = W.tls_matrix(m=20_000, n=30, dtype=np.float64)
    Mt = t(M)
    x, state, _ = lib.tls_solve(Mt[:, :30], Mt[:, 30:], kind="srht", s=124, seed=4)
    gx = 2.0 * x
    _check_async(spin_cycles, lambda: lib.tls_backward(state, 20_000, 30, gx, kind="srht", s=124, seed=4,
                                                       out_dtype=torch.float64))


@pytest.mark.skip(reason=BATCHED_FAULT)
def test_batched_returns_while_stream_busy(lib, spin_cycles):
    shapes = [(6000, 40), (9000, 130), (5000, 16)]
    As = [t(W.planted_matrix(m, n, seed=(4, 500 + i))[0]) for i, (m, n) in enumerate(shapes)]
    ks, ss, seeds = [4, 4, 2], [4 * n for _, n in shapes], [11, 12, 13]
    _check_async(spin_cycles, lambda: [x for o in lib.trailing_rsv_batched(As, ks, ss, seeds) for x in o[:2]])


def test_row_update_returns_while_stream_busy(lib, spin_cycles):
    a = np.random.default_rng(2).standard_normal((6000, 20))
    At = t(a)
    base = lib.sketch(At, "srht", 80, 9)
    vals = t(a[[3, 17]])          # made before the spin: indexing with a host list copies and waits

    def call():
        SA = base.clone()
        lib.sketch_rows(SA, vals, [3, 17], [-1, -1], 6000, kind="srht", seed=9)
        return (SA,)
    _check_async(spin_cycles, call)
