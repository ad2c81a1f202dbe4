"""Pins for the oracle's random draws (no GPU).

* Philox4x32-10 equals rocRAND's ``philox4x32_10_engine`` (an independent implementation,
  compiled from its source header) bit for bit.
* Draw objects have the exact structural properties their definitions fix (distinct rows,
  +-1 signs, sorted SRHT rows) and pass uniformity statistics.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

from oracle import draws
from oracle.philox import block, philox4x32

ROCRAND_PROG = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  for (int a = 1; a + 2 < argc; a += 3) {
    unsigned long long seed = strtoull(argv[a], 0, 0);
    unsigned long long sub = strtoull(argv[a + 1], 0, 0);
    unsigned long long idx = strtoull(argv[a + 2], 0, 0);
    rocrand_device::philox4x32_10_engine e(seed, sub, 4ull * idx);
    uint4 r = e.next4();
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_exe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not (os.path.exists(hipcc) and os.path.exists(hdr)):
        pytest.skip("rocRAND header or hipcc not available")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "rr.cpp")
    exe = os.path.join(d, "rr")
    with open(src, "w") as f:
        f.write(ROCRAND_PROG)
    subprocess.run([hipcc, "-O1", src, "-o", exe], check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(rocrand_exe):
    # rocRAND's engine(seed, subsequence, offset=4*idx) evaluates the block with counter
    # (lo(idx), hi(idx), lo(subsequence), hi(subsequence)) and key (lo(seed), hi(seed));
    # the offset is a 64-bit count of words, so idx < 2**62.
    cases = [(0, 0, 0), (1, 0, 0), (0xFFFFFFFFFFFFFFFF, 0xFFFFFFFFFFFFFFFF, (1 << 62) - 1),
             (0x123456789ABCDEF, (5 << 32) | 3, 77), (42, (1 << 32) | 2, 1 << 33),
             (2023, 7, 123456789)]
    args = []
    for c in cases:
        args += [str(x) for x in c]
    out = subprocess.run([rocrand_exe] + args, check=True, capture_output=True, text=True).stdout
    got = [list(map(int, line.split())) for line in out.strip().splitlines()]
    for (seed, sub, idx), ref in zip(cases, got):
        w = philox4x32(idx & 0xFFFFFFFF, idx >> 32, sub & 0xFFFFFFFF, sub >> 32,
                       seed & 0xFFFFFFFF, seed >> 32)
        assert [int(x) for x in w] == ref


def test_philox_known_answer_vectors():
    """The generator's published known-answer vectors (zero, all-ones and pi-digit inputs)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        c0, c1, c2, c3, k0, k1, *want = (int(x, 16) for x in r)
        got = philox4x32(c0, c1, c2, c3, k0, k1)
        assert [int(w) for w in got] == want, (r, [hex(int(w)) for w in got])


def test_philox_vectorised_equals_scalar():
    idx = np.arange(0, 5000, 37, dtype=np.uint64)
    v = np.stack(block(99, idx, 3, 2))
    for col, i in enumerate(idx):
        s = np.stack(block(99, int(i), 3, 2)).ravel()
        assert (v[:, col] == s).all()


def test_philox_uniform_words():
    w = np.concatenate(block(7, np.arange(20000, dtype=np.uint64), 0, 9))
    # top 4 bits uniform over 16 bins
    h = np.bincount((w >> np.uint64(28)).astype(np.int64), minlength=16)
    assert stats.chisquare(h).pvalue > 1e-4
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint64)) & np.uint64(1)).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 0.01)


def test_signs_balanced_and_deterministic():
    d = draws.signs(5, 100_003)
    assert set(np.unique(d)) == {-1, 1}
    assert abs(d.mean()) < 5 / np.sqrt(d.size)
    assert (draws.signs(5, 1000) == d[:1000]).all()      # prefix property of the counter map
    assert not (draws.signs(6, 1000) == d[:1000]).all()


@pytest.mark.parametrize("pool,s", [(16, 16), (64, 16), (2048, 200), (1 << 17, 1000)])
def test_srht_rows_distinct_sorted(pool, s):
    r = draws.srht_rows(3, pool, s)
    assert r.size == s and np.all(np.diff(r) > 0)
    assert r[0] >= 0 and r[-1] < pool
    if s == pool:
        assert (r == np.arange(pool)).all()


def test_srht_rows_uniform():
    pool, s = 32, 8
    counts = np.zeros(pool)
    for seed in range(3000):
        counts[draws.srht_rows(seed, pool, s)] += 1
    assert stats.chisquare(counts).pvalue > 1e-4


def test_floyd_draw_rule():
    # t-th draw: x = floor(u * (i+1) / 2^64) with u from words 0,1 of block (t, 0, stream 2)
    seed, pool, s = 11, 40, 10
    w0, w1, _, _ = block(seed, np.arange(s, dtype=np.uint64), 0, draws.STREAM_ROWS)
    taken = []
    for t in range(s):
        u = int(w0[t]) + (int(w1[t]) << 32)
        i = pool - s + t
        x = (u * (i + 1)) >> 64
        taken.append(i if x in taken else x)
    assert sorted(taken) == list(draws.srht_rows(seed, pool, s))


@pytest.mark.parametrize("s,zeta", [(8, 8), (30, 8), (804, 8), (100, 3), (64, 32)])
def test_sparse_supports(s, zeta):
    rows, sgn = draws.sparse(4, 5000, s, zeta)
    assert rows.shape == (5000, zeta) and sgn.shape == (5000, zeta)
    assert rows.min() >= 0 and rows.max() < s
    srt = np.sort(rows, axis=1)
    assert np.all(np.diff(srt, axis=1) > 0)               # distinct within each column of S
    assert set(np.unique(sgn)) <= {-1, 1}
    if zeta == s:
        assert (srt == np.arange(s)).all()


def test_sparse_rows_and_signs_uniform():
    rows, sgn = draws.sparse(8, 40_000, 50, 8)
    h = np.bincount(rows.ravel(), minlength=50)
    assert stats.chisquare(h).pvalue > 1e-4
    assert abs(sgn.mean()) < 5 / np.sqrt(sgn.size)


def test_gaussian_moments():
    g = draws.gaussian_block(12, 64, 0, 4000).ravel()
    assert abs(g.mean()) < 5 / np.sqrt(g.size)
    assert abs(g.var() - 1) < 0.02
    assert stats.kstest(g, "norm").pvalue > 1e-4
    # rows beyond s are a prefix of a larger draw (counter depends only on (i >> 2, j))
    g2 = draws.gaussian_block(12, 10, 0, 50)
    assert np.array_equal(g2, draws.gaussian_block(12, 64, 0, 50)[:10])
