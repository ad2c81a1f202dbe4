"""Pins for the oracle's AAA loop with sketch reuse (Section 6), no GPU."""
import numpy as np

from oracle import aaa


def samples(m, seed=0):
    z = np.sort(np.random.default_rng(seed).uniform(-1, 1, m))
    return z, np.tanh(50 * z)


def test_orthogonal_sketch_takes_the_plain_support_points():
    """s = m = m_p: the Hadamard sketch is orthogonal, so the sketched Loewner matrix has the
    right singular vectors of the Loewner matrix itself (LAPACK SVD in the plain loop)."""
    z, f = samples(1024)
    sp, wp, hp = aaa.aaa(z, f, 24, 1e-10, plain=True)
    ss, ws, hs = aaa.aaa(z, f, 24, 1e-10, kind="srht", s=1024, seed=3)
    assert ss == sp and len(sp) == 21
    assert np.allclose(hs, hp, rtol=1e-6, atol=1e-12)


def test_interpolates_at_support_points_and_converges():
    z, f = samples(4000, seed=1)
    sup, w, hist = aaa.aaa(z, f, 60, 1e-11, kind="sparse", s=120, seed=4)
    assert hist[-1] <= 1e-11 * np.abs(f).max() and len(sup) < 60
    # the barycentric form interpolates: evaluating it just off a support point gives f there
    zj = z[sup[3]] + 1e-12
    C = 1.0 / (zj - z[sup])
    assert abs((C @ (w * f[sup])) / (C @ w) - f[sup[3]]) < 1e-9
    assert len(set(sup)) == len(sup)


def test_sketched_loop_matches_plain_error_level():
    """A 4x-oversampled sketch reaches the same accuracy with about the same degree."""
    z, f = samples(6000, seed=2)
    sp, _, hp = aaa.aaa(z, f, 60, 1e-10, plain=True)
    for kind in ("srht", "srdct", "sparse"):
        ss, _, hs = aaa.aaa(z, f, 60, 1e-10, kind=kind, s=240, seed=5)
        assert hs[-1] <= 1e-10 and abs(len(ss) - len(sp)) <= 3, (kind, len(ss), len(sp))
