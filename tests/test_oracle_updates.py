"""Pins for the oracle's sketch updates (Section 5), no GPU: each update is checked against a
from-scratch product of the pinned explicit sketching matrix with the changed matrix."""
import math

import numpy as np
import pytest

from oracle import draws, operators, updates

KINDS = ["srht", "srdct", "sparse", "gauss"]


def explicit_sa(kind, a, s, seed):
    return operators.sketch(a, kind, s, seed, zeta=8, gauss_dtype="bf16")


@pytest.mark.parametrize("kind", KINDS)
def test_row_downdate_equals_sketch_without_the_row(kind):
    """Algorithm 3: removing rows j gives the sketch of A with those rows taken out (the columns
    of S that remain keep their indices, so this is S times A with the rows zeroed)."""
    rng = np.random.default_rng(3)
    m, n, s, seed = 3000, 7, 64, 11
    a = rng.standard_normal((m, n))
    if kind == "gauss":
        a = operators.round_to(a, "bf16")
    sa = explicit_sa(kind, a, s, seed)
    rows = [0, 17, 2999, 1024]
    got = updates.update_rows(sa, kind, seed, m, rows, a[rows], [-1] * len(rows))
    a2 = a.copy()
    a2[rows] = 0.0
    ref = explicit_sa(kind, a2, s, seed)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_gaussian_row_update_equals_sketch_of_longer_matrix():
    """Algorithm 2 for the Gaussian kind: S_r = [G | g] / sqrt(s) is the sketch of m + 1 rows."""
    rng = np.random.default_rng(4)
    m, n, s, seed = 2000, 5, 40, 12
    a = operators.round_to(rng.standard_normal((m + 2, n)), "bf16")
    sa = explicit_sa("gauss", a[:m], s, seed)
    got = updates.update_rows(sa, "gauss", seed, m, [m, m + 1], a[m:], [1, 1])
    ref = explicit_sa("gauss", a, s, seed)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("kind", ["srht", "srdct", "sparse"])
def test_non_gaussian_row_update_appends_a_gaussian_column(kind):
    """Section 5.3: the updated sketching matrix is [S | g / sqrt(s)] with g standard normal."""
    rng = np.random.default_rng(5)
    m, n, s, seed = 1500, 6, 48, 13
    a = rng.standard_normal((m + 1, n))
    S = operators.explicit(kind, seed, m, s, zeta=8)
    g = draws.gaussian_block(seed, s, m, m + 1) / math.sqrt(s)
    ref = np.hstack([S, g]) @ a
    got = updates.update_rows(S @ a[:m], kind, seed, m, [m], a[m:], [1])
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    # the appended column has the Gaussian kind's unrounded entries: mean 0, variance 1 / s
    cols = np.stack([updates.sketch_column(kind, seed, m, s, j) for j in range(m, m + 400)])
    assert abs(cols.mean()) < 4 / math.sqrt(cols.size) / math.sqrt(s)
    assert abs(cols.var() * s - 1) < 0.05


@pytest.mark.parametrize("kind", KINDS)
def test_downdate_undoes_update(kind):
    rng = np.random.default_rng(6)
    m, n, s, seed = 1200, 4, 32, 14
    sa = rng.standard_normal((s, n))
    row = rng.standard_normal((1, n))
    if kind == "gauss":
        row = operators.round_to(row, "bf16")
    for j in (5, m + 3):
        up = updates.update_rows(sa, kind, seed, m, [j], row, [1])
        back = updates.update_rows(up, kind, seed, m, [j], row, [-1])
        assert np.abs(back - sa).max() < 1e-13 * np.abs(sa).max()


def test_column_update_is_the_sketch_of_the_new_column():
    """Section 5: adding a column appends S a_new to SA; dropping one drops it."""
    rng = np.random.default_rng(7)
    m, s, seed = 2500, 30, 15
    a = rng.standard_normal((m, 9))
    for kind in ("srht", "srdct", "sparse"):
        whole = explicit_sa(kind, a, s, seed)
        parts = np.hstack([explicit_sa(kind, a[:, :8], s, seed), explicit_sa(kind, a[:, 8:], s, seed)])
        assert np.abs(whole - parts).max() < 1e-12 * np.abs(whole).max()
