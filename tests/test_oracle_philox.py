"""Pins for the oracle's generator: published Philox4x32-10 known-answer
vectors, Gaussian moments / KS, and column addressability."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import philox

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def load_kat():
    rows = []
    with open(GOLD) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_kat_vectors():
    rows = load_kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        got = philox.philox4x32_10(np.array(ctr, dtype=np.uint32), np.array(key, dtype=np.uint32))
        assert [int(x) for x in got] == out


def test_kat_vectors_batched():
    rows = load_kat()
    ctr = np.array([r[0] for r in rows], dtype=np.uint32)
    key = np.array([r[1] for r in rows], dtype=np.uint32)
    got = philox.philox4x32_10(ctr, key)
    assert got.tolist() == [r[2] for r in rows]


def test_gaussian_moments_and_ks():
    om = philox.gaussian_factor(seed=7, mode=3, n=1001, col0=0, ncols=200).ravel()
    m = om.size
    assert abs(om.mean()) < 5.0 / np.sqrt(m)
    assert abs(om.var() - 1.0) < 5.0 * np.sqrt(2.0 / m)
    assert abs(np.mean(om ** 4) - 3.0) < 5.0 * np.sqrt(96.0 / m)
    assert stats.kstest(om, "norm").pvalue > 1e-4


def test_column_addressable_and_independent_of_chunking():
    a = philox.gaussian_factor(11, 2, 17, 0, 10)
    b = np.concatenate([philox.gaussian_factor(11, 2, 17, 0, 4),
                        philox.gaussian_factor(11, 2, 17, 4, 6)], axis=1)
    assert np.array_equal(a, b)
    # odd n: rows are the prefix of the n+1 case
    c = philox.gaussian_factor(11, 2, 18, 0, 10)
    assert np.array_equal(a, c[:17])


def test_modes_and_seeds_differ():
    a = philox.gaussian_factor(11, 2, 8, 0, 8)
    b = philox.gaussian_factor(11, 3, 8, 0, 8)
    c = philox.gaussian_factor(12, 2, 8, 0, 8)
    assert not np.allclose(a, b) and not np.allclose(a, c)
    # 64-bit seeds use both key words
    d = philox.gaussian_factor((1 << 32) + 11, 2, 8, 0, 8)
    assert not np.allclose(a, d)


def test_box_muller_pairs_from_one_counter():
    """Rows 2p and 2p+1 come from one Philox call: recompute by hand."""
    seed, mode, col = 5, 4, 3
    om = philox.gaussian_factor(seed, mode, 4, col, 1)
    w = philox.philox4x32_10(np.array([1, col, mode, philox.OMEGA_TAG], dtype=np.uint32),
                             np.array([seed, 0], dtype=np.uint32))
    u1 = ((int(w[0]) * 2 ** 32 + int(w[1])) // 2 ** 11 + 0.5) / 2.0 ** 53
    u2 = ((int(w[2]) * 2 ** 32 + int(w[3])) // 2 ** 11 + 0.5) / 2.0 ** 53
    rad = np.sqrt(-2 * np.log(u1))
    assert om[2, 0] == pytest.approx(rad * np.cos(2 * np.pi * u2), rel=1e-14, abs=1e-15)
    assert om[3, 0] == pytest.approx(rad * np.sin(2 * np.pi * u2), rel=1e-14, abs=1e-15)
