"""Pins for the oracle's rounding of sums of TT tensors (the remark on
sums): the rounding of sum_i w_i X^(i) is defined as the rounding of the
formal sum, and the method relies on the partial contractions of the formal
sum being the summands' own contractions stacked by rows.

  * the stacked per-summand contractions against the definition (Eq. 6):
    explicit suffix unfolding of the formal sum (built by the input
    generator's layout helper, not the oracle's) times the explicit KRP;
  * at d=2 the fixed-rank sum rounding is the range finder applied to the
    dense weighted sum of the summands' matrices;
  * summands that add up to a low-rank tensor (Z, 0.5 Z, -0.25 Z) are
    recovered exactly, and with the recompression pass the ranks are
    TT-SVD's ranks of the dense sum.
"""
import numpy as np
import pytest

import ttgen
from oracle import krp, philox, tt, ttsvd
from tests.test_oracle_krp import _explicit_krp, _qr_pos_indep, _suffix_h


@pytest.mark.parametrize("d", [2, 4])
def test_sum_partial_contractions_vs_definition(d):
    tts, w = ttgen.sum_terms(70 + d, d, 3, 2, 3, weights=[1.0, -0.5, 2.0])
    dims = [3] * d
    ell = 4
    om = krp.draw_omegas(11, dims, range(2, d + 1), 0, ell)
    stacked = krp.partial_contractions_sum(tts, om, 2)
    fs = ttgen.formal_sum(tts, w)
    for k in range(2, d + 1):
        ref = _suffix_h(fs, k) @ _explicit_krp([om[j] for j in range(k, d + 1)])
        assert stacked[k].shape == ref.shape
        assert np.allclose(stacked[k], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def test_sum_fixed_d2_is_range_finder_of_weighted_sum():
    rng = ttgen.rng_for(71)
    tts, mats = [], []
    for r in (5, 3, 4):
        a = rng.standard_normal((1, 30, r))
        b = rng.standard_normal((r, 25, 1))
        tts.append([a, b])
        mats.append(a.reshape(30, r) @ b.reshape(r, 25))
    w = [1.0, 1e-2, -3.0]
    m = sum(wi * mi for wi, mi in zip(w, mats))
    ell = 6
    y, info = krp.round_sum_fixed(tts, ell, seed=5, weights=w)
    q = _qr_pos_indep(m @ philox.gaussian_factor(5, 2, 25, 0, ell))
    assert info["ranks"] == [1, ell, 1]
    assert np.linalg.norm(tt.full(y) - q @ (q.T @ m)) < 1e-13 * np.linalg.norm(m)


def _dense_sum(tts, w):
    return sum(wi * tt.full(x) for wi, x in zip(w, tts))


def test_sum_exact_recovery_and_ttsvd_ranks():
    z = ttgen.small_random(72, 5, 4, 3)
    tts, w = [z, z, z], [1.0, 0.5, -0.25]
    ref = _dense_sum(tts, w)
    y, info = krp.round_sum_adaptive(tts, 1e-8, 2, seed=9, weights=w, recompress=1)
    assert np.linalg.norm(tt.full(y) - ref) < 1e-12 * np.linalg.norm(ref)
    assert info["ranks"] == [1, 3, 3, 3, 3, 1]
    _, sv = ttsvd.tt_svd_round(ttgen.formal_sum(tts, w), tol=1e-8)
    assert info["ranks"] == sv["ranks"]
    yf, infof = krp.round_sum_fixed(tts, 5, seed=9, weights=w)
    assert np.linalg.norm(tt.full(yf) - ref) < 1e-12 * np.linalg.norm(ref)


def test_sum_adaptive_tolerance_on_dense():
    tts, w = ttgen.sum_terms(73, 4, 5, 4, 3)
    ref = _dense_sum(tts, w)
    tol = 1e-4
    y, info = krp.round_sum_adaptive(tts, tol, 2, seed=13, weights=w)
    err = np.linalg.norm(tt.full(y) - ref) / np.linalg.norm(ref)
    # the estimator holds w.h.p.; this seed keeps every margin above 10%
    assert info["min_margin"] > 0.1
    assert err <= tol
