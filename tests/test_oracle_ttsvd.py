"""Pins for deterministic TT-rounding: d=2 is the truncated SVD
(Eckart-Young), Oseledets' error bound from the dense unfoldings, exact rank
recovery on the C1 workload, orthonormality."""
import numpy as np

import ttgen
from oracle import tt, ttsvd


def test_truncation_rank_rule():
    s = np.array([4.0, 3.0, 1e-3, 1e-4])
    assert ttsvd.truncation_rank(s, 1e-3 * 1.01) == 2      # tail sqrt(1e-6+1e-8) <= tau
    assert ttsvd.truncation_rank(s, 1e-3) == 3             # tail 1.005e-3 > 1e-3
    assert ttsvd.truncation_rank(s, 1e-4) == 3             # tail 1e-4 <= 1e-4 (ties stop)
    assert ttsvd.truncation_rank(s, 0.0) == 4
    assert ttsvd.truncation_rank(s, 1e9) == 1              # never below 1


def test_d2_is_truncated_svd():
    rng = ttgen.rng_for(21)
    a = rng.standard_normal((30, 12)) @ np.diag(10.0 ** -np.arange(12)) @ rng.standard_normal((12, 25))
    x = [a.reshape(1, 30, 25), np.eye(25).reshape(25, 25, 1)]
    tol = 1e-5
    y, info = ttsvd.tt_svd_round(x, tol=tol)
    u, s, vt = np.linalg.svd(a)
    t = ttsvd.truncation_rank(s, tol * np.linalg.norm(a))
    assert info["ranks"] == [1, t, 1]
    best = (u[:, :t] * s[:t]) @ vt[:t]
    assert np.linalg.norm(tt.full(y) - best) < 1e-12 * np.linalg.norm(a)


def test_c1_recovers_true_ranks():
    x = ttgen.c1()
    y, info = ttsvd.tt_svd_round(x, tol=1e-8)
    assert info["ranks"] == [1, 10, 10, 10, 10, 10, 1]
    f = tt.full(x)
    assert np.linalg.norm(f - tt.full(y)) <= 1e-13 * np.linalg.norm(f)
    assert tt.left_orth_defect(y) < 1e-13


def test_oseledets_error_bound_and_tolerance():
    """||X - Y||^2 <= sum_k (tail of the dense unfolding X_(1:k))^2 for the
    fixed-rank mode, and ||X-Y|| <= eps ||X|| for the tolerance mode."""
    x = ttgen.small_random(22, 5, 4, 6)
    f = tt.full(x)
    ranks = [1, 3, 4, 3, 2, 1]
    y, _ = ttsvd.tt_svd_round(x, ranks=ranks)
    bound = 0.0
    for k in range(1, 5):
        s = np.linalg.svd(f.reshape(int(np.prod(f.shape[:k])), -1), compute_uv=False)
        bound += np.sum(s[ranks[k]:] ** 2)
    err = np.linalg.norm(f - tt.full(y))
    assert err ** 2 <= bound * (1 + 1e-10)
    for eps in (1e-1, 1e-2, 1e-3):
        y, _ = ttsvd.tt_svd_round(x, tol=eps)
        assert np.linalg.norm(f - tt.full(y)) <= eps * np.linalg.norm(f) * (1 + 1e-12)
