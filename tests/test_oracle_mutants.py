"""Planted mistakes: each test swaps one oracle routine for a plausibly
wrong version (a transposed or reversed index, a flipped sign, a dropped
factor, an off-by-one in the truncation rule) and checks that an
independent pin of the oracle then fails.  The mistakes live only in
these CPU tests; the oracle itself is unchanged afterwards."""
import numpy as np
import pytest

from oracle import krp, tt, ttsvd
from tests import test_oracle_krp as pins_krp
from tests import test_oracle_tt as pins_tt
from tests import test_oracle_ttsvd as pins_ttsvd


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_reversed_omega_rows_caught(monkeypatch):
    orig = krp.partial_contractions_rl

    def wrong(cores, om, t):
        return orig(cores, {k: v[::-1].copy() for k, v in om.items()}, t)

    monkeypatch.setattr(krp, "partial_contractions_rl", wrong)
    _fails(pins_krp.test_partial_contractions_vs_definition, 3)


def test_transposed_core_contraction_caught(monkeypatch):
    orig = krp.partial_contractions_rl

    def wrong(cores, om, t):
        # contract Omega against the rank index instead of the mode index
        sw = [np.ascontiguousarray(c.transpose(0, 2, 1)) if c.shape[1] == c.shape[2] else c
              for c in cores]
        return orig(sw, om, t)

    monkeypatch.setattr(krp, "partial_contractions_rl", wrong)
    # shapes with n_k == r_k so the transposed contraction still runs
    x = [np.random.default_rng(1).standard_normal(s) for s in [(1, 3, 3), (3, 3, 3), (3, 3, 1)]]
    om = krp.draw_omegas(7, [3, 3, 3], range(2, 4), 0, 4)
    w = krp.partial_contractions_rl(x, om, 2)
    ref = pins_krp._suffix_h(x, 2) @ pins_krp._explicit_krp([om[2], om[3]])
    assert not np.allclose(w[2], ref, rtol=1e-8)


def test_lr_reversed_omega_rows_caught(monkeypatch):
    orig = krp.partial_contractions_lr

    def wrong(cores, om, t):
        return orig(cores, {k: v[::-1].copy() for k, v in om.items()}, t)

    monkeypatch.setattr(krp, "partial_contractions_lr", wrong)
    _fails(pins_krp.test_partial_contractions_lr_vs_definition, 3)


def test_lr_krp_factor_order_caught(monkeypatch):
    def wrong(cores, om, t):
        # pairs row (a, i) of V(X_k) with Omega_k(a) * WL_{k-1}(i): the KRP
        # factors in the wrong order
        w = {1: krp.v_unf(cores[0]).T @ om[1]}
        for k in range(2, t + 1):
            w[k] = krp.v_unf(cores[k - 1]).T @ krp.khatri_rao(om[k], w[k - 1])
        return w

    monkeypatch.setattr(krp, "partial_contractions_lr", wrong)
    _fails(pins_krp.test_partial_contractions_lr_d2_is_gemm_and_meets_rl)


def test_residual_sign_flip_caught(monkeypatch):
    def wrong(sk, z, q, k, b):
        need = q.shape[1] + b
        if sk.ncols(k + 1) < need:
            sk.extend(k + 1, need - sk.ncols(k + 1))
        s = z @ sk.w[k + 1][:, q.shape[1]:need]
        return s + q @ (q.T @ s)

    monkeypatch.setattr(krp, "generate_residual_sketch", wrong)
    _fails(pins_krp.test_adaptive_d2_is_adaptive_range_finder)


def test_norm_estimate_missing_sqrt_caught(monkeypatch):
    def wrong(core1, w2):
        return float(np.linalg.norm(tt.v_unf(core1) @ w2))

    monkeypatch.setattr(krp, "norm_estimate", wrong)
    _fails(pins_krp.test_norm_estimate_unbiased_over_seeds)


def test_recompress_wrong_factor_caught(monkeypatch):
    def wrong(cores, tau=None, ranks=None):
        ys = [np.array(c, copy=True) for c in cores]
        d = len(ys)
        for k in range(d - 1, 0, -1):
            r0, n, r1 = ys[k].shape
            q, r = np.linalg.qr(tt.h_unf(ys[k]).T)
            u, s, vt = np.linalg.svd(r.T)
            t = ttsvd.truncation_rank(s, tau) if tau is not None else max(1, min(int(ranks[k]), s.size))
            ys[k] = (vt[:t, :] @ q.T).reshape(t, n, r1)
            p0, pn, _ = ys[k - 1].shape
            # drops the singular values when folding into core k-1
            ys[k - 1] = (tt.v_unf(ys[k - 1]) @ u[:, :t]).reshape(p0, pn, t)
        return ys

    monkeypatch.setattr(krp, "recompress_rl", wrong)
    _fails(pins_krp.test_recompress_d2_is_truncated_svd)


def test_truncation_off_by_one_caught(monkeypatch):
    orig = ttsvd.truncation_rank

    def wrong(s, tau):
        return min(orig(s, tau) + 1, np.asarray(s).size)

    monkeypatch.setattr(ttsvd, "truncation_rank", wrong)
    _fails(pins_ttsvd.test_truncation_rank_rule)


def test_diff_norm_sign_caught(monkeypatch):
    def wrong(a, b):
        return tt.norm(tt.formal_sum([a, b], [1.0, 1.0]))

    monkeypatch.setattr(tt, "diff_norm", wrong)
    _fails(pins_tt.test_diff_norm_matches_dense_for_unrelated_tensors)


def test_fixed_nonorthonormal_basis_caught(monkeypatch):
    """A QR whose Q columns are not unit length."""
    orig_qr = krp.qr_pos

    def wrong(s):
        q = orig_qr(s)
        return q * (1.0 + 1e-3 * np.arange(q.shape[1]))[None, :]

    monkeypatch.setattr(krp, "qr_pos", wrong)
    _fails(pins_krp.test_fixed_d2_is_halko_range_finder)


def test_sum_contractions_summand_order_caught(monkeypatch):
    from tests import test_oracle_sum as pins_sum
    orig = krp.partial_contractions_rl

    def wrong(tts, om, t):
        ws = [orig(x, om, t) for x in reversed(tts)]
        return {k: np.concatenate([w[k] for w in ws], axis=0) for k in ws[0]}

    monkeypatch.setattr(krp, "partial_contractions_sum", wrong)
    _fails(pins_sum.test_sum_partial_contractions_vs_definition, 4)


def test_sum_weight_applied_twice_caught(monkeypatch):
    """Each weight applied on both the first and the last core."""
    from tests import test_oracle_sum as pins_sum
    orig = tt.formal_sum

    def wrong(tts, weights=None):
        if weights is None:
            return orig(tts)
        return orig(tts, [w * w for w in weights])

    monkeypatch.setattr(tt, "formal_sum", wrong)
    _fails(pins_sum.test_sum_fixed_d2_is_range_finder_of_weighted_sum)


def test_threshold_without_sqrt_d_minus_1_caught(monkeypatch):
    """The whole accuracy given to every bond instead of eps/sqrt(d-1)."""
    monkeypatch.setattr(krp, "modewise_threshold", lambda tol, nrmx, d: tol * nrmx)
    _fails(pins_krp.test_adaptive_threshold_spreads_tolerance_over_bonds)


def test_ttsvd_threshold_without_sqrt_d_minus_1_caught(monkeypatch):
    monkeypatch.setattr(ttsvd, "bond_threshold", lambda tol, norm, d: tol * norm)
    _fails(pins_krp.test_adaptive_threshold_spreads_tolerance_over_bonds)


def test_initial_sketch_from_smallest_rank_caught(monkeypatch):
    """r0 from the smallest interior rank instead of the largest."""
    import math

    def wrong(cores, f_init):
        return int(math.ceil(f_init * min(c.shape[2] for c in cores[:-1])))

    monkeypatch.setattr(krp, "initial_sketch_columns", wrong)
    _fails(pins_krp.test_initial_sketch_uses_largest_rank)
