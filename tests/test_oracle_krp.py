"""Pins for the oracle's KRP rounding:
  * partial contractions against the definition (Eq. 6): the explicit
    suffix unfolding H(X_{k:d}) times the explicit Khatri-Rao product, and
    the left-to-right ones against the explicit prefix unfolding V(X_{1:k});
  * fixed rank at d=2 is Halko's randomized range finder; exact recovery
    when the sketch is at least the true rank (C1);
  * adaptive at d=2 is the adaptive range finder with the sketched
    residual estimate, written here at the matrix level;
  * the error identity ||X - Y||^2 = sum_k ||(I - Q_k Q_k^T) Z_k H(X_{k+1:d})||^2;
  * unbiasedness of the KRP Frobenius estimator (Theorem 1) with the
    closed-form variance (3^m - 1)||a||^4 for a Kronecker-structured row;
  * the recompression pass: d=2 is the truncated SVD; on C1 it lands on
    TT-SVD's exact ranks.
"""
import math

import numpy as np
import pytest

import ttgen
from oracle import krp, philox, tt, ttsvd


def _qr_pos_indep(s):
    q, r = np.linalg.qr(s)
    d = np.where(np.diag(r) < 0, -1.0, 1.0)
    return q * d


def _suffix_h(cores, k):
    """Explicit H(X_{k:d}) (1-based k): r_{k-1} x prod(n_k..n_d), i_d fastest."""
    acc = cores[k - 1].reshape(cores[k - 1].shape[0], -1)
    for c in cores[k:]:
        r0, n, r1 = c.shape
        acc = (acc.reshape(-1, r0) @ c.reshape(r0, n * r1)).reshape(acc.shape[0], -1)
    return acc.reshape(cores[k - 1].shape[0], -1)


def _explicit_krp(mats):
    """Omega_k (.) ... (.) Omega_d with the last factor fastest."""
    out = mats[0]
    for m in mats[1:]:
        out = np.einsum('ij,kj->ikj', out, m).reshape(-1, m.shape[1])
    return out


def test_khatri_rao_definition():
    a = np.arange(6.0).reshape(3, 2)
    b = np.arange(8.0).reshape(4, 2) + 1
    kr = krp.khatri_rao(a, b)
    for j in range(2):
        assert np.array_equal(kr[:, j], np.kron(a[:, j], b[:, j]))


@pytest.mark.parametrize("d", [2, 3, 5])
def test_partial_contractions_vs_definition(d):
    dims = [3, 4, 2, 3, 2][:d]
    ranks = [2, 3, 4, 2][:d - 1]
    x = ttgen.small_random(30 + d, d, dims, ranks)
    ell = 5
    om = krp.draw_omegas(99, dims, range(2, d + 1), 0, ell)
    w = krp.partial_contractions_rl(x, om, 2)
    for k in range(2, d + 1):
        ref = _suffix_h(x, k) @ _explicit_krp([om[j] for j in range(k, d + 1)])
        assert np.allclose(w[k], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
        # index formula, contracting b first (the other order)
        if k < d:
            u = np.einsum('aib,bj->aij', x[k - 1], w[k + 1])
            alt = np.einsum('aij,ij->aj', u, om[k])
            assert np.allclose(w[k], alt, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def _prefix_v(cores, k):
    """Explicit V(X_{1:k}) (1-based k): prod(n_1..n_k) x r_k, i_k fastest."""
    acc = cores[0].reshape(-1, cores[0].shape[2])
    for c in cores[1:k]:
        r0, n, r1 = c.shape
        acc = (acc @ c.reshape(r0, n * r1)).reshape(-1, r1)
    return acc


@pytest.mark.parametrize("d", [2, 3, 5])
def test_partial_contractions_lr_vs_definition(d):
    """WL_k = V(X_{1:k})^T (Omega_1 (.) ... (.) Omega_k) with the row order of
    the prefix unfolding (the last mode fastest), formed explicitly."""
    dims = [3, 4, 2, 3, 2][:d]
    ranks = [2, 3, 4, 2][:d - 1]
    x = ttgen.small_random(60 + d, d, dims, ranks)
    ell = 5
    om = krp.draw_omegas(98, dims, range(1, d + 1), 0, ell)
    w = krp.partial_contractions_lr(x, om, d)
    for k in range(1, d + 1):
        ref = _prefix_v(x, k).T @ _explicit_krp([om[j] for j in range(1, k + 1)])
        assert w[k].shape == (x[k - 1].shape[2], ell)
        assert np.allclose(w[k], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def test_partial_contractions_lr_d2_is_gemm_and_meets_rl():
    """d=2: WL_1 = V(X_1)^T Omega_1.  For any d the full contractions agree:
    WL_d (1 x l) from the left and W_1 (1 x l) from the right are both
    vec(X)^T (Omega_1 (.) ... (.) Omega_d)."""
    x = ttgen.small_random(71, 2, [6, 5], [4])
    om = krp.draw_omegas(3, [6, 5], range(1, 3), 0, 7)
    w = krp.partial_contractions_lr(x, om, 1)
    assert np.allclose(w[1], x[0].reshape(6, 4).T @ om[1], rtol=1e-14, atol=1e-14)
    for d, dims, ranks in [(3, [3, 4, 5], [2, 3]), (4, [2, 3, 2, 3], [3, 4, 2])]:
        x = ttgen.small_random(72 + d, d, dims, ranks)
        om = krp.draw_omegas(4, dims, range(1, d + 1), 0, 6)
        left = krp.partial_contractions_lr(x, om, d)[d]
        right = krp.partial_contractions_rl(x, om, 2)[2]
        # W_1 = H(X_1) [Omega_1 (.) W_2] from the right
        full_r = np.einsum('aib,ij,bj->aj', x[0], om[1], right)
        assert np.allclose(left, full_r, rtol=1e-12, atol=1e-12 * np.abs(full_r).max())
        f = tt.full(x).reshape(-1)
        ref = f @ _explicit_krp([om[j] for j in range(1, d + 1)])
        assert np.allclose(left[0], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_partial_contractions_chunk_invariant():
    x = ttgen.small_random(40, 4, 3, 3)
    dims = [3] * 4
    full = krp.partial_contractions_rl(x, krp.draw_omegas(5, dims, range(2, 5), 0, 9), 2)
    a = krp.partial_contractions_rl(x, krp.draw_omegas(5, dims, range(2, 5), 0, 4), 2)
    b = krp.partial_contractions_rl(x, krp.draw_omegas(5, dims, range(3, 5), 4, 5), 3)
    for k in (3, 4):
        assert np.array_equal(full[k], np.concatenate([a[k], b[k]], axis=1))


def test_fixed_d2_is_halko_range_finder():
    rng = ttgen.rng_for(50)
    r = 12
    x = [rng.standard_normal((1, 40, r)), rng.standard_normal((r, 30, 1))]
    xm = x[0].reshape(40, r) @ x[1].reshape(r, 30)
    ell = 7
    y, info = krp.round_fixed(x, ell, seed=3)
    om = philox.gaussian_factor(3, 2, 30, 0, ell)
    q = _qr_pos_indep(xm @ om)
    ref = q @ (q.T @ xm)
    assert info["ranks"] == [1, ell, 1]
    assert np.linalg.norm(tt.full(y) - ref) < 1e-13 * np.linalg.norm(xm)


@pytest.mark.parametrize("ell", [10, 12])
def test_fixed_exact_recovery_c1(ell):
    x = ttgen.c1()
    y, info = krp.round_fixed(x, ell, seed=42)
    # l_k = min(ell, l_{k-1} n_k, r_k)
    assert info["sketch_ranks"] == [1, 10] + [ell] * 4 + [1]
    f = tt.full(x)
    assert np.linalg.norm(f - tt.full(y)) < 1e-13 * np.linalg.norm(f)
    assert tt.left_orth_defect(y) < 1e-13
    assert tt.rel_err(x, y) < 1e-13


def test_fixed_with_truncation_lands_on_targets():
    x = ttgen.c1()
    y, info = krp.round_fixed(x, 12, seed=42, target_ranks=[1] + [10] * 5 + [1])
    assert info["ranks"] == [1, 10, 10, 10, 10, 10, 1]
    assert tt.rel_err(x, y) < 1e-13
    assert tt.right_orth_defect(y) < 1e-13


def _arf_matrix(xm, seed, tol_abs, f_init, b, rbar):
    """Adaptive randomized range finder with the sketched residual
    estimate, written for a plain matrix (the d=2 special case).  rbar is
    the rank cap, min of the sizes of V(Y_1) as the paper defines it."""
    m, n = xm.shape
    binit = max(1, math.ceil(f_init * rbar))
    q = _qr_pos_indep(xm @ philox.gaussian_factor(seed, 2, n, 0, binit))
    while q.shape[1] < rbar:
        bb = min(b, rbar - q.shape[1])
        s = xm @ philox.gaussian_factor(seed, 2, n, q.shape[1], bb)
        s = s - q @ (q.T @ s)
        if not np.linalg.norm(s) / math.sqrt(bb) > tol_abs:
            break
        qn = _qr_pos_indep(s)
        qn = _qr_pos_indep(qn - q @ (q.T @ qn))
        q = np.hstack([q, qn])
    return q


def test_adaptive_d2_is_adaptive_range_finder():
    rng = ttgen.rng_for(60)
    r = 40
    a = rng.standard_normal((50, r)) * (10.0 ** (-np.arange(r) / 4.0))[None, :]
    x = [a.reshape(1, 50, r), rng.standard_normal((r, 45, 1))]
    xm = tt.full(x)
    nrm = np.linalg.norm(xm)
    tol = 1e-4
    y, info = krp.round_adaptive(x, tol, ell_block=3, seed=8, nrmx=nrm)
    q = _arf_matrix(xm, 8, tol * nrm, 0.1, 3, rbar=min(50, r))
    assert info["ranks"] == [1, q.shape[1], 1]
    assert np.linalg.norm(tt.full(y) - q @ (q.T @ xm)) < 1e-12 * nrm


def _residual_norms(x, kept):
    """||(I - Q_k Q_k^T) Z_k H(X_{k+1:d})||_F for each mode, exactly, using
    the right-to-left orthogonalized suffix."""
    out = []
    for k, (z, q) in enumerate(kept, start=1):
        suf = tt.orthogonalize_rl([c.copy() for c in x[k:]])
        h = suf[0].reshape(suf[0].shape[0], -1)
        a = (z - q @ (q.T @ z)) @ h
        out.append(np.linalg.norm(a))
    return np.array(out)


def test_adaptive_error_identity_and_tolerance():
    x = ttgen.c1()
    nrm = tt.norm(x)
    tol = 1e-8
    y, info = krp.round_adaptive(x, tol, ell_block=4, seed=42, nrmx=nrm, keep=True)
    res = _residual_norms(x, info["ZQ"])
    err = tt.diff_norm(x, y)
    assert err ** 2 == pytest.approx(np.sum(res ** 2), rel=1e-6, abs=(1e-14 * nrm) ** 2)
    assert err <= tol * nrm


def test_adaptive_error_identity_decaying():
    """A TT whose bond spectra decay: the sum of the exact per-mode
    residuals reproduces ||X - Y||^2 for every seed and block size, and with
    6-column blocks the error meets the tolerance (tiny blocks give a noisy
    estimate and exceed it now and then, as the paper also observes)."""
    x = ttgen.c3(seed=7, d=5, n=6, r=20, noise_r=5, decay=3.0)
    nrm = tt.norm(x)
    tol = 1e-4
    for blk in (2, 6):
        for seed in range(6):
            y, info = krp.round_adaptive(x, tol, ell_block=blk, seed=seed, nrmx=nrm, keep=True)
            res = _residual_norms(x, info["ZQ"])
            err = tt.diff_norm(x, y)
            assert err ** 2 == pytest.approx(np.sum(res ** 2), rel=1e-6)
            assert tt.left_orth_defect(y) < 1e-12
            if blk == 6:
                assert err <= tol * nrm


def test_krp_estimator_unbiased_kronecker_row():
    """Theorem 1: E[(a^T w)^2] = ||a||^2 with Var = (3^m - 1)||a||^4 when
    a = a_1 (x) ... (x) a_m and w = w_1 (x) ... (x) w_m Gaussian."""
    rng = ttgen.rng_for(70)
    for m in (2, 3):
        facs = [rng.standard_normal(4) for _ in range(m)]
        a = facs[0]
        for f in facs[1:]:
            a = np.kron(a, f)
        L = 20000
        oms = [philox.gaussian_factor(123, j + 2, 4, 0, L) for j in range(m)]
        w = oms[0]
        for o in oms[1:]:
            w = np.einsum('ij,kj->ikj', w, o).reshape(-1, L)
        vals = (a @ w) ** 2
        na2 = float(a @ a)
        var = (3 ** m - 1) * na2 ** 2
        assert abs(vals.mean() - na2) < 5 * math.sqrt(var / L)
        if m == 2:
            assert vals.var() == pytest.approx(var, rel=0.5)


def test_norm_estimate_unbiased_over_seeds():
    """Remark 1: (1/r) ||V(X_1) W_2||_F^2 is unbiased for ||X||^2."""
    x = ttgen.small_random(80, 4, 3, 2)
    nrm2 = tt.norm(x) ** 2
    dims = [3] * 4
    vals = []
    for seed in range(600):
        w = krp.partial_contractions_rl(x, krp.draw_omegas(seed, dims, range(2, 5), 0, 2), 2)
        vals.append(krp.norm_estimate(x[0], w[2]) ** 2)
    vals = np.array(vals)
    assert abs(vals.mean() - nrm2) < 5 * vals.std() / math.sqrt(len(vals))


def test_recompress_d2_is_truncated_svd():
    rng = ttgen.rng_for(90)
    q, _ = np.linalg.qr(rng.standard_normal((20, 8)))
    x = [q.reshape(1, 20, 8), (rng.standard_normal((8, 15)) * (2.0 ** -np.arange(8))[:, None]).reshape(8, 15, 1)]
    xm = tt.full(x)
    y = krp.recompress_rl(x, ranks=[1, 3, 1])
    u, s, vt = np.linalg.svd(xm)
    assert np.linalg.norm(tt.full(y) - (u[:, :3] * s[:3]) @ vt[:3]) < 1e-13 * np.linalg.norm(xm)


def test_adaptive_recompress_matches_ttsvd_ranks_c1():
    x = ttgen.c1()
    y, info = krp.round_adaptive(x, 1e-8, ell_block=4, seed=42, recompress=1)
    ys, sinfo = ttsvd.tt_svd_round(x, tol=1e-8)
    assert info["ranks"] == sinfo["ranks"] == [1, 10, 10, 10, 10, 10, 1]
    assert tt.rel_err(x, y) < 1e-13
    assert tt.right_orth_defect(y) < 1e-13


def _orthogonal_rank_one_sum(rng, d, n, sig):
    """X = sum_j sig_j u_1^(j) (x) ... (x) u_d^(j) with the u_k^(j), j = 1..r,
    orthonormal in every mode k.  The left factors u_1^(j) (x) ... (x)
    u_k^(j) of any unfolding X_(1:k) are then orthonormal, and so are the
    right ones, so every bond's singular values are exactly sig (a closed
    form).  As a TT: first core U_1 diag(sig), diagonal middle cores
    X_k(j, :, j) = u_k^(j), last core U_d^T; all ranks r."""
    r = len(sig)
    us = [np.linalg.qr(rng.standard_normal((n, r)))[0] for _ in range(d)]
    cores = [(us[0] * np.asarray(sig)[None, :]).reshape(1, n, r)]
    for k in range(1, d - 1):
        c = np.zeros((r, n, r))
        for j in range(r):
            c[j, :, j] = us[k][:, j]
        cores.append(c)
    cores.append(np.ascontiguousarray(us[d - 1].T).reshape(r, n, 1))
    return cores


def test_orthogonal_rank_one_sum_has_known_bond_spectra():
    """The construction above, checked by brute force: the SVD of every
    dense unfolding is sig."""
    sig = np.array([1.0, 0.3, 0.05, 2e-3, 1e-4])
    x = _orthogonal_rank_one_sum(ttgen.rng_for(95), 4, 6, sig)
    f = tt.full(x)
    for k in range(1, 4):
        s = np.linalg.svd(f.reshape(6 ** k, -1), compute_uv=False)
        assert np.allclose(s[:5], sig, rtol=1e-12, atol=1e-14)
        assert np.all(s[5:] < 1e-13)


# d = 5 (so sqrt(d-1) = 2) with bond spectra 10^-(j-1), j = 1..8, and
# eps = 1.5e-3.  By hand: ||X|| = 1.00504, tau = eps ||X|| / 2 = 7.54e-4;
# the tails sqrt(sum_{j>t} sig_j^2) are 1.005e-3 at t = 3 (> tau) and
# 1.005e-4 at t = 4 (<= tau), so every bond keeps 4 terms.  The undivided
# threshold eps ||X|| = 1.51e-3 would already accept t = 3.
_SIG_D5 = 10.0 ** -np.arange(8)
_EPS_D5 = 1.5e-3
_RANKS_D5 = [1, 4, 4, 4, 4, 1]


def test_adaptive_threshold_spreads_tolerance_over_bonds():
    """Sec. 3.3: tau = eps ||X|| / sqrt(d-1).  With blocks as wide as the
    ranks the sweep captures X exactly (sketch ranks 8), so the Remark 2
    pass truncates the exact spectra with the tail rule at tau: the ranks
    must be the hand-computed ones above, and TT-SVD (Sec. 2.3) must land
    on the same ranks."""
    x = _orthogonal_rank_one_sum(ttgen.rng_for(96), 5, 10, _SIG_D5)
    nrm = math.sqrt(float(np.sum(_SIG_D5 ** 2)))
    y, info = krp.round_adaptive(x, _EPS_D5, ell_block=8, seed=3, nrmx=nrm, recompress=1)
    assert info["sketch_ranks"] == [1, 8, 8, 8, 8, 1]
    assert info["ranks"] == _RANKS_D5
    assert tt.rel_err(x, y) <= _EPS_D5
    ys, sinfo = ttsvd.tt_svd_round(x, tol=_EPS_D5)
    assert sinfo["ranks"] == _RANKS_D5


def test_initial_sketch_uses_largest_rank():
    """Sec. 3.3 (first step of the adaptive algorithm) and Remark 1: the
    Gaussian factors start with r = ceil(f_init max_j r_j) columns and the
    norm estimate uses all of them.  Ranks (1, 6, 23, 6, 1): by hand
    r = ceil(0.1 * 23) = 3 (the smallest rank would give 1).  The estimate
    must equal ||V(X_1) W_2||_F / sqrt(3) with W_2's three columns formed
    from the definition (explicit suffix unfolding times explicit KRP)."""
    dims = [6, 8, 8, 6]
    x = ttgen.small_random(97, 4, dims, [6, 23, 6])
    assert tt.ranks_of(x) == [1, 6, 23, 6, 1]
    y, info = krp.round_adaptive(x, 1e-3, 4, seed=5)
    assert info["r0"] == 3
    oms = [philox.gaussian_factor(5, j, dims[j - 1], 0, 3) for j in range(2, 5)]
    w2 = _suffix_h(x, 2) @ _explicit_krp(oms)
    est = np.linalg.norm(x[0].reshape(6, 6) @ w2) / math.sqrt(3)
    assert info["nrmx"] == pytest.approx(est, rel=1e-12)
