"""GPU kernel parity against the CPU oracle: the device Philox generator
(bitwise on the known-answer vectors and on the oracle's words), the
Gaussian mode factors, the KRP partial contractions in FP64 and FP32, and
the thin QR."""
import numpy as np
import pytest

import ttgen
from oracle import krp, philox
from tests.gpu_helpers import say, to_dev
from tests.test_oracle_philox import load_kat

pytestmark = pytest.mark.gpu


def test_device_info(lib):
    import torch
    p = torch.cuda.get_device_properties(0)
    say("device:", p.name, getattr(p, "gcnArchName", "?"), "CUs", p.multi_processor_count)


def test_philox_device_kat(lib):
    import torch
    rows = load_kat()
    ctr = torch.tensor(np.array([r[0] for r in rows], dtype=np.uint32).view(np.int32), device="cuda")
    key = torch.tensor(np.array([r[1] for r in rows], dtype=np.uint32).view(np.int32), device="cuda")
    out = lib.philox4x32_10(ctr, key).cpu().numpy().view(np.uint32)
    assert out.tolist() == [r[2] for r in rows]


def test_philox_device_matches_oracle_words(lib):
    import torch
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2 ** 32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(4096, 2), dtype=np.uint64).astype(np.uint32)
    got = lib.philox4x32_10(torch.tensor(ctr.view(np.int32), device="cuda"),
                            torch.tensor(key.view(np.int32), device="cuda")).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, philox.philox4x32_10(ctr, key))


@pytest.mark.parametrize("seed,mode,n,col0,ncols", [(42, 2, 10, 0, 12), (7, 5, 1, 3, 5),
                                                    (2 ** 40 + 3, 20, 64, 17, 60), (1, 3, 257, 0, 64)])
def test_gaussian_factor_matches_oracle(lib, seed, mode, n, col0, ncols):
    got = lib.gaussian_factor(seed, mode, n, col0, ncols).cpu().numpy()
    ref = philox.gaussian_factor(seed, mode, n, col0, ncols)
    # same Philox words; log/sin/cos from different math libraries (few ulp)
    assert np.max(np.abs(got - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref)))


def _pc_case(x, seed, col0, ncols, t, prec, tol):
    import torch
    d = len(x)
    dims = [c.shape[1] for c in x]
    om = krp.draw_omegas(seed, dims, range(t, d + 1), col0, ncols)
    ref = krp.partial_contractions_rl(x, om, t)
    got = lib_pc(x, seed, col0, ncols, t, prec)
    for k in range(t, d + 1):
        g = got[k - t]
        r = ref[k]
        err = np.linalg.norm(g - r, axis=0) / np.maximum(np.linalg.norm(r, axis=0), 1e-300)
        assert np.max(err) <= tol, (k, np.max(err))


def lib_pc(x, seed, col0, ncols, t, prec):
    import paper_2511_03598_amd as ttr
    return [w.cpu().numpy() for w in ttr.partial_contractions(to_dev(x), seed, col0, ncols, t, prec)]


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_partial_contractions_c1(lib, prec, tol):
    say("pc C1", prec)
    _pc_case(ttgen.c1(), 42, 0, 12, 2, prec, tol)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 2e-5)])
def test_partial_contractions_ragged(lib, prec, tol):
    """Sizes that are not multiples of the tiles: n=70 (two row chunks with
    a tail), r=37, 130 columns (three column blocks), a later pass (t=3,
    col0=9)."""
    say("pc ragged", prec)
    x = ttgen.small_random(11, 4, [5, 70, 3, 9], [7, 37, 6])
    _pc_case(x, 3, 0, 130, 2, prec, tol)
    _pc_case(x, 3, 9, 5, 3, prec, tol)


def test_partial_contractions_chunk_invariant_bitwise(lib):
    """A column is the same bits whichever pass produces it."""
    x = ttgen.small_random(12, 5, 6, 8)
    a = lib_pc(x, 9, 0, 20, 2, "f64")
    b = lib_pc(x, 9, 12, 8, 2, "f64")
    for wa, wb in zip(a, b):
        assert np.array_equal(wa[:, 12:20], wb)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_partial_contractions_c2_full_size(lib, prec, tol):
    """The benchmark's workload (d=20, n=64, formal ranks 200, ell=60)."""
    say("pc C2 full", prec)
    _pc_case(ttgen.c2(), 42, 0, 60, 2, prec, tol)


def _lr_case(x, seed, col0, ncols, t, tol=1e-12):
    """Every entry of W^L_k is a sum of products that can cancel (at k = d,
    r_d = 1, it is the sketch of the whole tensor), so the bar is the
    forward-error bound of such sums: |GPU - oracle| against the same
    recurrence run on |X_k| and |Omega_k|, which bounds the propagated
    error of the earlier cores as well."""
    import paper_2511_03598_amd as ttr
    dims = [c.shape[1] for c in x]
    om = krp.draw_omegas(seed, dims, range(1, t + 1), col0, ncols)
    ref = krp.partial_contractions_lr(x, om, t)
    bound = krp.partial_contractions_lr([np.abs(c) for c in x], {j: np.abs(o) for j, o in om.items()}, t)
    got = [w.cpu().numpy() for w in ttr.partial_contractions_lr(to_dev(x), seed, col0, ncols, t)]
    assert len(got) == t
    for k in range(1, t + 1):
        g, r = got[k - 1], ref[k]
        assert g.shape == r.shape, (k, g.shape, r.shape)
        err = np.abs(g - r) / np.maximum(bound[k], 1e-300)
        assert np.max(err) <= tol, (k, np.max(err))
    return got


def test_partial_contractions_lr_c1(lib):
    say("lr C1")
    x = ttgen.c1()
    _lr_case(x, 42, 0, 12, len(x))
    _lr_case(x, 42, 5, 4, 3)


def test_partial_contractions_lr_ragged(lib):
    """Sizes off the tiles: ranks 37/70/65 (row tiles with tails), n=33,
    67 columns (two column tiles, the second nearly empty), r0*n from 7 to
    2310 (one chunk to several split-K slices), t=1 and t=d, col0 > 0."""
    say("lr ragged")
    x = ttgen.small_random(21, 5, [7, 13, 5, 33, 9], [37, 70, 3, 65])
    _lr_case(x, 5, 0, 67, 5)
    _lr_case(x, 5, 11, 1, 1)
    _lr_case(x, 5, 3, 130, 4)


def test_partial_contractions_lr_c2_full_size(lib):
    """The benchmark's fixed-rank workload (d=20, n=64, formal ranks 200,
    ell=60), every core."""
    say("lr C2 full")
    x = ttgen.c2()
    _lr_case(x, 42, 0, 60, len(x))


def test_partial_contractions_lr_meets_rl_c2(lib):
    """Both recurrences give the full sketch: for every k the column-wise
    dot product of W^L_{k-1} with W_k is the same vector (the sketch of the
    whole tensor), whichever direction produced the two factors."""
    import paper_2511_03598_amd as ttr
    say("lr/rl meet C2")
    x = ttgen.c2()
    d = len(x)
    dev = to_dev(x)
    lr = [w.cpu().numpy() for w in ttr.partial_contractions_lr(dev, 7, 3, 60)]
    rl = [w.cpu().numpy() for w in ttr.partial_contractions(dev, 7, 3, 60, 2, "f64")]
    full = lr[d - 1][0]
    assert lr[d - 1].shape == (1, 60)
    for k in range(2, d + 1):
        meet = np.sum(lr[k - 2] * rl[k - 2], axis=0)
        scale = np.sum(np.abs(lr[k - 2]) * np.abs(rl[k - 2]), axis=0)
        assert np.max(np.abs(meet - full) / scale) <= 1e-12, k


def test_partial_contractions_lr_rejects_bad_t(lib):
    import paper_2511_03598_amd as ttr
    dev = to_dev(ttgen.small_random(3, 3, 4, 3))
    for t in (0, 4):
        with pytest.raises(ttr.TTError):
            ttr.partial_contractions_lr(dev, 1, 0, 4, t)
    with pytest.raises(ttr.TTError):
        ttr.partial_contractions_lr(dev, 1, 0, 0, 2)


@pytest.mark.parametrize("m,b", [(10, 3), (120, 12), (64, 64), (129, 64), (3840, 60), (1000, 17),
                                 (5000, 1), (20000, 16)])
def test_qr_matches_householder(lib, m, b):
    import torch
    say("qr", m, b)
    rng = np.random.default_rng(m * 100 + b)
    a = rng.standard_normal((m, b)) * (10.0 ** (-np.arange(b) / 8.0))[None, :]
    q = lib.qr(torch.tensor(a, device="cuda")).cpu().numpy()
    ref = krp.qr_pos(a)
    assert np.max(np.abs(q.T @ q - np.eye(b))) < 1e-13
    assert np.max(np.abs(q - ref)) < 1e-11


@pytest.mark.parametrize("cond", [1e2, 1e3, 1e5, 1e7])
def test_qr_second_pass_both_factor_paths(lib, cond):
    """After the first CholeskyQR pass the Gram is I + E with |E| about
    eps cond^2: below the near-identity bound 1e-9 for cond 1e2 and 1e3
    (closed-form factor), above it for 1e5 and 1e7 (pivoted Cholesky; 1e7
    also takes the shifted route).  Every case must give the positive-
    diagonal Householder Q and an orthonormal panel."""
    import torch
    rng = np.random.default_rng(int(np.log10(cond)))
    m, b = 3840, 60
    u, _ = np.linalg.qr(rng.standard_normal((m, b)))
    v, _ = np.linalg.qr(rng.standard_normal((b, b)))
    a = (u * np.geomspace(1.0, 1.0 / cond, b)[None, :]) @ v.T
    q = lib.qr(torch.tensor(a, device="cuda")).cpu().numpy()
    ref = krp.qr_pos(a)
    assert np.max(np.abs(q.T @ q - np.eye(b))) < 1e-13
    assert np.max(np.abs(q - ref)) < 1e-15 * cond * 100


def test_qr_fallback_after_qrs_of_other_shapes(lib):
    """Route flags that a QR leaves in the shared QR scratch (near-identity
    passes, shifted route, breakdown) must never reach the Householder tree
    counters of a later QR of another shape: well-conditioned and
    ill-conditioned 60-column panels of several heights, each followed by
    rank-deficient panels whose fallback trees have many levels."""
    import torch
    rng = np.random.default_rng(12)
    for m_good, m_bad in [(3840, 6480), (3200, 8000), (5000, 9000), (3840, 3840)]:
        for cond in (1e2, 1e7):
            u, _ = np.linalg.qr(rng.standard_normal((m_good, 60)))
            good = (u * np.geomspace(1.0, 1.0 / cond, 60)[None, :]) @ np.linalg.qr(rng.standard_normal((60, 60)))[0]
            lib.qr(torch.tensor(good, device="cuda"))
        bad = rng.standard_normal((m_bad, 12)) @ rng.standard_normal((12, 60))  # rank 12
        q = lib.qr(torch.tensor(bad, device="cuda")).cpu().numpy()
        say("qr fallback after", m_good, "->", m_bad)
        assert np.max(np.abs(q.T @ q - np.eye(60))) < 1e-12
        p = q[:, :12] @ (q[:, :12].T @ bad)
        assert np.linalg.norm(bad - p) < 1e-12 * np.linalg.norm(bad)


def test_qr_rank_deficient_still_orthonormal(lib):
    import torch
    rng = np.random.default_rng(3)
    a = rng.standard_normal((300, 10)) @ rng.standard_normal((10, 24))  # rank 10, 24 columns
    q = lib.qr(torch.tensor(a, device="cuda")).cpu().numpy()
    assert np.max(np.abs(q.T @ q - np.eye(24))) < 1e-12
    # the leading 10 columns span range(a)
    p = q[:, :10] @ (q[:, :10].T @ a)
    assert np.linalg.norm(a - p) < 1e-12 * np.linalg.norm(a)


def test_qr_ill_conditioned_full_rank_takes_householder_route(lib):
    """Two nearly parallel columns fail the Cholesky certificate; the panel
    must still come back as the Householder Q."""
    import torch
    rng = np.random.default_rng(8)
    a = rng.standard_normal((2000, 20))
    a[:, 19] = a[:, 0] + 1e-9 * rng.standard_normal(2000)
    q = lib.qr(torch.tensor(a, device="cuda")).cpu().numpy()
    ref = krp.qr_pos(a)
    assert np.max(np.abs(q.T @ q - np.eye(20))) < 1e-13
    assert np.max(np.abs(q[:, :19] - ref[:, :19])) < 1e-12
    assert np.max(np.abs(q[:, 19] - ref[:, 19])) < 1e-5   # sensitive direction


@pytest.mark.parametrize("p,q", [(60, 60), (64, 64), (40, 13), (7, 1), (30, 30)])
def test_svd_small_matches_lapack(lib, p, q):
    import torch
    from oracle.ttsvd import truncation_rank
    rng = np.random.default_rng(p * 7 + q)
    a = rng.standard_normal((p, q)) * (10.0 ** (-np.arange(q) / 6.0))[None, :]
    g, v, sig, t = lib.svd_small(torch.tensor(a, device="cuda"), tau=1e-3)
    g, v, sig = g.cpu().numpy(), v.cpu().numpy(), sig.cpu().numpy()
    s_ref = np.linalg.svd(a, compute_uv=False)
    assert np.max(np.abs(sig - s_ref) / s_ref) < 1e-12          # high relative accuracy
    assert np.max(np.abs(v.T @ v - np.eye(q))) < 1e-13
    assert np.linalg.norm(a @ v - g) < 1e-13 * np.linalg.norm(a)
    assert t == truncation_rank(s_ref, 1e-3)
    _, _, _, t2 = lib.svd_small(torch.tensor(a, device="cuda"), tau=-1.0, target=5)
    assert t2 == min(5, q)


@pytest.mark.parametrize("m,b", [(300, 100), (3000, 200), (129, 129), (20000, 80), (600, 512)])
def test_qr_wide_matches_householder(lib, m, b):
    """Panels past 64 columns: block Gram-Schmidt with reorthogonalisation
    over 64-column panels, each factored by the certified CholeskyQR."""
    import torch
    say("qr wide", m, b)
    rng = np.random.default_rng(m + 7 * b)
    a = rng.standard_normal((m, b)) * (10.0 ** (-np.arange(b) / 64.0))[None, :]
    q = lib.qr(torch.tensor(a, device="cuda")).cpu().numpy()
    ref = krp.qr_pos(a)
    assert np.max(np.abs(q.T @ q - np.eye(b))) < 1e-13
    assert np.max(np.abs(q - ref)) < 1e-10


@pytest.mark.parametrize("p,q", [(100, 100), (200, 130), (65, 65), (380, 380), (512, 512), (300, 40)])
def test_svd_wide_matches_lapack(lib, p, q):
    """The many-workgroup Jacobi (one launch per round of the tournament)
    for widths past 64 or heights past 64: singular values to high relative
    accuracy on graded columns, A V = G, orthonormal V, the tail rule."""
    import torch
    from oracle.ttsvd import truncation_rank
    say("svd wide", p, q)
    rng = np.random.default_rng(p * 13 + q)
    a = rng.standard_normal((p, q)) * (10.0 ** (-np.arange(q) / 40.0))[None, :]
    g, v, sig, t = lib.svd_small(torch.tensor(a, device="cuda"), tau=1e-3)
    g, v, sig = g.cpu().numpy(), v.cpu().numpy(), sig.cpu().numpy()
    s_ref = np.linalg.svd(a, compute_uv=False)
    assert np.max(np.abs(sig - s_ref) / s_ref) < 1e-11
    assert np.all(np.diff(sig) <= 0)
    assert np.max(np.abs(v.T @ v - np.eye(q))) < 1e-12
    assert np.linalg.norm(a @ v - g) < 1e-12 * np.linalg.norm(a)
    assert t == truncation_rank(s_ref, 1e-3)
    _, _, _, t2 = lib.svd_small(torch.tensor(a, device="cuda"), tau=-1.0, target=70)
    assert t2 == min(70, q)


def test_svd_small_rank_deficient(lib):
    import torch
    rng = np.random.default_rng(4)
    a = rng.standard_normal((50, 6)) @ rng.standard_normal((6, 40))
    g, v, sig, t = lib.svd_small(torch.tensor(a, device="cuda"), tau=1e-10 * np.linalg.norm(a))
    sig = sig.cpu().numpy()
    assert t == 6
    assert np.all(sig[6:] < 1e-12 * sig[0])


@pytest.mark.parametrize("case,tol", [("c1", 2e-2), ("ragged", 2e-2), ("c2", 5e-2)])
def test_partial_contractions_bf16(lib, case, tol):
    """BF16 sketch (bfloat16 operands and W storage, FP32 accumulation)
    against the FP64 oracle on the same Omega: the bound is a few bfloat16
    units (2^-8) per chained contraction; the measured error is printed."""
    if case == "c1":
        x, cols, seed = ttgen.c1(), 12, 42
    elif case == "ragged":
        x, cols, seed = ttgen.small_random(11, 4, [5, 70, 3, 9], [7, 37, 6]), 130, 3
    else:
        x, cols, seed = ttgen.c2(), 60, 42
    dims = [c.shape[1] for c in x]
    d = len(x)
    om = krp.draw_omegas(seed, dims, range(2, d + 1), 0, cols)
    ref = krp.partial_contractions_rl(x, om, 2)
    got = lib_pc(x, seed, 0, cols, 2, "bf16")
    worst = 0.0
    for k in range(2, d + 1):
        g, r = got[k - 2], ref[k]
        err = np.linalg.norm(g - r, axis=0) / np.maximum(np.linalg.norm(r, axis=0), 1e-300)
        worst = max(worst, float(np.max(err)))
    say("bf16 partial contractions", case, "max column rel err", worst)
    assert worst <= tol
