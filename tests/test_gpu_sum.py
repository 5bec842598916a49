"""Rounding of sums of TT tensors on the GPU (terms sketched separately,
the formal sum never assembled) against the oracle's rounding of the
formal sum with the same Gaussian factors, and against the GPU rounding of
the explicitly assembled formal sum.

Bar as for single tensors: ||Y_gpu - Y_oracle|| / ||X|| <= 1e-10 with FP64
partial contractions, <= 1e-5 with FP32; equal ranks."""
import numpy as np
import pytest

import ttgen
from oracle import krp, tt
from tests.gpu_helpers import rel_tensor_diff, say, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5}


def _terms(seed=700, d=5, n=6, ranks=(4, 3, 5), weights=(1.0, 1e-2, -0.5)):
    rng = ttgen.rng_for(seed)
    dims = [n] * d
    tts = [ttgen.random_tt(rng, dims, ttgen.clamp_ranks(dims, [1] + [r] * (d - 1) + [1]))
           for r in ranks]
    return tts, list(weights)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_sum_fixed_vs_oracle(lib, prec):
    tts, w = _terms()
    x = ttgen.formal_sum(tts, w)
    say("sum fixed", prec)
    yg, ig = lib.round_sum_fixed([to_dev(c) for c in tts], 8, 21, weights=w, prec=prec)
    yo, io = krp.round_sum_fixed(tts, 8, 21, weights=w)
    assert ig["ranks"] == io["ranks"]
    assert rel_tensor_diff(x, to_host(yg), yo) <= TOL[prec]
    assert tt.left_orth_defect(to_host(yg)) < 1e-12


def test_sum_fixed_with_truncation(lib):
    tts, w = _terms(701)
    x = ttgen.formal_sum(tts, w)
    tg = [1, 5, 6, 6, 5, 1]
    yg, ig = lib.round_sum_fixed([to_dev(c) for c in tts], 10, 4, weights=w, target_ranks=tg)
    yo, io = krp.round_sum_fixed(tts, 10, 4, weights=w, target_ranks=tg)
    assert ig["ranks"] == io["ranks"] == tg
    assert rel_tensor_diff(x, to_host(yg), yo) <= TOL["f64"]
    assert tt.right_orth_defect(to_host(yg)) < 1e-12


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_sum_adaptive_vs_oracle(lib, prec):
    tts, w = _terms(702, d=6, n=5, ranks=(5, 4, 3))
    x = ttgen.formal_sum(tts, w)
    tol = 1e-6
    yg, ig = lib.round_sum_adaptive([to_dev(c) for c in tts], tol, 3, 17, weights=w, prec=prec)
    yo, io = krp.round_sum_adaptive(tts, tol, 3, 17, weights=w)
    say("sum adaptive", prec, ig["ranks"], io["ranks"], "margin", io["min_margin"])
    assert ig["ranks"] == io["ranks"]
    assert rel_tensor_diff(x, to_host(yg), yo) <= TOL[prec]
    assert tt.rel_err(x, to_host(yg)) <= tol


def test_sum_equals_assembled_formal_sum(lib):
    """Sketching the terms separately gives the rounding of the assembled
    formal sum (same seed) up to rounding order."""
    tts, w = _terms(703, d=6, n=5, ranks=(5, 4, 3))
    x = ttgen.formal_sum(tts, w)
    ys, i_s = lib.round_sum_adaptive([to_dev(c) for c in tts], 1e-6, 3, 5, weights=w, recompress=1)
    yf, i_f = lib.round_adaptive(to_dev(x), 1e-6, 3, 5, recompress=1)
    assert i_s["ranks"] == i_f["ranks"]
    assert rel_tensor_diff(x, to_host(ys), to_host(yf)) <= TOL["f64"]
    yfs, ifs = lib.round_sum_fixed([to_dev(c) for c in tts], 7, 5, weights=w)
    yff, iff = lib.round_fixed(to_dev(x), 7, 5)
    assert ifs["ranks"] == iff["ranks"]
    assert rel_tensor_diff(x, to_host(yfs), to_host(yff)) <= TOL["f64"]


def test_sum_single_term_is_plain_rounding(lib):
    x = ttgen.small_random(704, 5, 6, 5)
    a, ia = lib.round_sum_adaptive([to_dev(x)], 1e-6, 2, 3)
    b, ib = lib.round_adaptive(to_dev(x), 1e-6, 2, 3)
    assert ia["ranks"] == ib["ranks"]
    assert all(np.array_equal(p, q) for p, q in zip(to_host(a), to_host(b)))


def test_sum_krylov_like_small_request(lib):
    """A small C5-style request: 8 terms (d=8, n=16, ranks 20) with
    coefficients g_i 10^-i, tol 1e-6."""
    tts, coef = ttgen.c5_terms(1005, small=True)
    x = ttgen.formal_sum(tts, coef)
    yg, ig = lib.round_sum_adaptive([to_dev(c) for c in tts], 1e-6, 20, 9, weights=coef)
    yo, io = krp.round_sum_adaptive(tts, 1e-6, 20, 9, weights=coef)
    say("c5 small sum ranks", ig["ranks"], io["ranks"], "margin", io["min_margin"])
    assert ig["ranks"] == io["ranks"]
    assert rel_tensor_diff(x, to_host(yg), yo) <= TOL["f64"]
    assert tt.rel_err(x, to_host(yg)) <= 1e-6


def test_sum_terms_of_different_ranks_and_rank_one_bonds(lib):
    rng = ttgen.rng_for(705)
    dims = [3, 4, 5, 4]
    t1 = ttgen.random_tt(rng, dims, [1, 1, 1, 1, 1])
    t2 = ttgen.random_tt(rng, dims, [1, 3, 6, 2, 1])
    t3 = ttgen.random_tt(rng, dims, [1, 2, 2, 2, 1])
    tts, w = [t1, t2, t3], [2.0, -1.0, 0.25]
    x = ttgen.formal_sum(tts, w)
    yg, ig = lib.round_sum_fixed([to_dev(c) for c in tts], 6, 8, weights=w)
    yo, io = krp.round_sum_fixed(tts, 6, 8, weights=w)
    assert ig["ranks"] == io["ranks"]
    assert rel_tensor_diff(x, to_host(yg), yo) <= TOL["f64"]
