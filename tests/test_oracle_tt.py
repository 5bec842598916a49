"""Pins for the oracle's TT utilities: brute-force reconstruction from the
index formula, norms against the dense tensor, and the stable difference
norm at 1e-12 relative resolution."""
import itertools

import numpy as np

import ttgen
from oracle import tt


def _entry(cores, idx):
    v = np.ones((1, 1))
    for c, i in zip(cores, idx):
        v = v @ c[:, i, :]
    return float(v[0, 0])


def test_full_matches_index_formula():
    x = ttgen.small_random(3, 4, [3, 2, 4, 3], [2, 3, 2])
    f = tt.full(x)
    for idx in itertools.product(*[range(n) for n in f.shape]):
        assert f[idx] == np.float64(_entry(x, idx)) or abs(f[idx] - _entry(x, idx)) < 1e-12


def test_orthogonalize_rl_preserves_tensor_and_orthonormal():
    x = ttgen.small_random(4, 5, 4, 3)
    y = tt.orthogonalize_rl(x)
    assert np.allclose(tt.full(x), tt.full(y), rtol=0, atol=1e-12 * np.abs(tt.full(x)).max())
    assert tt.right_orth_defect(y) < 1e-13


def test_norm_matches_dense():
    x = ttgen.small_random(5, 5, 4, 3)
    assert abs(tt.norm(x) - np.linalg.norm(tt.full(x))) < 1e-12 * np.linalg.norm(tt.full(x))


def test_formal_sum_is_sum():
    a = ttgen.small_random(6, 4, 3, 2)
    b = ttgen.small_random(7, 4, 3, 3)
    s = tt.formal_sum([a, b], [2.0, -0.5])
    assert tt.ranks_of(s) == [1, 5, 5, 5, 1]
    assert np.allclose(tt.full(s), 2.0 * tt.full(a) - 0.5 * tt.full(b), atol=1e-12)


def test_diff_norm_resolves_tiny_differences():
    """The formal-difference norm sees a 1e-12 relative perturbation that the
    <A,A>-2<A,B>+<B,B> expansion cannot."""
    x = ttgen.small_random(8, 5, 4, 3)
    y = [c.copy() for c in x]
    y[2] = y[2] * (1.0 + 1e-12)
    exact = 1e-12 * np.linalg.norm(tt.full(x))
    got = tt.diff_norm(x, y)
    assert abs(got - exact) < 1e-3 * exact
    assert tt.diff_norm(x, x) < 1e-15 * tt.norm(x)


def test_diff_norm_matches_dense_for_unrelated_tensors():
    a = ttgen.small_random(9, 4, 4, 3)
    b = ttgen.small_random(10, 4, 4, 2)
    assert abs(tt.diff_norm(a, b) - np.linalg.norm(tt.full(a) - tt.full(b))) < 1e-12 * np.linalg.norm(tt.full(a))


def test_ttgen_c1_structure():
    x = ttgen.c1()
    assert tt.ranks_of(x) == [1, 30, 30, 30, 30, 30, 1]
    z = ttgen.c1()  # deterministic
    assert all(np.array_equal(a, b) for a, b in zip(x, z))
    # X = 1.25 Z exactly: the norm of the formal sum equals 1.25 ||Z||
    rng = ttgen.rng_for(1001)
    zz = ttgen.random_tt(rng, [10] * 6, [1, 10, 10, 10, 10, 10, 1])
    assert abs(tt.norm(x) - 1.25 * tt.norm(zz)) < 1e-12 * tt.norm(x)
