"""Deterministic TT-SVD rounding on the GPU (Sec. 2.3, Algorithm
"TT-Rounding"), the same-GPU baseline of the randomized roundings, against
the oracle's TT-SVD on the same input.

Bar: equal ranks and ||Y_gpu - Y_oracle|| / ||X|| <= 1e-10 (stable
formal-difference norm), the same tau, the tolerance bound
||X - Y|| <= tol ||X||, and left-orthonormal cores.  The cases cover a
factor with fewer rows than columns on both sweeps (C2: n_1 = 64 < r_1 =
200 and n_d = 64 < r_{d-1}), bonds wider than 64 and 512-wide limits
(C5's formal ranks 400), ragged shapes and target ranks."""
import pytest

import ttgen
from oracle import tt, ttsvd
from tests.gpu_helpers import rel_tensor_diff, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _case(lib, x, tol=None, ranks=None):
    yg, ig = lib.round_ttsvd(to_dev(x), tol=tol, target_ranks=ranks)
    yo, io = ttsvd.tt_svd_round(x, tol=tol, ranks=ranks)
    yg = to_host(yg)
    say("  ranks", ig["ranks"])
    assert ig["ranks"] == io["ranks"]
    d = rel_tensor_diff(x, yg, yo)
    say("  rel diff vs oracle %.3e" % d)
    assert d <= 1e-10
    assert tt.left_orth_defect(yg) < 1e-12
    if tol is not None:
        assert abs(ig["tau"] - io["tau"]) <= 1e-12 * io["tau"]
        assert tt.diff_norm(x, yg) <= tol * tt.norm(x) * (1 + 1e-8)
    return yg, ig


def test_ttsvd_c1_recovers_true_ranks(lib):
    say("TT-SVD C1")
    _, info = _case(lib, ttgen.c1(), tol=1e-8)
    assert info["ranks"] == [1, 10, 10, 10, 10, 10, 1]


def test_ttsvd_ragged_tolerance_and_targets(lib):
    say("TT-SVD ragged")
    x = ttgen.small_random(41, 5, [4, 9, 13, 6, 5], [4, 30, 70, 5])
    _case(lib, x, tol=1e-3)
    _case(lib, x, ranks=[1, 3, 20, 40, 4, 1])
    _case(lib, x, ranks=[1, 1, 1, 1, 1, 1])


def test_ttsvd_c2_full_size(lib):
    say("TT-SVD C2 full size")
    _case(lib, ttgen.c2(), tol=1e-6)


def test_ttsvd_c5_large_request(lib):
    say("TT-SVD C5 large request (formal ranks 400)")
    tts, coef = ttgen.c5_terms(2000)
    _case(lib, ttgen.formal_sum(tts, coef), tol=1e-6)


def test_ttsvd_rejects_bad_arguments(lib):
    x = to_dev(ttgen.small_random(3, 3, 4, 3))
    with pytest.raises(lib.TTError):
        lib.round_ttsvd(x, tol=-1.0)
    with pytest.raises(lib.TTError):
        lib.round_ttsvd(x, target_ranks=[1, 0, 2, 1])
