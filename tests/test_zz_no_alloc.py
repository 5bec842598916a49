"""The allocation-free fixed-rank entry point (tt_round_fixed_noalloc)
against tt_round_fixed through the C ABI: the same ranks and bitwise the
same cores, on two calls in a row that share the library's static scratch
array, the second with a smaller input (so stale contents of the first call
would show), and against the oracle on the small one."""
import numpy as np
import pytest
import torch

import ttgen
from oracle import krp, tt
from gpu_helpers import rel_tensor_diff, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _both(lib, x, ell, seed, tgt, prec):
    dev = to_dev(x)
    ya, ia = lib.round_fixed(dev, ell, seed, target_ranks=tgt, prec=prec)
    yb, ib = lib.round_fixed_noalloc(dev, ell, seed, target_ranks=tgt, prec=prec)
    torch.cuda.synchronize()
    assert ib["ranks"] == ia["ranks"]
    assert ib["orth"] == ia["orth"]
    assert ib["qr_retries"] == 0
    for u, v in zip(ya, yb):
        assert torch.equal(u, v)
    return to_host(yb), ib


def test_noalloc_matches_fixed_large_then_small(lib):
    say("noalloc: C2 full size, f32 sketch, ell 60 -> 50")
    x2 = ttgen.c2()
    tgt2 = [1] + [50] * 19 + [1]
    y2, i2 = _both(lib, x2, 60, 42, tgt2, "f32")
    assert i2["ranks"] == tgt2
    say("noalloc: C1, f64, ell 12 -> 10 (second, smaller call)")
    x1 = ttgen.c1()
    tgt1 = [1] + [10] * 5 + [1]
    y1, i1 = _both(lib, x1, 12, 7, tgt1, "f64")
    yo, io = krp.round_fixed(x1, 12, 7, tgt1)
    assert i1["ranks"] == io["ranks"] == tgt1
    assert rel_tensor_diff(x1, y1, yo) <= 1e-10
    say("noalloc: C1 without truncation, then C1 edge shape")
    _both(lib, x1, 9, 3, None, "f64")
    xs = ttgen.small_random(24, 5, [7, 70, 3, 9, 4], [7, 37, 20, 4])
    ys, isx = _both(lib, xs, 30, 5, None, "bf16")
    assert all(np.isfinite(c).all() for c in ys)


def test_noalloc_rejects_oversize_before_work(lib):
    """A shape whose workspace estimate exceeds the scratch array is
    refused with TT_ENOMEM, and the next call still works."""
    big = [torch.zeros(1, 4096, 300, dtype=torch.float64, device="cuda"),
           torch.zeros(300, 4096, 300, dtype=torch.float64, device="cuda"),
           torch.zeros(300, 64, 1, dtype=torch.float64, device="cuda")]
    with pytest.raises(lib.TTError) as e:
        lib.round_fixed_noalloc(big, 60, 1)
    assert e.value.status == -2
    del big
    x1 = ttgen.c1()
    _both(lib, x1, 12, 9, [1] + [10] * 5 + [1], "f64")
