"""Batched and served rounding through the C ABI: every result must be
bitwise the same as the synchronous single-tensor call with the same
arguments (alone or in the mix), admission must honour the memory budget,
and the results must match the oracle."""
import numpy as np
import pytest

import ttgen
from oracle import krp, tt
from tests.gpu_helpers import rel_tensor_diff, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _mix(count=6, seed=300):
    """Small TTs of uneven d, n and ranks, each a weighted sum of three TTs
    (true ranks below the formal ones)."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        d = int(rng.integers(3, 7))
        n = int(rng.integers(4, 11))
        s = int(rng.integers(2, 7))
        out.append(ttgen.c4_one(seed + t, d, n, s, q=1e-3))
    return out


def _same(a, b):
    return len(a) == len(b) and all(np.array_equal(x, y) for x, y in zip(a, b))


def test_batch_equals_single_calls(lib):
    """The float64 batch (one persistent launch) gives the single calls'
    ranks and tensors to rounding error, and the oracle's within 1e-10."""
    xs = _mix()
    devs = [to_dev(x) for x in xs]
    res = lib.round_adaptive_batch(devs, 1e-6, 4, [11 + i for i in range(len(xs))])
    for i, (x, dv) in enumerate(zip(xs, devs)):
        ys, info = res[i]
        y1, i1 = lib.round_adaptive(dv, 1e-6, 4, 11 + i)
        say("batch", i, info["ranks"])
        assert info["ranks"] == i1["ranks"]
        assert rel_tensor_diff(x, to_host(ys), to_host(y1)) <= 1e-12
        yo, io = krp.round_adaptive(x, 1e-6, 4, 11 + i)
        assert info["ranks"] == io["ranks"]
        assert rel_tensor_diff(x, to_host(ys), yo) <= 1e-10


def test_batch_f32_sketch_equals_single_calls(lib):
    """A float32-sketch batch runs as concurrent single roundings: bitwise
    the same results as the single calls."""
    xs = _mix()
    devs = [to_dev(x) for x in xs]
    res = lib.round_adaptive_batch(devs, 1e-6, 4, [11 + i for i in range(len(xs))], prec="f32")
    for i, dv in enumerate(devs):
        ys, info = res[i]
        y1, i1 = lib.round_adaptive(dv, 1e-6, 4, 11 + i, prec="f32")
        assert info["ranks"] == i1["ranks"]
        assert _same(to_host(ys), to_host(y1))


def test_server_results_same_alone_and_in_mix(lib):
    xs = _mix(8, 400)
    devs = [to_dev(x) for x in xs]
    srv = lib.Server(workers=4)
    try:
        tickets = []
        for i, dv in enumerate(devs):
            if i % 3 == 2:
                tickets.append(srv.submit(dv, kind="fixed", ell=6, seed=5 + i))
            else:
                tickets.append(srv.submit(dv, kind="adaptive", tol=1e-6, ell_block=4, seed=5 + i))
        got = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for i, (dv, (ys, info)) in enumerate(zip(devs, got)):
        if i % 3 == 2:
            y1, i1 = lib.round_fixed(dv, 6, 5 + i)
        else:
            y1, i1 = lib.round_adaptive(dv, 1e-6, 4, 5 + i)
        assert info["ranks"] == i1["ranks"]
        assert _same(to_host(ys), to_host(y1)), i
        assert info["done_s"] >= info["start_s"] >= info["submit_s"]


def test_server_fixed_truncation_concurrent_equals_direct(lib):
    """Fixed-rank roundings with a truncation (sketch ell = 12, target 10)
    served concurrently by four workers give bitwise the direct call's
    result (QR scratch, truncation buffers and SVD state are per
    workspace)."""
    x = ttgen.c1()
    dv = to_dev(x)
    tgt = [1] + [10] * 5 + [1]
    y1, i1 = lib.round_fixed(dv, 12, 42, target_ranks=tgt)
    srv = lib.Server(workers=4)
    try:
        tickets = [srv.submit(dv, kind="fixed", ell=12, target_ranks=tgt, seed=42) for _ in range(12)]
        got = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for ys, info in got:
        assert info["ranks"] == i1["ranks"] == tgt
        assert _same(to_host(ys), to_host(y1))


def test_server_budget_serialises_and_rejects(lib):
    xs = _mix(3, 500)
    devs = [to_dev(x) for x in xs]
    need = max(lib.workspace_bytes(dv, 0) for dv in devs)
    # room for one request at a time (each reserves at least its workspace
    # estimate, which is dominated by a fixed 16 MiB here): admission must
    # serialise them
    srv = lib.Server(mem_budget=need * 3 // 2, workers=4)
    try:
        tickets = [srv.submit(dv, tol=1e-6, ell_block=4, seed=1) for dv in devs]
        got = [srv.wait(t) for t in tickets]
        starts = sorted((g[1]["start_s"], g[1]["done_s"]) for g in got)
        for a, b in zip(starts, starts[1:]):
            assert b[0] >= a[1] - 1e-6  # no overlap under this budget
    finally:
        srv.close()
    tiny = lib.Server(mem_budget=1 << 20, workers=2)
    try:
        with pytest.raises(lib.TTError, match="ECAPACITY"):
            tiny.submit(devs[0], tol=1e-6, ell_block=4, seed=1)
    finally:
        tiny.close()


def test_server_poll_until_done(lib):
    x = ttgen.c1()
    dv = to_dev(x)
    srv = lib.Server(workers=2)
    try:
        t = srv.submit(dv, tol=1e-8, ell_block=4, seed=42)
        out = None
        for _ in range(200000):
            out = srv.poll(t)
            if out is not None:
                break
        assert out is not None
        ys, info = out
        assert tt.rel_err(x, to_host(ys)) <= 1.5e-8
        with pytest.raises(lib.TTError, match="ENOTFOUND"):
            srv.poll(t)
    finally:
        srv.close()


def test_server_failed_request_leaves_neighbours_intact(lib):
    """A request that the library rejects after its sweep has been queued
    (Remark 2 recompression of ranks above the truncation pass's limit of
    512, on a flat bond spectrum)
    returns TT_EUNSUPPORTED, and the requests served beside it stay bitwise
    equal to their solo runs (the failed request's buffers go back to the
    pools only after its stream has drained)."""
    wide = ttgen.c3(seed=7, d=4, n=32, r=600, noise_r=10, decay=1e9)
    dw = to_dev(wide)
    y_alone, i_alone = lib.round_adaptive(dw, 1e-6, 16, 3)
    assert max(i_alone["ranks"]) > 512
    xs = _mix(6, 600)
    devs = [to_dev(x) for x in xs]
    solo = [lib.round_adaptive(dv, 1e-6, 4, 20 + i) for i, dv in enumerate(devs)]
    srv = lib.Server(workers=4)
    try:
        tickets = []
        for i, dv in enumerate(devs):
            tickets.append((i, srv.submit(dv, tol=1e-6, ell_block=4, seed=20 + i)))
            if i % 2 == 0:
                tickets.append((-1, srv.submit(dw, tol=1e-6, ell_block=16, seed=3, recompress=1)))
        for i, t in tickets:
            if i < 0:
                with pytest.raises(lib.TTError, match="EUNSUPPORTED"):
                    srv.wait(t)
            else:
                ys, info = srv.wait(t)
                assert info["ranks"] == solo[i][1]["ranks"]
                assert _same(to_host(ys), to_host(solo[i][0])), i
    finally:
        srv.close()
    # the failure left no error behind for later calls on this thread
    y2, i2 = lib.round_adaptive(dw, 1e-6, 16, 3)
    assert _same(to_host(y2), to_host(y_alone))
