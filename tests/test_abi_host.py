"""The C ABI library loads, exports every symbol include/ttround.h declares,
and rejects malformed arguments on the host (no GPU needed: validation
happens before any device call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ttround.h")


def declared_symbols():
    text = open(HEADER).read()
    return re.findall(r"^\s*(?:tt_status|const char\*|void)\s+(tt_\w+)\s*\(", text, re.M)


def test_header_declares_the_boundary():
    names = set(declared_symbols())
    for n in ("tt_round_fixed", "tt_round_adaptive", "tt_out_capacity", "tt_last_error",
              "tt_partial_contractions", "tt_partial_contractions_lr", "tt_gaussian_factor", "tt_qr", "tt_philox4x32_10"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2511_03598_amd as ttr
    L = ttr.lib()
    missing = [n for n in declared_symbols() if not hasattr(L, n)]
    assert missing == []


def _view(d, n, ranks, ptrs):
    import paper_2511_03598_amd as ttr
    na = (ctypes.c_int64 * max(d, 1))(*n)
    ra = (ctypes.c_int64 * (max(d, 1) + 1))(*ranks)
    pa = (ctypes.c_void_p * max(d, 1))(*ptrs)
    return ttr._View(d, na, ra, pa), (na, ra, pa)


def test_out_capacity_host_only():
    import paper_2511_03598_amd as ttr
    L = ttr.lib()
    v, keep = _view(3, [4, 5, 6], [1, 7, 9, 1], [1, 2, 3])
    cap = (ctypes.c_int64 * 3)()
    assert L.tt_out_capacity(ctypes.byref(v), None, cap) == 0
    # c = (1, min(7,4), min(9,20), 1) = (1, 4, 9, 1)
    assert list(cap) == [1 * 4 * 4, 4 * 5 * 9, 9 * 6 * 1]


@pytest.mark.parametrize("d,n,ranks", [
    (1, [4], [1, 1]),                 # d < 2
    (2, [4, 4], [2, 3, 1]),           # r_0 != 1
    (2, [4, 4], [1, 3, 2]),           # r_d != 1
    (2, [0, 4], [1, 3, 1]),           # n < 1
    (3, [4, 4, 4], [1, 0, 2, 1]),     # zero rank
])
def test_malformed_views_rejected(d, n, ranks):
    import paper_2511_03598_amd as ttr
    L = ttr.lib()
    v, keep = _view(d, n, ranks, [1] * max(d, 1))
    cap = (ctypes.c_int64 * 4)()
    assert L.tt_out_capacity(ctypes.byref(v), None, cap) == ttr.TTError(-1, "").status
    assert L.tt_last_error()


def test_round_entry_points_validate_before_device():
    import paper_2511_03598_amd as ttr
    L = ttr.lib()
    v, keep = _view(2, [4, 4], [1, 3, 1], [1, 2])
    out = ttr._Out(2, (ctypes.c_int64 * 3)(), (ctypes.c_void_p * 2)(1, 2), (ctypes.c_int64 * 2)(100, 100), 0)
    assert L.tt_round_fixed(ctypes.byref(v), None, 0, 1, None, ctypes.byref(out)) == -1   # ell < 1
    assert L.tt_round_adaptive(ctypes.byref(v), 0.0, 4, 1, None, ctypes.byref(out)) == -1  # tol <= 0
    assert L.tt_round_adaptive(ctypes.byref(v), -1.0, 4, 1, None, ctypes.byref(out)) == -1
    bad = ttr._Out(3, (ctypes.c_int64 * 4)(), (ctypes.c_void_p * 3)(1, 2, 3), (ctypes.c_int64 * 3)(1, 1, 1), 0)
    assert L.tt_round_adaptive(ctypes.byref(v), 1e-3, 4, 1, None, ctypes.byref(bad)) == -1  # d mismatch
    assert L.tt_round_fixed(None, None, 4, 1, None, ctypes.byref(out)) == -1
    nul, keep2 = _view(2, [4, 4], [1, 3, 1], [1, 0])
    assert L.tt_round_fixed(ctypes.byref(nul), None, 4, 1, None, ctypes.byref(out)) == -1  # null core
    opts = ttr._Opts(7, 0.0, 0.0, 0, None)                       # no such precision
    assert L.tt_round_fixed(ctypes.byref(v), None, 4, 1, ctypes.byref(opts), ctypes.byref(out)) == -1
    assert b"precision" in L.tt_last_error()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2511_03598_amd as ttr
    monkeypatch.setattr(ttr, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(ttr, "_lib", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        ttr.lib()


def test_kernel_timing_host_only():
    """Enabling (a mask of kinds), disabling and reading the timers makes no
    device call when nothing was launched; bad kinds are rejected."""
    import paper_2511_03598_amd as ttr
    L = ttr.lib()
    assert L.tt_kernel_timing(1) == 0
    n, ms = ctypes.c_int64(-1), ctypes.c_double(-1.0)
    assert L.tt_kernel_timing_read(0, ctypes.byref(n), ctypes.byref(ms)) == 0
    assert n.value == 0 and ms.value == 0.0
    assert L.tt_kernel_timing(0) == 0
    assert L.tt_kernel_timing(0xF) == 0  # every kind
    assert L.tt_kernel_timing(0x10) == -1 and L.tt_kernel_timing(-1) == -1  # unknown kinds
    assert L.tt_kernel_timing(0) == 0
    assert L.tt_kernel_timing_read(7, ctypes.byref(n), ctypes.byref(ms)) == -1
    assert L.tt_kernel_timing_read(0, None, ctypes.byref(ms)) == -1


def test_workspace_bytes_host_only():
    import paper_2511_03598_amd as ttr
    L = ttr.lib()
    v, keep = _view(4, [8, 9, 10, 11], [1, 20, 30, 25, 1], [1, 2, 3, 4])
    b_small, b_big, b_ad = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    assert L.tt_workspace_bytes(ctypes.byref(v), 4, 0, ctypes.byref(b_small)) == 0
    assert L.tt_workspace_bytes(ctypes.byref(v), 16, 0, ctypes.byref(b_big)) == 0
    assert L.tt_workspace_bytes(ctypes.byref(v), 0, 0, ctypes.byref(b_ad)) == 0
    assert 0 < b_small.value < b_big.value <= b_ad.value
    assert L.tt_workspace_bytes(ctypes.byref(v), 4, 9, ctypes.byref(b_small)) == -1
    assert L.tt_workspace_bytes(None, 4, 0, ctypes.byref(b_small)) == -1


def test_batch_and_server_validate_on_host():
    import paper_2511_03598_amd as ttr
    L = ttr.lib()
    # empty batch is a no-op; malformed arguments fail before any device call
    assert L.tt_round_adaptive_batch(None, 0, None, 4, None, None, None) == 0
    v, keep = _view(2, [4, 4], [1, 3, 1], [1, 2])
    out = ttr._Out(2, (ctypes.c_int64 * 3)(), (ctypes.c_void_p * 2)(1, 2), (ctypes.c_int64 * 2)(100, 100), 0)
    views = (ttr._View * 1)(v)
    outs = (ttr._Out * 1)(out)
    seeds = (ctypes.c_uint64 * 1)(1)
    assert L.tt_round_adaptive_batch(views, 1, (ctypes.c_double * 1)(0.0), 4, seeds, None, outs) == -1
    assert L.tt_round_adaptive_batch(views, -1, (ctypes.c_double * 1)(1e-3), 4, seeds, None, outs) == -1
    assert L.tt_round_adaptive_batch(views, 1, None, 4, seeds, None, outs) == -1
    t = ctypes.c_uint64()
    assert L.tt_round_submit(None, None, ctypes.byref(t)) == -1
    r = ctypes.POINTER(ttr._Result)()
    assert L.tt_round_poll(None, 1, ctypes.byref(r)) == -1
    assert L.tt_server_create(None, None) == -1
    assert L.tt_result_copy(None, None, None) == -1
    L.tt_result_release(None)
    L.tt_server_destroy(None)


def test_sum_capacity_and_validation_host_only():
    import paper_2511_03598_amd as ttr
    L = ttr.lib()
    v1, k1 = _view(3, [4, 5, 6], [1, 2, 3, 1], [1, 2, 3])
    v2, k2 = _view(3, [4, 5, 6], [1, 3, 4, 1], [4, 5, 6])
    views = (ttr._View * 2)(v1, v2)
    cap = (ctypes.c_int64 * 3)()
    assert L.tt_sum_out_capacity(views, 2, None, cap) == 0
    # formal ranks (1, 5, 7, 1), capped at (1, min(5,4), min(7,20), 1) = (1, 4, 7, 1)
    assert list(cap) == [1 * 4 * 4, 4 * 5 * 7, 7 * 6 * 1]
    assert L.tt_sum_out_capacity(views, 0, None, cap) == -1
    bad, kb = _view(3, [4, 5, 7], [1, 2, 3, 1], [1, 2, 3])  # mode sizes differ
    views_bad = (ttr._View * 2)(v1, bad)
    assert L.tt_sum_out_capacity(views_bad, 2, None, cap) == -1
    assert b"mode sizes" in L.tt_last_error()
    outs = ttr._Out(3, (ctypes.c_int64 * 4)(), (ctypes.c_void_p * 3)(1, 2, 3), cap, 0)
    w = (ctypes.c_double * 2)(1.0, float("nan"))
    assert L.tt_round_sum_adaptive(views, 2, w, 1e-6, 4, 1, None, ctypes.byref(outs)) == -1
    assert b"finite" in L.tt_last_error()
    assert L.tt_round_sum_fixed(views, 2, None, None, 0, 1, None, ctypes.byref(outs)) == -1
    assert L.tt_round_sum_adaptive(views, 2, None, 0.0, 4, 1, None, ctypes.byref(outs)) == -1
    assert L.tt_round_sum_adaptive(views_bad, 2, None, 1e-6, 4, 1, None, ctypes.byref(outs)) == -1


def test_noalloc_entry_point_rejects_oversize_on_the_host():
    """tt_round_fixed_noalloc refuses a shape whose workspace estimate
    exceeds TT_NOALLOC_SCRATCH_BYTES before any device call."""
    import paper_2511_03598_amd as ttr
    L = ttr.lib()
    text = open(HEADER).read()
    m = re.search(r"#define TT_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == 64 << 20
    v, keep = _view(3, [4096, 4096, 64], [1, 300, 300, 1], [1, 2, 3])
    ranks = (ctypes.c_int64 * 4)()
    ptrs = (ctypes.c_void_p * 3)(1, 2, 3)
    cap = (ctypes.c_int64 * 3)(1 << 40, 1 << 40, 1 << 40)
    out = ttr._Out(3, ranks, ptrs, cap, 0)
    st = L.tt_round_fixed_noalloc(ctypes.byref(v), None, 60, ctypes.c_uint64(1), None, ctypes.byref(out))
    assert st == -2
    assert b"scratch" in L.tt_last_error()
