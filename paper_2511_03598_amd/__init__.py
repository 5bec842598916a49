"""Python binding of libttround.so: KRP-sketched randomized TT-rounding on
MI355X (gfx950).

This module only marshals arguments for the C ABI declared in
include/ttround.h; every step of the rounding runs in the library's HIP
kernels.  PyTorch provides device memory and streams.  If the shared
library is missing, every call raises: there is no fallback.

TT tensors are lists of float64 CUDA tensors of shape (r_{k-1}, n_k, r_k),
r_0 = r_d = 1 (contiguous).
"""
import ctypes
import os

__all__ = ["lib", "round_fixed", "round_fixed_noalloc", "round_adaptive", "gaussian_factor", "philox4x32_10",
           "partial_contractions", "qr", "svd_small", "BatchPlan", "round_adaptive_batch", "out_capacity", "last_info", "TTError",
           "PREC_F64", "PREC_F32", "PREC_BF16", "LIB_PATH"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libttround.so")

PREC_F64, PREC_F32, PREC_BF16 = 0, 1, 2
_PREC = {"f64": 0, "fp64": 0, "float64": 0, "f32": 1, "fp32": 1, "float32": 1,
         "bf16": 2, "bfloat16": 2, 0: 0, 1: 1, 2: 2}

_STATUS = {0: "TT_OK", 1: "TT_PENDING", -1: "TT_EINVAL", -2: "TT_ENOMEM", -3: "TT_ECAPACITY",
           -4: "TT_EDEVICE", -5: "TT_ENOTFOUND", -6: "TT_EUNSUPPORTED"}


class TTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


class _View(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("n", ctypes.POINTER(ctypes.c_int64)),
                ("ranks", ctypes.POINTER(ctypes.c_int64)),
                ("cores", ctypes.POINTER(ctypes.c_void_p))]


class _Out(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("ranks", ctypes.POINTER(ctypes.c_int64)),
                ("cores", ctypes.POINTER(ctypes.c_void_p)),
                ("capacity", ctypes.POINTER(ctypes.c_int64)), ("orth", ctypes.c_int32)]


class _Opts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("f_init", ctypes.c_double), ("nrmx", ctypes.c_double),
                ("recompress", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class _Info(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("nrmx", ctypes.c_double),
                ("min_margin", ctypes.c_double), ("passes", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("qr_retries", ctypes.c_int32),
                ("pc_launches", ctypes.c_int64), ("pc_bytes", ctypes.c_double),
                ("pc_flops", ctypes.c_double)]


class _ServerCfg(ctypes.Structure):
    _fields_ = [("mem_budget", ctypes.c_size_t), ("workers", ctypes.c_int32)]


class _Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("x", _View), ("tol", ctypes.c_double),
                ("ell_block", ctypes.c_int64), ("ell", ctypes.c_int64),
                ("target_ranks", ctypes.POINTER(ctypes.c_int64)), ("seed", ctypes.c_uint64),
                ("opts", _Opts)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("error", ctypes.c_char_p), ("d", ctypes.c_int32),
                ("ranks", ctypes.POINTER(ctypes.c_int64)), ("cores", ctypes.POINTER(ctypes.c_void_p)),
                ("orth", ctypes.c_int32), ("info", _Info), ("submit_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("done_s", ctypes.c_double)]


_lib = None


def lib():
    """Load libttround.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libttround.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2511_03598_amd.build); there is no fallback")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, u64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double
        P = ctypes.POINTER
        sig = {
            "tt_out_capacity": [P(_View), P(i64), P(i64)],
            "tt_round_fixed": [P(_View), P(i64), i64, u64, P(_Opts), P(_Out)],
            "tt_round_fixed_noalloc": [P(_View), P(i64), i64, u64, P(_Opts), P(_Out)],
            "tt_round_adaptive": [P(_View), dbl, i64, u64, P(_Opts), P(_Out)],
            "tt_round_ttsvd": [P(_View), dbl, P(i64), P(_Opts), P(_Out)],
            "tt_last_info": [P(_Info)],
            "tt_gaussian_factor": [u64, i32, i64, i64, i64, vp, vp],
            "tt_philox4x32_10": [vp, vp, vp, i64, vp],
            "tt_partial_contractions": [P(_View), u64, i64, i64, i32, ctypes.c_int, P(vp), vp],
            "tt_partial_contractions_lr": [P(_View), u64, i64, i64, i32, P(vp), vp],
            "tt_qr": [vp, i64, i64, vp],
            "tt_svd_small": [vp, i64, i64, vp, vp, vp, dbl, i64, P(i64), vp],
            "tt_kernel_timing": [i32],
            "tt_workspace_bytes": [P(_View), i64, ctypes.c_int, P(ctypes.c_size_t)],
            "tt_round_adaptive_batch": [P(_View), i32, P(dbl), i64, P(u64), P(_Opts), P(_Out)],
            "tt_batch_workspace_bytes": [P(_View), i32, i64, P(_Opts), P(ctypes.c_size_t)],
            "tt_batch_create": [P(_View), i32, P(dbl), i64, P(u64), P(_Opts), P(_Out), vp,
                                ctypes.c_size_t, P(vp)],
            "tt_batch_launch": [vp, vp],
            "tt_batch_finish": [vp, vp],
            "tt_batch_info": [vp, i32, P(_Info)],
            "tt_batch_team": [vp, i32, P(i32)],
            "tt_batch_record": [vp, i32, P(dbl), i32, P(i32)],
            "tt_batch_autotune": [P(_View), i32, P(dbl), i64, P(u64), P(_Opts), P(_Out), P(dbl), i32,
                                  P(dbl), P(dbl)],
            "tt_batch_team_flops": [dbl, P(dbl)],
            "tt_server_create": [P(_ServerCfg), P(vp)],
            "tt_round_submit": [vp, P(_Request), P(u64)],
            "tt_round_poll": [vp, u64, P(P(_Result))],
            "tt_round_wait": [vp, u64, P(P(_Result))],
            "tt_result_copy": [P(_Result), P(vp), vp],
            "tt_kernel_timing_read": [i32, P(i64), P(dbl)],
            "tt_sum_out_capacity": [P(_View), i32, P(i64), P(i64)],
            "tt_round_sum_fixed": [P(_View), i32, P(dbl), P(i64), i64, u64, P(_Opts), P(_Out)],
            "tt_round_sum_adaptive": [P(_View), i32, P(dbl), dbl, i64, u64, P(_Opts), P(_Out)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.tt_last_error.argtypes = []
        L.tt_last_error.restype = ctypes.c_char_p
        L.tt_result_release.argtypes = [P(_Result)]
        L.tt_result_release.restype = None
        L.tt_batch_destroy.argtypes = [vp]
        L.tt_batch_destroy.restype = None
        L.tt_server_destroy.argtypes = [vp]
        L.tt_server_destroy.restype = None
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise TTError(status, lib().tt_last_error().decode())


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class _ViewHolder:
    """Keeps the ctypes arrays of a tt_view alive."""

    def __init__(self, cores):
        torch = _torch()
        d = len(cores)
        if d < 2:
            raise ValueError("a TT needs d >= 2 cores")
        for c in cores:
            if c.dtype != torch.float64 or not c.is_cuda or c.dim() != 3 or not c.is_contiguous():
                raise ValueError("cores must be contiguous float64 CUDA tensors of rank 3")
        self.cores = cores
        self.dims = [int(c.shape[1]) for c in cores]
        self.ranks = [1] + [int(c.shape[2]) for c in cores]
        self.n_arr = (ctypes.c_int64 * d)(*self.dims)
        self.r_arr = (ctypes.c_int64 * (d + 1))(*self.ranks)
        self.p_arr = (ctypes.c_void_p * d)(*[c.data_ptr() for c in cores])
        self.view = _View(d, self.n_arr, self.r_arr, self.p_arr)


def out_capacity(cores):
    h = _ViewHolder(cores)
    d = len(cores)
    cap = (ctypes.c_int64 * d)()
    _check(lib().tt_out_capacity(ctypes.byref(h.view), None, cap))
    return list(cap)


def _run(cores, call):
    torch = _torch()
    h = _ViewHolder(cores)
    d = len(cores)
    caps = out_capacity(cores)
    bufs = [torch.empty(max(int(c), 1), dtype=torch.float64, device=cores[0].device) for c in caps]
    ranks = (ctypes.c_int64 * (d + 1))()
    ptrs = (ctypes.c_void_p * d)(*[b.data_ptr() for b in bufs])
    capa = (ctypes.c_int64 * d)(*caps)
    out = _Out(d, ranks, ptrs, capa, 0)
    _check(call(h, out))
    rk = list(ranks)
    res = [bufs[k][: rk[k] * h.dims[k] * rk[k + 1]].view(rk[k], h.dims[k], rk[k + 1])
           for k in range(d)]
    return res, {"ranks": rk, "orth": int(out.orth), **last_info()}


def _opts(prec, f_init, nrmx, recompress, stream):
    return _Opts(_PREC[prec], float(f_init or 0.0), float(nrmx or 0.0), int(recompress),
                 _stream(stream))


def round_fixed(cores, ell, seed, target_ranks=None, prec="f64", stream=None):
    """Fixed-rank Rand-Orth-KRP (sketch size ell), optionally truncated to
    target_ranks (list of d+1).  Returns (cores, info)."""
    d = len(cores)
    tg = None
    if target_ranks is not None:
        if len(target_ranks) != d + 1:
            raise ValueError("target_ranks needs d+1 entries")
        tg = (ctypes.c_int64 * (d + 1))(*[int(x) for x in target_ranks])
    o = _opts(prec, 0.0, 0.0, 0, stream)
    return _run(cores, lambda h, out: lib().tt_round_fixed(
        ctypes.byref(h.view), tg, int(ell), ctypes.c_uint64(seed), ctypes.byref(o),
        ctypes.byref(out)))


def round_fixed_noalloc(cores, ell, seed, target_ranks=None, prec="f64", stream=None):
    """round_fixed through the allocation-free entry point (the library's
    static scratch array instead of its workspace pool).  The output
    buffers are still allocated here by torch.  Returns (cores, info)."""
    d = len(cores)
    tg = None
    if target_ranks is not None:
        if len(target_ranks) != d + 1:
            raise ValueError("target_ranks needs d+1 entries")
        tg = (ctypes.c_int64 * (d + 1))(*[int(x) for x in target_ranks])
    o = _opts(prec, 0.0, 0.0, 0, stream)
    return _run(cores, lambda h, out: lib().tt_round_fixed_noalloc(
        ctypes.byref(h.view), tg, int(ell), ctypes.c_uint64(seed), ctypes.byref(o),
        ctypes.byref(out)))


def round_adaptive(cores, tol, ell_block, seed, nrmx=None, f_init=None, recompress=0, prec="f64",
                   stream=None):
    """Adaptive-rank Rand-Orth-KRP to relative tolerance tol.  Returns
    (cores, info)."""
    o = _opts(prec, f_init, nrmx, recompress, stream)
    return _run(cores, lambda h, out: lib().tt_round_adaptive(
        ctypes.byref(h.view), float(tol), int(ell_block), ctypes.c_uint64(seed),
        ctypes.byref(o), ctypes.byref(out)))


def round_ttsvd(cores, tol=None, target_ranks=None, stream=None):
    """Deterministic TT-SVD rounding (Sec. 2.3) to relative tolerance tol,
    or to target_ranks (d+1 list).  Returns (cores, info)."""
    if (tol is None) == (target_ranks is None):
        raise ValueError("give exactly one of tol or target_ranks")
    o = _opts("f64", None, None, 0, stream)
    tg = None if target_ranks is None else (ctypes.c_int64 * len(target_ranks))(*[int(t) for t in target_ranks])
    return _run(cores, lambda h, out: lib().tt_round_ttsvd(
        ctypes.byref(h.view), float(tol or 0.0), tg, ctypes.byref(o), ctypes.byref(out)))


class _SumHolder:
    """ctypes array of tt_view for a list of TTs (kept alive)."""

    def __init__(self, tts, weights):
        self.holders = [_ViewHolder(c) for c in tts]
        self.views = (_View * len(tts))(*[h.view for h in self.holders])
        self.count = len(tts)
        self.weights = None if weights is None else (ctypes.c_double * len(tts))(*[float(w) for w in weights])
        if weights is not None and len(weights) != len(tts):
            raise ValueError("one weight per term")


def sum_out_capacity(tts):
    h = _SumHolder(tts, None)
    d = len(tts[0])
    cap = (ctypes.c_int64 * d)()
    _check(lib().tt_sum_out_capacity(h.views, h.count, None, cap))
    return list(cap)


def _run_sum(tts, weights, call):
    torch = _torch()
    h = _SumHolder(tts, weights)
    d = len(tts[0])
    dims = h.holders[0].dims
    caps = sum_out_capacity(tts)
    bufs = [torch.empty(max(int(c), 1), dtype=torch.float64, device=tts[0][0].device) for c in caps]
    ranks = (ctypes.c_int64 * (d + 1))()
    ptrs = (ctypes.c_void_p * d)(*[b.data_ptr() for b in bufs])
    capa = (ctypes.c_int64 * d)(*caps)
    out = _Out(d, ranks, ptrs, capa, 0)
    _check(call(h, out))
    rk = list(ranks)
    res = [bufs[k][: rk[k] * dims[k] * rk[k + 1]].view(rk[k], dims[k], rk[k + 1]) for k in range(d)]
    return res, {"ranks": rk, "orth": int(out.orth), **last_info()}


def round_sum_fixed(tts, ell, seed, weights=None, target_ranks=None, prec="f64", stream=None):
    """Fixed-rank rounding of sum_i w_i X^(i) (tts: list of core lists), the
    terms sketched separately.  Returns (cores, info)."""
    d = len(tts[0])
    tg = None
    if target_ranks is not None:
        if len(target_ranks) != d + 1:
            raise ValueError("target_ranks needs d+1 entries")
        tg = (ctypes.c_int64 * (d + 1))(*[int(x) for x in target_ranks])
    o = _opts(prec, 0.0, 0.0, 0, stream)
    return _run_sum(tts, weights, lambda h, out: lib().tt_round_sum_fixed(
        h.views, h.count, h.weights, tg, int(ell), ctypes.c_uint64(seed), ctypes.byref(o),
        ctypes.byref(out)))


def round_sum_adaptive(tts, tol, ell_block, seed, weights=None, nrmx=None, f_init=None, recompress=0,
                       prec="f64", stream=None):
    """Adaptive rounding of sum_i w_i X^(i) to relative tolerance tol, the
    terms sketched separately.  Returns (cores, info)."""
    o = _opts(prec, f_init, nrmx, recompress, stream)
    return _run_sum(tts, weights, lambda h, out: lib().tt_round_sum_adaptive(
        h.views, h.count, h.weights, float(tol), int(ell_block), ctypes.c_uint64(seed),
        ctypes.byref(o), ctypes.byref(out)))


def last_info():
    i = _Info()
    _check(lib().tt_last_info(ctypes.byref(i)))
    return {"tau": i.tau, "nrmx": i.nrmx, "min_margin": i.min_margin, "passes": i.passes,
            "iterations": i.iterations, "qr_retries": i.qr_retries,
            "pc_launches": i.pc_launches, "pc_bytes": i.pc_bytes, "pc_flops": i.pc_flops}


def gaussian_factor(seed, mode, n, col0, ncols, device="cuda", stream=None):
    torch = _torch()
    out = torch.empty((n, ncols), dtype=torch.float64, device=device)
    _check(lib().tt_gaussian_factor(ctypes.c_uint64(seed), int(mode), int(n), int(col0),
                                    int(ncols), ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def philox4x32_10(ctr, key, stream=None):
    """ctr: int32 CUDA tensor (count, 4), key: int32 CUDA tensor (count, 2),
    both holding uint32 bit patterns.  Returns int32 (count, 4)."""
    torch = _torch()
    count = int(ctr.shape[0])
    out = torch.empty((count, 4), dtype=torch.int32, device=ctr.device)
    _check(lib().tt_philox4x32_10(ctypes.c_void_p(ctr.data_ptr()), ctypes.c_void_p(key.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), count, _stream(stream)))
    return out


def partial_contractions(cores, seed, col0, ncols, t=2, prec="f64", stream=None):
    """W_k for k = t..d (1-based) over sketch columns [col0, col0+ncols);
    returns a list [W_t, ..., W_d] of float64 (r_{k-1} x ncols) tensors."""
    torch = _torch()
    h = _ViewHolder(cores)
    d = len(cores)
    ws = [torch.empty((h.ranks[k - 1], ncols), dtype=torch.float64, device=cores[0].device)
          for k in range(t, d + 1)]
    arr = (ctypes.c_void_p * len(ws))(*[w.data_ptr() for w in ws])
    _check(lib().tt_partial_contractions(ctypes.byref(h.view), ctypes.c_uint64(seed), int(col0),
                                         int(ncols), int(t), _PREC[prec], arr, _stream(stream)))
    return ws


def partial_contractions_lr(cores, seed, col0, ncols, t=None, stream=None):
    """Left-to-right contractions W^L_1..W^L_t (t defaults to d) over sketch
    columns [col0, col0+ncols); returns a list of float64 (r_k x ncols)
    tensors, k = 1..t."""
    torch = _torch()
    h = _ViewHolder(cores)
    d = len(cores)
    t = d if t is None else int(t)
    # buffers for the k the library accepts; it rejects t outside [1, d]
    ws = [torch.empty((h.ranks[k], max(int(ncols), 0)), dtype=torch.float64, device=cores[0].device)
          for k in range(1, min(t, d) + 1)]
    arr = (ctypes.c_void_p * max(len(ws), 1))(*[w.data_ptr() for w in ws])
    _check(lib().tt_partial_contractions_lr(ctypes.byref(h.view), ctypes.c_uint64(seed), int(col0),
                                            int(ncols), int(t), arr, _stream(stream)))
    return ws


def svd_small(a, tau=-1.0, target=0, stream=None):
    """One-sided Jacobi SVD of a (p x q) float64 CUDA tensor, p >= q <= 512.
    Returns (G = U Sigma sorted, V, sigma, kept rank t)."""
    torch = _torch()
    p, q = a.shape
    buf = a.t().contiguous()
    g = torch.empty((q, p), dtype=torch.float64, device=a.device)
    v = torch.empty((q, q), dtype=torch.float64, device=a.device)
    sig = torch.empty(q, dtype=torch.float64, device=a.device)
    t = ctypes.c_int64()
    _check(lib().tt_svd_small(ctypes.c_void_p(buf.data_ptr()), int(p), int(q),
                              ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                              ctypes.c_void_p(sig.data_ptr()), float(tau), int(target),
                              ctypes.byref(t), _stream(stream)))
    return g.t(), v.t(), sig, int(t.value)


def qr(a, stream=None):
    """Thin QR (diag(R) >= 0) of an (m x b) float64 CUDA tensor; returns Q."""
    torch = _torch()
    m, b = a.shape
    buf = a.t().contiguous()  # column-major m x b
    _check(lib().tt_qr(ctypes.c_void_p(buf.data_ptr()), int(m), int(b), _stream(stream)))
    return buf.t()


KERNEL_KINDS = {"partial_contraction": 0, "gemm": 1, "qr": 2, "svd": 3}


def kernel_timing(enable, kinds=None):
    """Start (clearing the counters) or stop recording HIP events around the
    library's launches.  kinds: names from KERNEL_KINDS to record (default
    all); each recorded pair costs a little stream time, so a measurement
    that needs one kind should name only that kind."""
    mask = 0
    if enable:
        names = KERNEL_KINDS if kinds is None else kinds
        for k in names:
            mask |= 1 << KERNEL_KINDS[k]
    _check(lib().tt_kernel_timing(mask))


def kernel_timing_read(kind):
    """(launches, total milliseconds) recorded for a kind (name or id)."""
    k = KERNEL_KINDS[kind] if isinstance(kind, str) else int(kind)
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(lib().tt_kernel_timing_read(k, ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def workspace_bytes(cores, ell_max=0, prec="f64"):
    """Upper estimate of the device workspace of one rounding (ell_max > 0:
    fixed rank with that sketch size; <= 0: adaptive)."""
    h = _ViewHolder(cores)
    b = ctypes.c_size_t()
    _check(lib().tt_workspace_bytes(ctypes.byref(h.view), int(ell_max), _PREC[prec], ctypes.byref(b)))
    return int(b.value)


def round_adaptive_batch(tts, tol, ell_block, seeds, f_init=None, nrmx=None, recompress=0,
                         prec="f64", stream=None):
    """Adaptive rounding of many TTs (lists of cores) in one call; tol and
    seeds are scalars or per-tensor lists.  Returns a list of
    (cores, info) pairs (info has ranks and orth)."""
    torch = _torch()
    count = len(tts)
    tols = [float(tol)] * count if not hasattr(tol, "__len__") else [float(t) for t in tol]
    sds = [int(seeds)] * count if not hasattr(seeds, "__len__") else [int(x) for x in seeds]
    holders, outs, bufs, rk_arrays = [], [], [], []
    for cores in tts:
        h = _ViewHolder(cores)
        d = len(cores)
        caps = out_capacity(cores)
        b = [torch.empty(max(int(c), 1), dtype=torch.float64, device=cores[0].device) for c in caps]
        rk = (ctypes.c_int64 * (d + 1))()
        ptrs = (ctypes.c_void_p * d)(*[x.data_ptr() for x in b])
        capa = (ctypes.c_int64 * d)(*caps)
        holders.append((h, ptrs, capa))
        outs.append(_Out(d, rk, ptrs, capa, 0))
        bufs.append(b)
        rk_arrays.append(rk)
    views = (_View * count)(*[h[0].view for h in holders])
    out_arr = (_Out * count)(*outs)
    o = _opts(prec, f_init, nrmx, recompress, stream)
    _check(lib().tt_round_adaptive_batch(views, count, (ctypes.c_double * count)(*tols),
                                         int(ell_block), (ctypes.c_uint64 * count)(*sds),
                                         ctypes.byref(o), out_arr))
    res = []
    for i, cores in enumerate(tts):
        rk = [int(out_arr[i].ranks[k]) for k in range(len(cores) + 1)]
        dims = holders[i][0].dims
        ys = [bufs[i][k][: rk[k] * dims[k] * rk[k + 1]].view(rk[k], dims[k], rk[k + 1])
              for k in range(len(cores))]
        res.append((ys, {"ranks": rk, "orth": int(out_arr[i].orth)}))
    return res


def _batch_arrays(obj, tts, tol, seeds, f_init, nrmx, stream):
    """Marshal a batch (views, capacity-sized output buffers, tolerances,
    seeds, options) onto obj."""
    torch = _torch()
    obj.count = count = len(tts)
    tols = [float(tol)] * count if not hasattr(tol, "__len__") else [float(t) for t in tol]
    sds = [int(seeds)] * count if not hasattr(seeds, "__len__") else [int(x) for x in seeds]
    obj.tts = tts
    obj.holders, outs, obj.bufs = [], [], []
    for cores in tts:
        h = _ViewHolder(cores)
        d = len(cores)
        caps = out_capacity(cores)
        b = [torch.empty(max(int(c), 1), dtype=torch.float64, device=cores[0].device) for c in caps]
        rk = (ctypes.c_int64 * (d + 1))()
        ptrs = (ctypes.c_void_p * d)(*[x.data_ptr() for x in b])
        capa = (ctypes.c_int64 * d)(*caps)
        obj.holders.append((h, ptrs, capa, rk))
        outs.append(_Out(d, rk, ptrs, capa, 0))
        obj.bufs.append(b)
    obj.views = (_View * count)(*[h[0].view for h in obj.holders])
    obj.out_arr = (_Out * count)(*outs)
    obj.opts = _opts("f64", f_init, nrmx, 0, stream)
    obj.tol_arr = (ctypes.c_double * count)(*tols)
    obj.seed_arr = (ctypes.c_uint64 * count)(*sds)


BATCH_TUNE_CANDIDATES = (3e8, 1e9, 2e9, 2.5e9, 3e9, 1e10, 1e12)


def batch_autotune(tts, tol, ell_block, seeds, candidates=BATCH_TUNE_CANDIDATES, f_init=None, stream=None):
    """Time the persistent batch three times per candidate team threshold
    and make the candidate with the fastest median the device's
    (tt_batch_autotune).  Returns (best, {candidate: median ms})."""
    class _A:
        pass
    a = _A()
    _batch_arrays(a, tts, tol, seeds, f_init, None, stream)
    cands = [float(c) for c in candidates]
    carr = (ctypes.c_double * len(cands))(*cands)
    times = (ctypes.c_double * len(cands))()
    best = ctypes.c_double()
    _check(lib().tt_batch_autotune(a.views, a.count, a.tol_arr, int(ell_block), a.seed_arr,
                                   ctypes.byref(a.opts), a.out_arr, carr, len(cands), times,
                                   ctypes.byref(best)))
    return float(best.value), {c: float(t) for c, t in zip(cands, times)}


def batch_team_flops(value=0.0):
    """The device's team threshold of the persistent batch: value > 0 sets
    it, < 0 clears it, 0 only reads it."""
    cur = ctypes.c_double()
    _check(lib().tt_batch_team_flops(float(value), ctypes.byref(cur)))
    return float(cur.value)


class BatchPlan:
    """A batch of adaptive roundings laid out for the persistent kernel
    (tt_batch_create): the workspace and the output buffers are torch
    tensors owned by this object.  launch(stream) only enqueues kernels, so
    it may run under torch.cuda.graph capture and be replayed; finish()
    synchronises the stream and returns [(cores, info)] like
    round_adaptive_batch."""

    def __init__(self, tts, tol, ell_block, seeds, f_init=None, nrmx=None, stream=None):
        torch = _torch()
        _batch_arrays(self, tts, tol, seeds, f_init, nrmx, stream)
        count = self.count
        nbytes = ctypes.c_size_t()
        _check(lib().tt_batch_workspace_bytes(self.views, count, int(ell_block), ctypes.byref(self.opts),
                                              ctypes.byref(nbytes)))
        self.workspace = torch.empty(max(int(nbytes.value), 8), dtype=torch.uint8, device=tts[0][0].device)
        self.handle = ctypes.c_void_p()
        _check(lib().tt_batch_create(self.views, count, self.tol_arr, int(ell_block), self.seed_arr,
                                     ctypes.byref(self.opts), self.out_arr,
                                     ctypes.c_void_p(self.workspace.data_ptr()),
                                     ctypes.c_size_t(self.workspace.numel()), ctypes.byref(self.handle)))

    def records(self):
        """Raw run records (kBatchInfo doubles per tensor) after finish()."""
        import numpy as np
        out = []
        for i in range(self.count):
            buf = (ctypes.c_double * 64)()
            n = ctypes.c_int32()
            _check(lib().tt_batch_record(self.handle, i, buf, 64, ctypes.byref(n)))
            out.append(np.array(buf[: n.value]))
        return out

    def team(self, i):
        t = ctypes.c_int32()
        _check(lib().tt_batch_team(self.handle, int(i), ctypes.byref(t)))
        return int(t.value)

    def launch(self, stream=None):
        _check(lib().tt_batch_launch(self.handle, _stream(stream)))

    def finish(self, stream=None):
        _check(lib().tt_batch_finish(self.handle, _stream(stream)))
        res = []
        for i, cores in enumerate(self.tts):
            rk = [int(self.holders[i][3][k]) for k in range(len(cores) + 1)]
            dims = self.holders[i][0].dims
            ys = [self.bufs[i][k][: rk[k] * dims[k] * rk[k + 1]].view(rk[k], dims[k], rk[k + 1])
                  for k in range(len(cores))]
            info = _Info()
            _check(lib().tt_batch_info(self.handle, i, ctypes.byref(info)))
            res.append((ys, {"ranks": rk, "orth": 1, "tau": info.tau, "nrmx": info.nrmx,
                             "iterations": info.iterations, "passes": info.passes,
                             "min_margin": info.min_margin, "pc_launches": info.pc_launches,
                             "pc_bytes": info.pc_bytes, "pc_flops": info.pc_flops}))
        return res

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.tt_batch_destroy(h)
            self.handle = None


class Server:
    """Served rounding: submit requests (device-resident TT cores), poll
    for results.  Results are copied into torch tensors and the library's
    buffers released when a poll returns them."""

    def __init__(self, mem_budget=0, workers=8):
        self._h = ctypes.c_void_p()
        cfg = _ServerCfg(int(mem_budget), int(workers))
        _check(lib().tt_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))
        self._keep = {}

    def submit(self, cores, kind="adaptive", tol=1e-6, ell_block=0, ell=0, target_ranks=None,
               seed=0, prec="f64", f_init=None, nrmx=None, recompress=0):
        h = _ViewHolder(cores)
        d = len(cores)
        tg = None
        if target_ranks is not None:
            tg = (ctypes.c_int64 * (d + 1))(*[int(x) for x in target_ranks])
        o = _Opts(_PREC[prec], float(f_init or 0.0), float(nrmx or 0.0), int(recompress), None)
        req = _Request(0 if kind == "adaptive" else 1, h.view, float(tol), int(ell_block), int(ell),
                       tg, ctypes.c_uint64(seed), o)
        t = ctypes.c_uint64()
        _check(lib().tt_round_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._keep[int(t.value)] = (h, cores, tg)
        return int(t.value)

    def _collect(self, ticket, fn):
        torch = _torch()
        r = ctypes.POINTER(_Result)()
        st = fn(self._h, ctypes.c_uint64(ticket), ctypes.byref(r))
        if st == 1:
            return None
        _check(st)
        try:
            res = r.contents
            if res.status != 0:
                raise TTError(res.status, res.error.decode())
            d = res.d
            rk = [int(res.ranks[k]) for k in range(d + 1)]
            h = self._keep[ticket][0]
            ys = [torch.empty((rk[k], h.dims[k], rk[k + 1]), dtype=torch.float64, device="cuda")
                  for k in range(d)]
            dst = (ctypes.c_void_p * d)(*[t.data_ptr() for t in ys])
            _check(lib().tt_result_copy(r, dst, _stream(None)))
            info = {"ranks": rk, "orth": int(res.orth), "submit_s": res.submit_s,
                    "start_s": res.start_s, "done_s": res.done_s, "tau": res.info.tau,
                    "nrmx": res.info.nrmx}
            return ys, info
        finally:
            lib().tt_result_release(r)
            self._keep.pop(ticket, None)

    def poll(self, ticket):
        """(cores, info) when done, None while pending."""
        return self._collect(ticket, lib().tt_round_poll)

    def wait(self, ticket):
        return self._collect(ticket, lib().tt_round_wait)

    def close(self):
        if self._h:
            lib().tt_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
