#!/usr/bin/env python
"""Benchmark: KRP-sketched TT-rounding on one MI355X.

Workload (the configuration the metric is quoted on): fixed-rank
randomize-then-orthogonalize rounding with KRP sketches of
X = sum of 4 random TTs (d=20, n=64, ranks 50, N(0,1) cores) weighted
(1, 1e-2, 1e-4, 1e-6): formal ranks 200, sketch size ell=60, truncated to
target ranks 50.  Partial contractions (the sketch) in FP32 with FP32
accumulation; sketch GEMM, QR, projection, next core and truncation in FP64.

A step is one whole rounding of X (all hot-path steps), inputs resident in
HBM.  Prints one JSON line.  Also reported:
  * sketch GB/s and the roofline of the partial-contraction kernel
    (algorithmic bytes per launch / average launch duration, from HIP event
    pairs that the library records on this stream around every launch of
    that kernel during the timed steps);
  * the CPU oracle on the host cores (a bounded sample of full roundings);
  * parity of the last result against the oracle (relative to ||X||).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
D, N, R, TERMS, ELL, TARGET, SEED = 20, 64, 50, 4, 60, 50, 42


def workload_desc():
    return ("fixed-rank KRP TT-rounding, X = sum of 4 random TTs (d=20, n=64, ranks 50, "
            "weights 1,1e-2,1e-4,1e-6; formal ranks 200), ell=60 -> target ranks 50, "
            "FP32 sketch + FP64 QR")


def sketch_bytes(dims, ranks, ell, w_bytes):
    """Algorithmic bytes of one right-to-left partial-contraction pass:
    one FP64 read of cores 2..d plus the W_k writes (Omega, W reads are
    negligible and not counted)."""
    d = len(dims)
    core = sum(ranks[k - 1] * dims[k - 1] * ranks[k] * 8 for k in range(2, d + 1))
    wout = sum(ranks[k - 1] * ell * w_bytes for k in range(2, d + 1))
    return core + wout


PMC_SUMMARY = os.path.join(ROOT, "profiles", "pc_kernel_c2_pmc.txt")
PC_SOURCE = os.path.join(ROOT, "paper_2511_03598_amd", "csrc", "partial.hip")


def pmc_traffic(alg_bytes_per_launch):
    """HBM bytes per partial-contraction launch from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when there is none or the
    kernel source changed since it was taken (the summary records the
    source's sha256)."""
    import hashlib
    try:
        text = open(PMC_SUMMARY).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    src = hashlib.sha256(open(PC_SOURCE, "rb").read()).hexdigest()
    if vals.get("source_sha256") != src or "hbm_bytes_per_launch" not in vals:
        return None
    return float(vals["hbm_bytes_per_launch"])


def cpu_baseline(x, budget_s):
    from oracle import krp
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    tgt = [1] + [TARGET] * (D - 1) + [1]
    krp.round_fixed(x, ELL, SEED, tgt)  # warm-up
    n, t0 = 0, time.perf_counter()
    while True:
        krp.round_fixed(x, ELL, SEED, tgt)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 50:
            break
    return {"value": n / el, "unit": "TT-roundings/s", "cores": int(threads), "kind": "oracle",
            "sample": "%d full roundings of the same workload (CPU FP64 NumPy oracle, %.1f s)" % (n, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-concurrent", action="store_true",
                    help="skip the served-concurrency figure (profiling runs: it would mix "
                         "concurrent kernels into the per-kernel statistics)")
    ap.add_argument("--workload", choices=["c2", "c4", "c5", "sum", "precision"], default="c2",
                    help="c2 (default): the fixed-rank rounding the metric is quoted on; "
                         "c4: batched adaptive rounding vs a plain loop; c5: served rounding "
                         "under Poisson arrivals (p50/p99 latency); sum: one large C5 request "
                         "rounded term by term vs the assembled formal sum; precision: adaptive "
                         "rounding of C3 with FP64/FP32/BF16 sketches at tol 1e-4..1e-10")
    ap.add_argument("--count", type=int, default=256, help="c4: tensors in the batch")
    ap.add_argument("--requests", type=int, default=120, help="c5: requests per arrival rate")
    ap.add_argument("--workers", type=int, default=8, help="c4/c5: concurrent roundings")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (the "
                         "reference kernel that scales rocprofv3 FETCH_SIZE/WRITE_SIZE to bytes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the design notes "
              "describe how it would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.workload == "c4":
        return run_c4(args)
    if args.workload == "c5":
        return run_c5(args)
    if args.workload == "sum":
        return run_sum(args)
    if args.workload == "precision":
        return run_precision(args)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": src.numel() * 8, "dispatches": 3}), flush=True)
        return

    import paper_2511_03598_amd as ttr
    import ttgen

    x = ttgen.c2(d=D, n=N, r=R)
    dims = [c.shape[1] for c in x]
    ranks = [1] + [c.shape[2] for c in x]
    dev = [torch.tensor(c, device="cuda") for c in x]
    tgt = [1] + [TARGET] * (D - 1) + [1]
    stream = torch.cuda.current_stream()

    def step():
        return ttr.round_fixed(dev, ELL, SEED, target_ranks=tgt, prec="f32", stream=stream)

    for _ in range(args.warmup):
        y, info = step()
    torch.cuda.synchronize()
    # Timed region: K whole roundings, with the library's HIP-event timers on
    # around each partial-contraction launch only (the roofline's launch
    # duration); the breakdown over all kernel kinds comes from a separate
    # untimed pass, since event pairs around every GEMM, QR and SVD add about
    # a tenth to the rounding time.
    ttr.kernel_timing(True, kinds=["partial_contraction"])
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        y, info = step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ttr.kernel_timing(False)
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    value = args.steps / (gpu_ms / 1e3)
    kt = {k: ttr.kernel_timing_read(k) for k in ttr.KERNEL_KINDS}
    # per-kind breakdown (untimed pass with every kind's timers on)
    ttr.kernel_timing(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ttr.kernel_timing(False)
    kbreak = {k: ttr.kernel_timing_read(k)[1] / args.steps for k in ttr.KERNEL_KINDS}

    # Roofline of the partial-contraction kernel: algorithmic bytes of one
    # pass / launches per pass, over the average recorded launch duration.
    npc_launches, pc_ms = kt["partial_contraction"]
    npc = D - 1
    assert npc_launches == npc * args.steps, (npc_launches, npc, args.steps)
    pc_bytes = sketch_bytes(dims, ranks, ELL, 4)
    avg_launch_s = pc_ms / 1e3 / npc_launches
    achieved = pc_bytes / npc / avg_launch_s / 1e9
    sketch_gbps = pc_bytes / (pc_ms / 1e3 / args.steps) / 1e9
    traffic = pmc_traffic(pc_bytes / npc)

    out = {
        "metric": "TT-roundings/s + sketch GB/s vs plain & TT-SVD at rel err <=1e-6",
        "value": value,
        "unit": "TT-roundings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 sketch / f64 sweep",
        "data": "synthetic",
        "config": {"workload": workload_desc(), "d": D, "n": N, "formal_rank": R * TERMS,
                   "ell": ELL, "target_rank": TARGET, "seed": SEED},
        "sketch_GBps": sketch_gbps,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": "partial contraction (pc_kernel<float>)",
                     "bytes_per_launch": pc_bytes / npc, "avg_launch_us": avg_launch_s * 1e6},
        "kernel_ms_per_step": kbreak,
        "wall_s": wall,
    }
    # Headroom beyond one stream: a single rounding is latency-bound (its
    # SVDs and QR factorisations each run on one CU), so the same rounding
    # is also submitted 32 times to the library's server (8 workers, one HIP
    # stream each).  Reported beside `value`, which stays the one-stream rate.
    if args.no_concurrent:
        srv = None
    else:
        srv = ttr.Server(workers=8)
    def submit():
        return srv.submit(dev, kind="fixed", ell=ELL, target_ranks=tgt, seed=SEED, prec="f32")
    if srv is not None:
        for t in [submit() for _ in range(8)]:
            srv.wait(t)
        nreq = 32
        t0 = time.perf_counter()
        tks = [submit() for _ in range(nreq)]
        served = [srv.wait(t) for t in tks]
        conc_s = time.perf_counter() - t0
        srv.close()
        out["concurrent"] = {
            "roundings_per_s": nreq / conc_s, "requests": nreq, "workers": 8,
            "bitwise_equal_to_one_stream": all(torch.equal(u, v) for u, v in zip(served[-1][0], y)),
        }
    if not args.no_parity:
        from oracle import krp, tt
        yo, io = krp.round_fixed(x, ELL, SEED, tgt)
        yh = [c.cpu().numpy() for c in y]
        nx = tt.norm(x)
        out["parity"] = {"rel_diff_vs_oracle": tt.diff_norm(yh, yo) / nx,
                         "ranks_equal": info["ranks"] == io["ranks"], "tol": 1e-5}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(x, args.cpu_budget)
    print(json.dumps(out), flush=True)


def run_c4(args):
    """Batched adaptive rounding (tol 1e-6, ell blocks of 16) of `count`
    independent TTs of uneven d, n and ranks, against the plain loop of
    single calls on one stream.  Both produce bitwise the same results."""
    import torch

    import paper_2511_03598_amd as ttr
    import ttgen
    from oracle import tt

    t0 = time.perf_counter()
    xs = ttgen.c4(count=args.count)
    gen_s = time.perf_counter() - t0
    devs = [[torch.tensor(c, device="cuda") for c in x] for x in xs]
    seeds = [42 + t for t in range(len(xs))]
    tol, blk = 1e-6, 16
    nbytes = sum(c.numel() * 8 for x in devs for c in x)
    # warm-up (workspaces, code objects)
    ttr.round_adaptive_batch(devs[:8], tol, blk, seeds[:8])
    for i in range(4):
        ttr.round_adaptive(devs[i], tol, blk, seeds[i])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [ttr.round_adaptive(devs[i], tol, blk, seeds[i]) for i in range(len(devs))]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    batch = ttr.round_adaptive_batch(devs, tol, blk, seeds)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    same = all(p[1]["ranks"] == b[1]["ranks"] and all(torch.equal(u, v) for u, v in zip(p[0], b[0]))
               for p, b in zip(plain, batch))
    sample = list(range(0, len(xs), max(1, len(xs) // 6)))[:6]
    errs = [tt.rel_err(xs[i], [c.cpu().numpy() for c in batch[i][0]]) for i in sample]
    out = {
        "metric": "TT-roundings/s (batched, C4)", "value": len(xs) / t_batch,
        "unit": "TT-roundings/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
        "config": {"workload": "C4: %d TTs, d in [4,16], n in [16,128], formal ranks in [8,128], "
                               "sum of 3 N(0,1) TTs weighted (1, 1e-4, 1e-8), adaptive tol 1e-6, "
                               "ell blocks of 16, FP64" % len(xs),
                   "workers": 8, "input_GB": nbytes / 1e9},
        "plain_loop_value": len(xs) / t_plain, "speedup_vs_plain": t_plain / t_batch,
        "batch_s": t_batch, "plain_s": t_plain, "bitwise_equal_to_plain": same,
        "rel_err_sample": {"tensors": sample, "max": max(errs)}, "generate_s": gen_s,
    }
    print(json.dumps(out), flush=True)


def run_sum(args):
    """Rounding of a sum of TTs: one large C5 request (8 terms, d=30, n=32,
    ranks 50, coefficients g_i 10^-i; formal ranks 400), adaptive to tol
    1e-6 with ell blocks of 20, FP64.  The terms sketched separately
    (tt_round_sum_adaptive) against the rounding of the assembled formal sum
    (tt_round_adaptive) with the same seed: rates, kernel time per kind, and
    the difference between the two results."""
    import torch

    import numpy as np

    import paper_2511_03598_amd as ttr
    import ttgen

    tts, coef = ttgen.c5_terms(2000)
    dev_terms = [[torch.tensor(c, device="cuda") for c in x] for x in tts]
    dev_formal = [torch.tensor(c, device="cuda") for c in ttgen.formal_sum(tts, coef)]
    tol, blk, seed = 1e-6, 20, 7

    def run(kind):
        if kind == "sum":
            return ttr.round_sum_adaptive(dev_terms, tol, blk, seed, weights=coef)
        return ttr.round_adaptive(dev_formal, tol, blk, seed)

    res, timing = {}, {}
    for kind in ("sum", "formal"):
        for _ in range(max(1, args.warmup)):
            run(kind)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = run(kind)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        ttr.kernel_timing(True)  # breakdown in a separate pass
        for _ in range(args.steps):
            run(kind)
        torch.cuda.synchronize()
        ttr.kernel_timing(False)
        kms = {k: ttr.kernel_timing_read(k)[1] / args.steps for k in ttr.KERNEL_KINDS}
        res[kind] = out
        timing[kind] = {"s_per_rounding": dt, "kernel_ms_per_rounding": kms}
    ys = [c.cpu().numpy() for c in res["sum"][0]]
    yf = [c.cpu().numpy() for c in res["formal"][0]]
    # entries at 256 random multi-indices (a chain of small products each)
    rng = np.random.default_rng(11)
    idx = rng.integers(0, 32, size=(256, len(ys)))

    def entries(cs):
        v = np.ones((idx.shape[0], 1))
        for k, c in enumerate(cs):
            v = np.einsum("sa,sab->sb", v, c[:, idx[:, k], :].transpose(1, 0, 2))
        return v[:, 0]

    es, ef = entries(ys), entries(yf)
    entry_diff = float(np.max(np.abs(es - ef)) / np.max(np.abs(ef)))
    t_sum, t_formal = timing["sum"]["s_per_rounding"], timing["formal"]["s_per_rounding"]
    out = {
        "metric": "TT-roundings/s (sum of TTs, terms sketched separately)", "value": 1.0 / t_sum,
        "unit": "TT-roundings/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "higher_is_better": True, "data": "synthetic", "dtype": "f64",
        "config": {"workload": "C5 large request: sum of 8 TTs d=30 n=32 ranks 50 (formal 400), "
                               "coefficients g_i 10^-i, adaptive tol 1e-6, ell blocks of 20, FP64"},
        "formal_sum_value": 1.0 / t_formal, "speedup_vs_formal_sum": t_formal / t_sum,
        "ranks_sum": res["sum"][1]["ranks"], "ranks_formal": res["formal"][1]["ranks"],
        "same_ranks": res["sum"][1]["ranks"] == res["formal"][1]["ranks"],
        "max_entry_diff_sum_vs_formal": entry_diff, "entries_sampled": int(idx.shape[0]),
        "timing": timing,
    }
    print(json.dumps(out), flush=True)


def run_precision(args):
    """Adaptive rounding of C3 (d=10, n=256, base ranks 200 with bond
    spectra 10^-(j-1)/8, plus a noise TT of ranks 100; formal ranks 300) with
    the sketch (W) kept in FP64, FP32 or BF16, at tol 1e-4 .. 1e-10 (ell
    blocks of 16): rate, ranks, range-finder iterations, regeneration passes
    and partial-contraction time per precision.  The error against X is
    measured on a reduced C3 (d=6, n=64, ranks 100 + 50) with the oracle's
    TT norms.  The estimator and the sweep run in FP64 from S = V(Y_k) W, so
    a reduced-precision W only perturbs the test matrix; whether it ever
    stalls the adaptive loop is what this run checks."""
    import torch

    import paper_2511_03598_amd as ttr
    import ttgen
    from oracle import tt as ott

    tols = (1e-4, 1e-6, 1e-8, 1e-10)
    precs = ("f64", "f32", "bf16")
    big = [torch.tensor(c, device="cuda") for c in ttgen.c3()]
    small_h = ttgen.c3(d=6, n=64, r=100, noise_r=50)
    small = [torch.tensor(c, device="cuda") for c in small_h]
    rows = []
    for tol in tols:
        for prec in precs:
            for _ in range(max(1, args.warmup)):
                ttr.round_adaptive(big, tol, 16, 42, prec=prec)
            torch.cuda.synchronize()
            ttr.kernel_timing(True, kinds=["partial_contraction"])
            t0 = time.perf_counter()
            for _ in range(args.steps):
                y, info = ttr.round_adaptive(big, tol, 16, 42, prec=prec)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
            ttr.kernel_timing(False)
            pc_ms = ttr.kernel_timing_read("partial_contraction")[1] / args.steps
            ys, infos = ttr.round_adaptive(small, tol, 16, 42, prec=prec)
            err = float(ott.rel_err(small_h, [c.cpu().numpy() for c in ys]))
            rows.append({"tol": tol, "prec": prec, "roundings_per_s": 1.0 / dt,
                         "ranks": info["ranks"], "iterations": info["iterations"],
                         "passes": info["passes"], "partial_contraction_ms": pc_ms,
                         "reduced_c3_ranks": infos["ranks"], "reduced_c3_rel_err": err})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    same = all(r["ranks"] == next(q["ranks"] for q in rows if q["tol"] == r["tol"] and q["prec"] == "f64")
               and r["iterations"] == next(q["iterations"] for q in rows
                                           if q["tol"] == r["tol"] and q["prec"] == "f64")
               for r in rows)
    within = all(r["reduced_c3_rel_err"] <= r["tol"] for r in rows)
    bf = next(r for r in rows if r["tol"] == 1e-8 and r["prec"] == "bf16")
    out = {
        "metric": "adaptive TT-roundings/s (C3, BF16 sketch, tol 1e-8)", "value": bf["roundings_per_s"],
        "unit": "TT-roundings/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "higher_is_better": True, "data": "synthetic", "dtype": "bf16/f32/f64 sketch, f64 sweep",
        "config": {"workload": "C3: d=10 n=256 base ranks 200 (spectra 10^-(j-1)/8) + noise TT ranks "
                               "100 (sigma 1e-6), formal ranks 300; adaptive, ell blocks of 16"},
        "same_ranks_and_iterations_all_precisions": same, "errors_within_tol": within,
        "rows": rows,
    }
    print(json.dumps(out), flush=True)


def run_c5(args):
    """Served rounding: requests are weighted sums of 8 TTs (d=30, n=32,
    ranks 50: formal ranks 400) mixed with 20% small ones (d=8, n=16, ranks
    20), rounded adaptively to tol 1e-6 (ell blocks of 20).  The inputs stay
    on the device (a pool of distinct tensors that requests draw from).
    First the saturation throughput mu (all requests queued at once), then
    Poisson arrivals at lambda = (0.25, 0.5, 0.75, 0.9) mu: p50/p99 of
    completion minus arrival, and the achieved throughput."""
    import numpy as np
    import torch

    import paper_2511_03598_amd as ttr
    import ttgen

    rng = np.random.default_rng(5000)
    pool_large = [[torch.tensor(c, device="cuda") for c in ttgen.c5_request(2000 + i)] for i in range(3)]
    pool_small = [[torch.tensor(c, device="cuda") for c in ttgen.c5_request(3000 + i, small=True)]
                  for i in range(3)]
    srv = ttr.Server(workers=args.workers)

    def pick(k):
        small = rng.random() < 0.2
        pool = pool_small if small else pool_large
        return pool[k % len(pool)], small

    def submit(x, seed):
        return srv.submit(x, tol=1e-6, ell_block=20, seed=seed)

    # warm-up and the alone-vs-mix spot check
    ref = ttr.round_adaptive(pool_large[0], 1e-6, 20, 7)
    w = srv.wait(submit(pool_large[0], 7))
    same = w[0][0].shape == ref[0][0].shape and all(torch.equal(a, b) for a, b in zip(w[0], ref[0]))
    srv.wait(submit(pool_small[0], 8))
    # saturation
    nsat = max(16, args.requests // 4)
    t0 = time.perf_counter()
    tk = [submit(pick(i)[0], 100 + i) for i in range(nsat)]
    res = [srv.wait(t) for t in tk]
    t_sat = time.perf_counter() - t0
    mu = nsat / t_sat
    runs = []
    for frac in (0.25, 0.5, 0.75, 0.9):
        lam = frac * mu
        gaps = rng.exponential(1.0 / lam, size=args.requests)
        pending, lat, nsmall = [], [], 0
        t0 = time.perf_counter()
        tnext = t0
        for i in range(args.requests):
            tnext += gaps[i]
            while True:
                now = time.perf_counter()
                if now >= tnext:
                    break
                # collect finished requests while waiting for the next arrival
                still = []
                for (t, ta) in pending:
                    r = srv.poll(t)
                    if r is None:
                        still.append((t, ta))
                    else:
                        lat.append(r[1]["done_s"] - r[1]["submit_s"])
                pending = still
                time.sleep(min(0.0005, max(0.0, tnext - now)))
            x, small = pick(i)
            nsmall += small
            pending.append((submit(x, 1000 + i), tnext))
        for (t, ta) in pending:
            r = srv.wait(t)
            lat.append(r[1]["done_s"] - r[1]["submit_s"])
        wall = time.perf_counter() - t0
        lat = np.sort(np.array(lat))
        runs.append({"lambda_frac": frac, "lambda_per_s": lam, "requests": args.requests,
                     "small": nsmall, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                     "p99_ms": float(np.percentile(lat, 99) * 1e3),
                     "throughput_per_s": args.requests / wall})
    srv.close()
    out = {"metric": "served TT-roundings/s and p50/p99 latency (C5)", "value": mu,
           "unit": "TT-roundings/s (saturation)", "n_gpus": 1, "higher_is_better": True,
           "data": "synthetic",
           "config": {"workload": "C5: 80% sums of 8 TTs (d=30, n=32, ranks 50, coefficients "
                                  "g_i 10^-i; formal ranks 400), 20% small (d=8, n=16, ranks 20 x 8), "
                                  "adaptive tol 1e-6, ell blocks of 20, FP64", "workers": args.workers},
           "saturation": {"requests": nsat, "seconds": t_sat},
           "poisson": runs, "alone_equals_mix": same}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
