#!/usr/bin/env python
"""Benchmark: KRP-sketched adaptive TT-rounding on one MI355X.

Headline workload (default): the batch of 256 independent TT tensors (d
uniform in [4,16], n in [16,128], formal ranks in [8,128]; each a sum of 3
N(0,1) TTs weighted 1, 1e-4, 1e-8) rounded adaptively to tol 1e-6 with
blocks of 16 sketch columns, all in FP64, through the batch entry point.
A step is one rounding of the whole batch (every hot-path step of every
tensor) as one persistent kernel launch plus the readback of the ranks,
inputs resident in HBM and the batch laid out once beforehand; `value` is
tensors rounded per second over the timed steps.  Printed beside it, in one JSON line:

  * the plain single-instance rate (one tt_round_adaptive call after the
    other on one stream, same tensors and seeds; the same ranks, tensors
    equal to rounding error) and the rate of the synchronous batch call;
  * the same-GPU deterministic baseline: TT-SVD rounding (tt_round_ttsvd)
    to the same tolerance on a systematic sample of the batch, its rate and
    the batch's speed-up over it;
  * median / p10 / p90 of the step times;
  * sketch GB/s: the partial contractions' algorithmic bytes (one FP64
    read of each contracted core plus the W writes, every pass including
    the regeneration passes) over the batch's wall time;
  * `roofline`: the persistent batch kernel (the whole rounding of the
    batch in one launch) -- its algorithmic bytes and flops per launch (the
    partial contractions as run, a second read of every core for the
    next-core products, the output writes) over the launch duration timed
    with events on the launch stream;
  * the partial-contraction kernel at the two sizes where it is a large launch: the
    fixed-rank C2 rounding with an FP32 sketch (HBM-bound) and the adaptive
    C3 rounding with an FP64 sketch (FP64-MFMA-bound), with their rates,
    and the left-to-right contractions of C2 (FP64, ell 60);
  * parity of sampled tensors against the CPU oracle and their error
    against X;
  * `cpu_baseline`: the CPU oracle's KRP rounding (and its TT-SVD rounding)
    of a systematic sample of the batch on the host cores, with the thread
    count, and single-threaded.
Other workloads: --workload c2 | c5 | sum | precision | lr.
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
FP64_MFMA_PEAK_TFLOPS = 78.6
FP32_MFMA_PEAK_TFLOPS = 157.3
D, N, R, TERMS, ELL, TARGET, SEED = 20, 64, 50, 4, 60, 50, 42
C4_TOL, C4_BLOCK = 1e-6, 16
C3_TOL, C3_BLOCK, C3_SEED = 1e-6, 16, 42


def c2_desc():
    return ("fixed-rank KRP TT-rounding, X = sum of 4 random TTs (d=20, n=64, ranks 50, "
            "weights 1,1e-2,1e-4,1e-6; formal ranks 200), ell=60 -> target ranks 50, "
            "FP32 sketch + FP64 QR")


def c4_desc(count):
    return ("adaptive KRP TT-rounding of a batch of %d TTs (d in [4,16], n in [16,128], formal "
            "ranks in [8,128]; sums of 3 N(0,1) TTs weighted 1,1e-4,1e-8), tol 1e-6, ell blocks "
            "of 16, FP64, one batch call per step" % count)


def sketch_bytes(dims, ranks, ell, w_bytes):
    """Algorithmic bytes of one right-to-left partial-contraction pass over
    all of cores 2..d with ell columns: one FP64 read of the cores plus the
    W_k writes (Omega and W reads are negligible and not counted)."""
    d = len(dims)
    core = sum(ranks[k - 1] * dims[k - 1] * ranks[k] * 8 for k in range(2, d + 1))
    wout = sum(ranks[k - 1] * ell * w_bytes for k in range(2, d + 1))
    return core + wout


CSRC = os.path.join(ROOT, "paper_2511_03598_amd", "csrc")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "pc_kernel_c2_pmc.txt")
PC_SOURCES = [os.path.join(CSRC, "partial.hip")]
BATCH_PMC_SUMMARY = os.path.join(ROOT, "profiles", "batch_kernel_c4_pmc.txt")
BATCH_SOURCES = [os.path.join(CSRC, f) for f in ("batch.hip", "batch.hpp", "batch_host.cpp", "philox.hpp")]


def source_digest(paths):
    """sha256 over the kernel's source files, in order."""
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def pmc_traffic(path, sources=PC_SOURCES):
    """HBM bytes per launch from a committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, or None when there is none or the kernel's source
    changed since it was taken (the summary records source_sha256, the
    digest of `sources`)."""
    try:
        text = open(path).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != source_digest(sources) or "hbm_bytes_per_launch" not in vals:
        return None
    return float(vals["hbm_bytes_per_launch"])


def roofline(bytes_per_launch, flops_per_launch, avg_launch_s, flop_peak_tflops, kernel, traffic=None):
    """Roofline entry of one kernel: the bound is the one that gives the
    longer ideal time (HBM at 8 TB/s or the MFMA peak of its precision)."""
    t_hbm = bytes_per_launch / (HBM_PEAK_GBPS * 1e9)
    t_mfma = flops_per_launch / (flop_peak_tflops * 1e12)
    if t_hbm >= t_mfma:
        ach = bytes_per_launch / avg_launch_s / 1e9
        out = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
               "frac": ach / HBM_PEAK_GBPS}
    else:
        ach = flops_per_launch / avg_launch_s / 1e12
        out = {"bound": "mfma", "achieved": ach, "peak": flop_peak_tflops, "unit": "TFLOP/s",
               "frac": ach / flop_peak_tflops}
    out.update({"traffic": traffic, "kernel": kernel, "bytes_per_launch": bytes_per_launch,
                "flops_per_launch": flops_per_launch, "avg_launch_us": avg_launch_s * 1e6})
    return out


def pctl(vals, q):
    import numpy as np
    return float(np.percentile(np.asarray(vals, dtype=float), q))


def oracle_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count() or 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle work per CPU-baseline leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-side", action="store_true",
                    help="headline only: skip the C2 and C3 partial-contraction segments")
    ap.add_argument("--no-concurrent", action="store_true",
                    help="c2: skip the served-concurrency figure (profiling runs: it would mix "
                         "concurrent kernels into the per-kernel statistics)")
    ap.add_argument("--workload", choices=["c4", "c2", "c5", "sum", "precision", "lr"], default="c4",
                    help="c4 (default): the batch of 256 adaptive roundings at tol 1e-6 (FP64); "
                         "c2: the fixed-rank rounding with an FP32 sketch; c5: served rounding "
                         "under Poisson arrivals (p50/p99 latency); sum: one large C5 request "
                         "rounded term by term vs the assembled formal sum; precision: adaptive "
                         "rounding of C3 with FP64/FP32/BF16 sketches at tol 1e-4..1e-10; lr: the "
                         "left-to-right partial contractions of C2 (FP64, ell 60)")
    ap.add_argument("--count", type=int, default=256, help="c4: tensors in the batch")
    ap.add_argument("--team-flops", type=float, default=0.0,
                    help="c4: use this team threshold instead of autotuning (profiler runs)")
    ap.add_argument("--plain-reps", type=int, default=3, help="c4: repetitions of the plain loop")
    ap.add_argument("--ttsvd-sample", type=int, default=64,
                    help="c4: tensors (systematic sample) rounded by the GPU TT-SVD for its rate")
    ap.add_argument("--no-plain", action="store_true",
                    help="c4: skip the plain loop and the synchronous batch call (profiling runs)")
    ap.add_argument("--requests", type=int, default=500, help="c5: requests per arrival rate")
    ap.add_argument("--workers", type=int, default=8, help="c5: concurrent roundings")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (the "
                         "reference kernel that scales rocprofv3 FETCH_SIZE/WRITE_SIZE to bytes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": src.numel() * 8, "dispatches": 3}), flush=True)
        return
    if args.workload == "c4":
        return run_headline(args)
    if args.workload == "c5":
        return run_c5(args)
    if args.workload == "sum":
        return run_sum(args)
    if args.workload == "precision":
        return run_precision(args)
    if args.workload == "lr":
        return run_lr(args)
    return run_c2(args)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def batch_model(xs, res):
    """Algorithmic bytes and flops of the batch rounding (Sec. 3.1 cost
    model): the partial contractions as each tensor ran them (every pass,
    one float64 read of each contracted core and its W writes), one more
    float64 read of every core for the products with the next cores, the
    output writes, and the next-core products' flops."""
    b = f = 0.0
    for x, (y, info) in zip(xs, res):
        rk = info["ranks"]
        b += info["pc_bytes"] + sum(c.size for c in x) * 8.0 + sum(c.numel() for c in y) * 8.0
        f += info["pc_flops"]
        for k in range(1, len(x)):
            r0, n1, r1 = x[k].shape
            f += 2.0 * rk[k] * r0 * n1 * r1
    return b, f


def run_headline(args):
    import numpy as np
    import torch

    import paper_2511_03598_amd as ttr
    import ttgen

    t0 = time.perf_counter()
    xs = ttgen.c4(count=args.count)
    devs = [[torch.tensor(c, device="cuda") for c in x] for x in xs]
    seeds = [42 + t for t in range(len(xs))]
    log("generated and uploaded %d tensors in %.1f s" % (len(xs), time.perf_counter() - t0))

    # the device's team threshold tuned on this batch (set-up, untimed),
    # then the batch laid out once (descriptors uploaded); each step is one
    # persistent launch plus the readback of ranks and run records
    t1 = time.perf_counter()
    if args.team_flops > 0.0:
        tuned, tune_ms = ttr.batch_team_flops(args.team_flops), {}
    else:
        tuned, tune_ms = ttr.batch_autotune(devs, C4_TOL, C4_BLOCK, seeds)
    tune_s = time.perf_counter() - t1
    log("autotune: team threshold %.3g (%s) in %.1f s" % (tuned, tune_ms, tune_s))
    t1 = time.perf_counter()
    plan = ttr.BatchPlan(devs, C4_TOL, C4_BLOCK, seeds)
    plan_s = time.perf_counter() - t1
    for _ in range(max(1, args.warmup)):
        plan.launch()
        res = plan.finish()
    torch.cuda.synchronize()
    log("warm-up done")
    step_s, kern_ms = [], []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for _ in range(args.steps):
        t1 = time.perf_counter()
        ev0.record()
        plan.launch()
        ev1.record()
        res = plan.finish()
        step_s.append(time.perf_counter() - t1)
        kern_ms.append(ev0.elapsed_time(ev1))
    wall = time.perf_counter() - wall0
    log("timed %d batch steps: median %.3f s" % (args.steps, pctl(step_s, 50)))
    # the synchronous batch call (plan built inside every call)
    call_s = []
    for _ in range(0 if args.no_plain else 3):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ttr.round_adaptive_batch(devs, C4_TOL, C4_BLOCK, seeds)
        torch.cuda.synchronize()
        call_s.append(time.perf_counter() - t1)

    # plain single-instance loop (untimed for `value`)
    plain_s, plain = [], None
    for _ in range(0 if args.no_plain else max(1, args.plain_reps)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plain = [ttr.round_adaptive(devs[i], C4_TOL, C4_BLOCK, seeds[i]) for i in range(len(devs))]
        torch.cuda.synchronize()
        plain_s.append(time.perf_counter() - t1)
    ranks_equal = None if plain is None else all(p[1]["ranks"] == b[1]["ranks"] for p, b in zip(plain, res))
    # the same-GPU deterministic baseline: TT-SVD rounding (Sec. 2.3) to the
    # same tolerance, one call after the other, on a systematic sample
    ttsvd = None
    if not args.no_plain and args.ttsvd_sample > 0:
        sidx = c4_sample(len(xs), args.ttsvd_sample)
        ttr.round_ttsvd(devs[sidx[0]], tol=C4_TOL)  # warm-up
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sres = [ttr.round_ttsvd(devs[i], tol=C4_TOL) for i in sidx]
        torch.cuda.synchronize()
        svd_s = time.perf_counter() - t1
        krp_rank = sum(sum(res[i][1]["ranks"]) for i in sidx)
        svd_rank = sum(sum(r[1]["ranks"]) for r in sres)
        ttsvd = {"value": len(sidx) / svd_s, "tensors": len(sidx), "seconds": svd_s,
                 "rank_sum_krp_over_ttsvd": krp_rank / svd_rank,
                 "sample": "systematic, every %d-th tensor of the batch" % max(1, len(xs) // len(sidx))}
        log("TT-SVD: %d tensors in %.2f s" % (len(sidx), svd_s))
    # result of a sampled tensor alone vs in the batch (bitwise)
    j = len(xs) // 3
    alone = ttr.BatchPlan([devs[j]], C4_TOL, C4_BLOCK, [seeds[j]])
    alone.launch()
    (ya, ia), = alone.finish()
    alone_same = ia["ranks"] == res[j][1]["ranks"] and all(torch.equal(u, v) for u, v in zip(ya, res[j][0]))
    bytes_step, flops_step = batch_model(xs, res)
    pc_bytes = sum(r[1]["pc_bytes"] for r in res)
    step_total = sum(step_s)
    value = len(xs) * args.steps / step_total
    kern_s = pctl(kern_ms, 50) / 1e3
    out = {
        "metric": "TT-roundings/s + sketch GB/s vs plain & TT-SVD at rel err <=1e-6",
        "value": value,
        "unit": "TT-roundings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": c4_desc(len(xs)), "tensors": len(xs), "tol": C4_TOL,
                   "ell_block": C4_BLOCK, "sketch_precision": "f64",
                   "input_GB": sum(c.numel() * 8 for x in devs for c in x) / 1e9,
                   "launch": "one persistent kernel per step (graph-capturable), plan built once, " +
                             ("team threshold given" if args.team_flops > 0.0 else
                              "team threshold autotuned on the batch beforehand")},
        "step_s": {"median": pctl(step_s, 50), "p10": pctl(step_s, 10), "p90": pctl(step_s, 90),
                   "steps": args.steps},
        "kernel_ms": {"median": pctl(kern_ms, 50), "p10": pctl(kern_ms, 10), "p90": pctl(kern_ms, 90)},
        "plan_create_s": plan_s,
        "autotune": {"team_flops": tuned, "launch_ms": {"%g" % k: v for k, v in tune_ms.items()},
                     "seconds": tune_s,
                     "teams": [int(x) for x in np.bincount([plan.team(i) for i in range(len(xs))])]},
        "batch_call_value": len(xs) / pctl(call_s, 50) if call_s else None,
        "plain_value": len(xs) / pctl(plain_s, 50) if plain_s else None,
        "plain_step_s": {"median": pctl(plain_s, 50), "reps": len(plain_s)} if plain_s else None,
        "speedup_vs_plain": pctl(plain_s, 50) / pctl(step_s, 50) if plain_s else None,
        "ttsvd_value": ttsvd["value"] if ttsvd else None,
        "speedup_vs_ttsvd": value / ttsvd["value"] if ttsvd else None,
        "ttsvd": ttsvd,
        "ranks_equal_to_plain": ranks_equal,
        "alone_equals_in_batch": alone_same,
        "sketch_GBps": pc_bytes * args.steps / step_total / 1e9,
        "roofline": roofline(bytes_step, flops_step, kern_s, FP64_MFMA_PEAK_TFLOPS,
                             "persistent batched rounding (batch_kernel), whole rounding of the batch",
                             pmc_traffic(BATCH_PMC_SUMMARY, BATCH_SOURCES)),
        "wall_s": wall,
    }
    out["roofline"]["launches_per_step"] = 1
    if not args.no_side:
        out["side"] = {"c2_f32": side_c2(args), "c3_f64": side_c3(args), "c2_lr_f64": side_lr(args)}
    if not args.no_parity and plain is not None:
        out["parity"] = c4_parity(xs, res, seeds, plain)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = c4_cpu_baseline(xs, seeds, args.cpu_budget)
    print(json.dumps(out), flush=True)


def side_c2(args):
    """The partial contractions of the C2 fixed-rank rounding (FP32 sketch,
    200-row cores: the HBM-bound launch) and that rounding's rate."""
    import torch

    import paper_2511_03598_amd as ttr
    import ttgen

    x = ttgen.c2(d=D, n=N, r=R)
    dims = [c.shape[1] for c in x]
    ranks = [1] + [c.shape[2] for c in x]
    dev = [torch.tensor(c, device="cuda") for c in x]
    tgt = [1] + [TARGET] * (D - 1) + [1]
    for _ in range(max(1, args.warmup)):
        ttr.round_fixed(dev, ELL, SEED, target_ranks=tgt, prec="f32")
    torch.cuda.synchronize()
    ttr.kernel_timing(True, kinds=["partial_contraction"])
    times = []
    for _ in range(args.steps):
        t1 = time.perf_counter()
        y, info = ttr.round_fixed(dev, ELL, SEED, target_ranks=tgt, prec="f32")
        times.append(time.perf_counter() - t1)
    ttr.kernel_timing(False)
    n, ms = ttr.kernel_timing_read("partial_contraction")
    assert n == info["pc_launches"] * args.steps
    b = sketch_bytes(dims, ranks, ELL, 4)
    assert abs(b - info["pc_bytes"]) <= 1e-6 * b
    per = info["pc_launches"]
    return {"workload": c2_desc(), "roundings_per_s": 1.0 / pctl(times, 50),
            "roofline": roofline(b / per, info["pc_flops"] / per, ms / 1e3 / n, FP32_MFMA_PEAK_TFLOPS,
                                 "partial contraction, FP32 (pc_kernel<float>)",
                                 pmc_traffic(PMC_SUMMARY)),
            "sketch_GBps": b / (ms / 1e3 / args.steps) / 1e9, "ranks_max": max(info["ranks"])}


def side_c3(args):
    """The partial contractions of the adaptive C3 rounding (FP64 sketch,
    300-row cores of 256 x 300: FP64-MFMA-bound) and that rounding's rate."""
    import torch

    import paper_2511_03598_amd as ttr
    import ttgen

    x = ttgen.c3()
    dev = [torch.tensor(c, device="cuda") for c in x]
    del x
    steps = max(3, args.steps // 2)
    for _ in range(max(1, min(args.warmup, 2))):
        ttr.round_adaptive(dev, C3_TOL, C3_BLOCK, C3_SEED)
    torch.cuda.synchronize()
    ttr.kernel_timing(True, kinds=["partial_contraction"])
    times = []
    for _ in range(steps):
        t1 = time.perf_counter()
        y, info = ttr.round_adaptive(dev, C3_TOL, C3_BLOCK, C3_SEED)
        times.append(time.perf_counter() - t1)
    ttr.kernel_timing(False)
    n, ms = ttr.kernel_timing_read("partial_contraction")
    assert n == info["pc_launches"] * steps
    per = info["pc_launches"]
    return {"workload": "adaptive KRP TT-rounding of C3 (d=10, n=256, formal ranks 300), tol 1e-6, "
                        "ell blocks of 16, FP64 sketch", "roundings_per_s": 1.0 / pctl(times, 50),
            "roofline": roofline(info["pc_bytes"] / per, info["pc_flops"] / per, ms / 1e3 / n,
                                 FP64_MFMA_PEAK_TFLOPS, "partial contraction, FP64 (pc_kernel<double>)"),
            "sketch_GBps": info["pc_bytes"] / (ms / 1e3 / steps) / 1e9, "ranks": info["ranks"],
            "passes": info["passes"]}


def lr_model(x, ell):
    """Algorithmic bytes and flops of one left-to-right pass over every core:
    each core read once in FP64 and W^L_k (r_k x ell) written; the products
    2 r_{k-1} n_k r_k ell (the Khatri-Rao operand is formed in registers)."""
    b = sum(8 * c.shape[0] * c.shape[1] * c.shape[2] + 8 * c.shape[2] * ell for c in x)
    f = sum(2 * c.shape[0] * c.shape[1] * c.shape[2] * ell for c in x)
    return b, f


def side_lr(args):
    """The left-to-right partial contractions (Sec. 3.1, the recurrence run
    from the first core) of C2 with ell = 60 sketch columns in FP64, every
    core: passes per second and the kernel's roofline."""
    import torch

    import paper_2511_03598_amd as ttr
    import ttgen

    x = ttgen.c2(d=D, n=N, r=R)
    dev = [torch.tensor(c, device="cuda") for c in x]
    for _ in range(max(1, args.warmup)):
        ttr.partial_contractions_lr(dev, SEED, 0, ELL)
    torch.cuda.synchronize()
    ttr.kernel_timing(True, kinds=["partial_contraction"])
    times = []
    for _ in range(args.steps):
        t1 = time.perf_counter()
        ttr.partial_contractions_lr(dev, SEED, 0, ELL)
        times.append(time.perf_counter() - t1)
    ttr.kernel_timing(False)
    n, ms = ttr.kernel_timing_read("partial_contraction")
    per = len(x)  # one timed launch (contraction and slice sum) per core
    assert n == per * args.steps
    b, f = lr_model(x, ELL)
    return {"workload": "left-to-right KRP partial contractions W^L_1..W^L_20 of C2 (d=20, n=64, formal "
                        "ranks 200), ell=60, FP64", "passes_per_s": 1.0 / pctl(times, 50),
            "roofline": roofline(b / per, f / per, ms / 1e3 / n, FP64_MFMA_PEAK_TFLOPS,
                                 "left-to-right contraction, FP64 (lr_kernel and its in-order slice sum)"),
            "pass_ms_events": ms / args.steps}


def run_lr(args):
    out = side_lr(args)
    out.update({"steps": args.steps, "warmup": args.warmup})
    print(json.dumps(out), flush=True)


def c4_sample(count, k):
    """A systematic sample of k tensors of the batch (every count/k-th)."""
    step = max(1, count // k)
    return list(range(0, count, step))[:k]


def c4_parity(xs, res, seeds, plain):
    """Sampled tensors of the last batch step against the oracle (same
    Gaussian factors) and against the plain single-instance rounding:
    relative differences and ranks, and their error against X."""
    from oracle import krp, tt
    idx = c4_sample(len(xs), 6)
    diffs, dplain, errs, same = [], [], [], True
    for i in idx:
        yg = [c.cpu().numpy() for c in res[i][0]]
        yp = [c.cpu().numpy() for c in plain[i][0]]
        yo, io = krp.round_adaptive(xs[i], C4_TOL, C4_BLOCK, seeds[i])
        same = same and io["ranks"] == res[i][1]["ranks"]
        nx = tt.norm(xs[i])
        diffs.append(tt.diff_norm(yg, yo) / nx)
        dplain.append(tt.diff_norm(yg, yp) / nx)
        errs.append(tt.diff_norm(xs[i], yg) / nx)
    return {"tensors": idx, "max_rel_diff_vs_oracle": max(diffs), "ranks_equal": same,
            "max_rel_diff_vs_plain": max(dplain), "max_rel_err_vs_X": max(errs), "tol_vs_oracle": 1e-10,
            "tol_vs_X": C4_TOL}


def c4_cpu_baseline(xs, seeds, budget_s):
    """The oracle (plain NumPy/SciPy FP64) on a systematic sample of the
    batch: its KRP adaptive rounding (the same algorithm and Gaussian
    factors) and its TT-SVD rounding to the same tolerance, with the BLAS
    threads the host gives it, then single-threaded."""
    from oracle import krp, ttsvd
    try:
        from threadpoolctl import threadpool_limits
    except Exception:
        threadpool_limits = None
    order = c4_sample(len(xs), 64)

    def rate(fn, budget):
        fn(order[0])  # warm-up
        n, t0 = 0, time.perf_counter()
        for i in order:
            fn(i)
            n += 1
            if time.perf_counter() - t0 >= budget:
                break
        el = time.perf_counter() - t0
        return n / el, n, el

    krp_fn = lambda i: krp.round_adaptive(xs[i], C4_TOL, C4_BLOCK, seeds[i])
    svd_fn = lambda i: ttsvd.tt_svd_round(xs[i], tol=C4_TOL)
    threads = oracle_threads()
    v, n, el = rate(krp_fn, budget_s)
    sv, sn, sel = rate(svd_fn, budget_s / 2)
    out = {"value": v, "unit": "TT-roundings/s", "cores": int(threads), "kind": "oracle",
           "sample": "the first %d of a systematic sample (every %d-th tensor) of the batch, "
                     "KRP adaptive rounding, CPU FP64 NumPy oracle, %.1f s"
                     % (n, max(1, len(xs) // 64), el),
           "ttsvd_value": sv, "ttsvd_sample": "%d tensors, %.1f s" % (sn, sel)}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            v1, n1, el1 = rate(krp_fn, budget_s / 3)
            s1, sn1, sel1 = rate(svd_fn, budget_s / 6)
        out.update({"one_thread_value": v1, "one_thread_sample": "%d tensors, %.1f s" % (n1, el1),
                    "one_thread_ttsvd_value": s1,
                    "one_thread_ttsvd_sample": "%d tensors, %.1f s" % (sn1, sel1)})
    return out


def run_c2(args):
    """The fixed-rank C2 rounding with an FP32 sketch (the earlier headline
    workload), with the per-kind kernel breakdown and the served-concurrency
    figure."""
    import torch

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
    ttr.kernel_timing(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ttr.kernel_timing(False)
    kbreak = {k: ttr.kernel_timing_read(k)[1] / args.steps for k in ttr.KERNEL_KINDS}
    npc_launches, pc_ms = kt["partial_contraction"]
    npc = info["pc_launches"]
    assert npc_launches == npc * args.steps, (npc_launches, npc, args.steps)
    pc_bytes = sketch_bytes(dims, ranks, ELL, 4)
    avg_launch_s = pc_ms / 1e3 / npc_launches
    out = {
        "metric": "TT-roundings/s (fixed-rank C2, FP32 sketch)",
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
        "config": {"workload": c2_desc(), "d": D, "n": N, "formal_rank": R * TERMS,
                   "ell": ELL, "target_rank": TARGET, "seed": SEED},
        "sketch_GBps": pc_bytes / (pc_ms / 1e3 / args.steps) / 1e9,
        "roofline": roofline(pc_bytes / npc, info["pc_flops"] / npc, avg_launch_s,
                             FP32_MFMA_PEAK_TFLOPS, "partial contraction (pc_kernel<float>)",
                             pmc_traffic(PMC_SUMMARY)),
        "kernel_ms_per_step": kbreak,
        "wall_s": wall,
    }
    if not args.no_concurrent:
        srv = ttr.Server(workers=8)

        def submit():
            return srv.submit(dev, kind="fixed", ell=ELL, target_ranks=tgt, seed=SEED, prec="f32")
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
    log("c5 saturation: %d requests in %.2f s (%.2f/s)" % (nsat, t_sat, mu))
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
            if (i + 1) % 100 == 0:
                log("c5 lambda %.2f mu: %d of %d submitted" % (frac, i + 1, args.requests))
        for (t, ta) in pending:
            r = srv.wait(t)
            lat.append(r[1]["done_s"] - r[1]["submit_s"])
        wall = time.perf_counter() - t0
        log("c5 lambda %.2f mu done in %.1f s" % (frac, wall))
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
