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
    # (event pairs on this stream around each partial-contraction launch and
    # around each GEMM, QR and SVD).
    ttr.kernel_timing(True)
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
                     "kernel": "partial contraction (pc_wide_kernel<float>)",
                     "bytes_per_launch": pc_bytes / npc, "avg_launch_us": avg_launch_s * 1e6},
        "kernel_ms_per_step": {k: v[1] / args.steps for k, v in kt.items()},
        "wall_s": wall,
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


if __name__ == "__main__":
    main()
