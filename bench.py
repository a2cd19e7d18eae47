"""Benchmark: batched AM-QFT CDFT, 16384 signals of N = 4096, complex FP32.

One step = one forward transform of the whole batch (load, D_c/D_r, the
recursion's forward and backward phases, combine, store) by one kernel launch
through the C ABI.  Inputs are resident in HBM before the timed region.

Prints ONE JSON line (rank 0, one GPU):
  value      GFLOP/s in the 5 N log2 N convention for the headline variant
  roofline   HBM roofline of the transform kernel: algorithmic bytes per
             launch (read N points + write N points, 16 B per point) divided
             by the kernel's average launch duration (HIP events on the
             launch stream), against the 8 TB/s HBM peak of MI355X
  cpu_baseline  the FP64 CPU oracle timed on a bounded sample of the same
             workload on this host's cores (same 5 N log2 N convention)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "batched FFT GFLOP/s (5N log2N) + HBM GB/s, N=4096 fp32, plain vs fused"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def flops_5nlogn(n: int, batch: int) -> float:
    import math
    return 5.0 * n * math.log2(n) * batch


def time_launches(fn, steps: int, warmup: int, stream):
    """Average duration of each launch (events on the launch stream) and the
    wall time of the whole timed region."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) for a, b in evs]
    total = t0.elapsed_time(t1)
    per.sort()
    return {"avg_ms": sum(per) / len(per), "median_ms": per[len(per) // 2], "min_ms": per[0],
            "total_ms": total, "ms_per_step": total / steps}


def cpu_baseline(x_np, n: int, variant: int, target_s: float = 12.0):
    """Time the FP64 oracle on the first signals of the same workload."""
    import concurrent.futures as cf

    import numpy as np

    import oracle
    cores = os.cpu_count() or 1
    t = time.perf_counter()
    oracle.cdft(x_np[:2].astype(np.complex128), variant)
    per_sig = max((time.perf_counter() - t) / 2, 1e-6)
    sample = int(max(cores, min(len(x_np), target_s * cores / per_sig)))
    sample = min(sample, len(x_np))
    chunks = np.array_split(np.arange(sample), cores)
    xs = x_np[:sample].astype(np.complex128)

    def work(idx):
        if len(idx):
            oracle.cdft(xs[idx], variant)

    t = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(work, chunks))
    el = time.perf_counter() - t
    return {"value": flops_5nlogn(n, sample) / el / 1e9, "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "sample": "first %d signals of the workload (N=%d, FP64 recursive oracle, variant %d), %.1f s wall"
                      % (sample, n, variant, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", type=int, default=4)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true", help="time only the headline variant")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(signals shard across GPUs with no communication; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1404_1810_amd import api, inputs

    n, batch = args.n, args.batch
    log("generating %d x %d complex64 (seed %d)" % (batch, n, inputs.SEEDS["fp32_n4096"]))
    t0 = time.time()
    x = torch.empty((batch, n), dtype=torch.complex64, device="cuda")
    head_rows = min(batch, 4096)
    x_np = np.empty((head_rows, n), dtype=np.complex64)  # rows kept for the CPU checks
    for s0, rows in inputs.chunks("normal", inputs.SEEDS["fp32_n4096"], batch, n):
        r32 = rows.astype(np.complex64)
        x[s0:s0 + len(r32)].copy_(torch.from_numpy(r32))
        if s0 < head_rows:
            m = min(len(r32), head_rows - s0)
            x_np[s0:s0 + m] = r32[:m]
    torch.cuda.synchronize()
    log("inputs resident in HBM after %.1f s" % (time.time() - t0))
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    algo_bytes = batch * n * 16.0
    fl = flops_5nlogn(n, batch)

    results = {}
    variants = [args.variant] if args.no_variants else [args.variant] + [v for v in range(1, 9) if v != args.variant]
    for v in variants:
        plan = api.get_plan(n, batch, v, 1)
        r = time_launches(lambda: plan.exec(x, out=y), args.steps, args.warmup, stream)
        results[v] = r
        log("variant %d: avg %.4f ms  median %.4f ms  %.1f GFLOP/s  %.1f GB/s"
            % (v, r["avg_ms"], r["median_ms"], fl / r["avg_ms"] / 1e6, algo_bytes / r["avg_ms"] / 1e6))

    # spot check of the headline variant against the oracle (first 4 signals)
    head = results[args.variant]
    plan = api.get_plan(n, batch, args.variant, 1)
    plan.exec(x, out=y)
    torch.cuda.synchronize()
    import oracle
    ref = oracle.cdft(x_np[:4].astype(np.complex128), args.variant)
    got = y[:4].cpu().numpy()
    rel_err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    log("spot check rel L2 vs oracle: %.2e" % rel_err)

    achieved = algo_bytes / (head["avg_ms"] * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": round(fl / (head["ms_per_step"] * 1e-3) / 1e9, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch %d x N=%d complex64, re/im N(0,1) seed 0, forward, variant %d"
                               % (batch, n, args.variant),
                   "n": n, "batch": batch, "variant": args.variant, "layout": "interleaved, contiguous"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "amqft_lds_kernel<%d, float2>" % args.variant,
                     "algorithmic_bytes_per_launch": algo_bytes, "avg_launch_ms": round(head["avg_ms"], 5)},
        "rel_l2_vs_oracle": rel_err,
        "variants": {str(v): {"avg_ms": round(r["avg_ms"], 5),
                              "gflops": round(fl / r["avg_ms"] / 1e6, 1),
                              "hbm_gbs": round(algo_bytes / r["avg_ms"] / 1e6, 1)} for v, r in results.items()},
    }
    if not args.no_cpu:
        log("timing the CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(x_np, n, args.variant)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
