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
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1404_1810_amd", "csrc")
# sources each kernel family is built from (a traffic measurement is valid
# only for the exact sources it was taken on)
KERNEL_SOURCES = {
    "amqft_a4096_kernel": ["amqft_k4096.hip", "amqft_leaf.h", "amqft_device.h"],
    "amqft_fast_kernel": ["amqft_fast.hip", "amqft_levels.h", "amqft_leaf.h", "amqft_device.h"],
    "amqft_lds_kernel": ["amqft_lds.hip", "amqft_levels.h", "amqft_device.h"],
}
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


def kernel_family(desc: str) -> str:
    return desc.split("<", 1)[0].split()[0]


def sources_digest(family: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(family, []):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def traffic_file(family: str, variant: int, n: int, batch: int) -> str:
    return os.path.join(PROFILES, "traffic_%s_v%d_fp32_n%d_b%d.json" % (family, variant, n, batch))


def load_traffic(family: str, variant: int, n: int, batch: int):
    """HBM bytes per launch from the committed counter summary, or None when
    there is none or the kernel's sources changed since it was taken."""
    path = traffic_file(family, variant, n, batch)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("sources_sha256_16") != sources_digest(family):
        log("traffic record %s is stale (kernel sources changed): traffic = null" % os.path.basename(path))
        return None
    return rec


def _pmc_per_dispatch(csv_path: str, counter: str, kernel_sub: str):
    import csv
    vals = {}
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter or kernel_sub not in row.get("Kernel_Name", ""):
                continue
            d = row.get("Dispatch_Id") or row.get("Correlation_Id")
            vals[d] = vals.get(d, 0.0) + float(row["Counter_Value"])
    if not vals:
        raise SystemExit("no %s rows for kernels matching %r in %s" % (counter, kernel_sub, csv_path))
    v = sorted(vals.values())
    return v[len(v) // 2], len(v)


def ingest_pmc(args, fetch_csv, write_csv, copy_fetch_csv, copy_write_csv):
    """Turn four rocprofv3 --pmc counter files (FETCH_SIZE and WRITE_SIZE of
    the transform run and of the --copy-calibration run) into the traffic
    record bench.py reports.  Counters are KiB per dispatch; each is scaled by
    the factor that maps the copy kernel's reading to its known byte count."""
    from paper_1404_1810_amd import api  # noqa: F401  (plan description needs the library)
    n, batch = args.n, args.batch
    desc = args.kernel_desc
    family = kernel_family(desc)
    fk, nd = _pmc_per_dispatch(fetch_csv, "FETCH_SIZE", family)
    wk, _ = _pmc_per_dispatch(write_csv, "WRITE_SIZE", family)
    fc, _ = _pmc_per_dispatch(copy_fetch_csv, "FETCH_SIZE", "elementwise")
    wc, _ = _pmc_per_dispatch(copy_write_csv, "WRITE_SIZE", "elementwise")
    copy_bytes = batch * n * 8.0
    f_read = copy_bytes / (fc * 1024.0)
    f_write = copy_bytes / (wc * 1024.0)
    read_b = fk * 1024.0 * f_read
    write_b = wk * 1024.0 * f_write
    rec = {"kernel": desc, "variant": args.variant, "n": n, "batch": batch,
           "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk, "dispatches": nd,
           "copy_fetch_kib": fc, "copy_write_kib": wc, "copy_bytes_each_way": copy_bytes,
           "read_scale": f_read, "write_scale": f_write,
           "traffic_bytes_per_launch": read_b + write_b,
           "algorithmic_bytes_per_launch": batch * n * 16.0,
           "traffic_over_algorithmic": (read_b + write_b) / (batch * n * 16.0),
           "sources_sha256_16": sources_digest(family)}
    os.makedirs(PROFILES, exist_ok=True)
    path = traffic_file(family, args.variant, n, batch)
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec))


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
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain elementwise copy (torch.neg) of the workload's size, for "
                         "calibrating the HBM byte counters")
    ap.add_argument("--ingest-pmc", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write the traffic record from rocprofv3 counter files (no GPU work)")
    ap.add_argument("--kernel-desc", default="", help="kernel description for --ingest-pmc")
    args = ap.parse_args()
    if args.ingest_pmc:
        ingest_pmc(args, *args.ingest_pmc)
        return
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
    if args.copy_calibration:
        r = time_launches(lambda: torch.neg(x, out=y), args.steps, args.warmup, stream)
        log("copy calibration: %d bytes read + %d written per launch, avg %.4f ms, %.1f GB/s"
            % (batch * n * 8, batch * n * 8, r["avg_ms"], algo_bytes / r["avg_ms"] / 1e6))
        print(json.dumps({"copy_calibration": True, "bytes_read": batch * n * 8, "bytes_written": batch * n * 8,
                          "avg_ms": r["avg_ms"], "gbs": algo_bytes / r["avg_ms"] / 1e6}), flush=True)
        return

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
    desc = plan.describe()
    family = kernel_family(desc)
    log("headline kernel: %s" % desc)
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
                     "kernel": desc,
                     "algorithmic_bytes_per_launch": algo_bytes, "avg_launch_ms": round(head["avg_ms"], 5)},
        "rel_l2_vs_oracle": rel_err,
        "variants": {str(v): {"avg_ms": round(r["avg_ms"], 5),
                              "gflops": round(fl / r["avg_ms"] / 1e6, 1),
                              "hbm_gbs": round(algo_bytes / r["avg_ms"] / 1e6, 1)} for v, r in results.items()},
    }
    tr = load_traffic(family, args.variant, n, batch)
    if tr is not None:
        line["roofline"]["traffic"] = round(tr["traffic_bytes_per_launch"])
        line["roofline"]["traffic_over_algorithmic"] = round(tr["traffic_over_algorithmic"], 4)
    if not args.no_cpu:
        log("timing the CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(x_np, n, args.variant)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
