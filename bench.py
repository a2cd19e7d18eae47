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
    "amqft_kA_kernel": ["amqft_kA.hip", "amqft_kA_passes.h", "amqft_leaf.h", "amqft_device.h"],
    "amqft_kB_kernel": ["amqft_kB.hip", "amqft_kB_passes.h", "amqft_kA_passes.h", "amqft_leaf.h", "amqft_device.h"],
    "amqft_fast_kernel": ["amqft_fast.hip", "amqft_levels.h", "amqft_leaf.h", "amqft_device.h"],
    "amqft_lds_kernel": ["amqft_lds.hip", "amqft_levels.h", "amqft_device.h"],
}
METRIC = "batched FFT GFLOP/s (5N log2N) + HBM GB/s, N=4096 fp32, plain vs fused"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def flops_5nlogn(n: int, batch: int) -> float:
    import math
    return 5.0 * n * math.log2(n) * batch


# Warm-up floor applied before every timed workload, whatever --warmup says:
# the GPU's clocks take some tens of milliseconds of back-to-back work to
# settle, so launches continue until at least WARMUP_FLOOR_MS of wall time has
# passed and the median launch time of the last window of launches agrees
# with that of the window before within WARMUP_TOL (or WARMUP_CAP_MS passed).
WARMUP_FLOOR_MS = 200.0
WARMUP_TOL = 0.02
WARMUP_WINDOW = 10
WARMUP_CAP_MS = 3000.0


def settle(fn, stream):
    """Run fn back to back until its launch time is steady; returns the
    warm-up's wall time in ms."""
    import torch
    t0 = time.perf_counter()
    prev = None
    while True:
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(WARMUP_WINDOW)]
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        ts = sorted(a.elapsed_time(b) for a, b in evs)
        med = ts[len(ts) // 2]
        spent = (time.perf_counter() - t0) * 1e3
        steady = prev is not None and abs(med - prev) <= WARMUP_TOL * prev
        if (spent >= WARMUP_FLOOR_MS and steady) or spent >= WARMUP_CAP_MS:
            return spent
        prev = med


def time_launches(fn, steps: int, warmup: int, stream, floor: bool = True):
    """Average duration of each launch (events on the launch stream) and the
    wall time of the whole timed region, after `warmup` untimed launches and
    the time-based warm-up floor (settle; floor=False only for the long
    reference loops, whose single launch already runs for over 100 ms)."""
    import torch
    t0 = time.perf_counter()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    warm_ms = settle(fn, stream) if floor else (time.perf_counter() - t0) * 1e3
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
            "total_ms": total, "ms_per_step": total / steps, "warmup_ms": warm_ms}


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
    n, batch = args.n, args.batch
    desc = args.kernel_desc
    family = kernel_family(desc)
    fk, nd = _pmc_per_dispatch(fetch_csv, "FETCH_SIZE", family)
    wk, _ = _pmc_per_dispatch(write_csv, "WRITE_SIZE", family)
    fc, _ = _pmc_per_dispatch(copy_fetch_csv, "FETCH_SIZE", "neg_kernel")
    wc, _ = _pmc_per_dispatch(copy_write_csv, "WRITE_SIZE", "neg_kernel")
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


def cpu_baseline(x_np, n: int, variant: int, target_s: float = 12.0, single_s: float = 4.0):
    """Time the FP64 oracle on the first signals of the same workload: one
    thread per host core across signals, and a single thread."""
    import concurrent.futures as cf

    import numpy as np

    import oracle
    cores = os.cpu_count() or 1
    t = time.perf_counter()
    oracle.cdft(x_np[:2].astype(np.complex128), variant)
    per_sig = max((time.perf_counter() - t) / 2, 1e-6)
    # single thread: whole signals until about single_s seconds
    n1 = max(1, min(len(x_np), int(single_s / per_sig)))
    x1 = x_np[:n1].astype(np.complex128)
    t = time.perf_counter()
    oracle.cdft(x1, variant)
    el1 = time.perf_counter() - t
    one = {"value": flops_5nlogn(n, n1) / el1 / 1e9, "sample": "first %d signals, %.1f s on 1 thread" % (n1, el1)}
    want = max(cores, int(target_s * cores / per_sig))  # signal transforms for ~target_s of wall time
    sample = min(want, len(x_np))
    passes = max(1, min(20, (want + sample - 1) // sample))  # the sample again when it is short
    chunks = np.array_split(np.arange(sample), cores)
    xs = x_np[:sample].astype(np.complex128)

    def work(idx):
        for _ in range(passes):
            if len(idx):
                oracle.cdft(xs[idx], variant)

    t = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(work, chunks))
    el = time.perf_counter() - t
    return {"value": flops_5nlogn(n, sample * passes) / el / 1e9, "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "sample": "first %d signals of the workload x %d passes (N=%d, FP64 recursive oracle, variant %d), "
                      "%.1f s wall on %d threads" % (sample, passes, n, variant, el, cores),
            "value_1thread": round(one["value"], 4), "sample_1thread": one["sample"]}



def _rel(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / nb) if nb > 0 else float(np.linalg.norm(a.ravel()))


def _event_time(fn, reps: int, stream, between=None):
    """Per-rep HIP-event times of fn on the stream; `between` runs outside the
    timed events before every rep (e.g. a cache scrub)."""
    import torch
    ts = []
    for _ in range(reps):
        if between is not None:
            between()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return {"avg_ms": sum(ts) / len(ts), "median_ms": ts[len(ts) // 2], "min_ms": ts[0]}


def bench_fp64_small(args, stream):
    """64 x N=256 complex128, U[-1,1), seed 0, variant 4: latency-bound."""
    import numpy as np
    import torch

    import oracle
    from paper_1404_1810_amd import _lib, api, inputs
    x_np = inputs.cfg_fp64_n256()
    x = torch.from_numpy(x_np).cuda()
    y = torch.empty_like(x)
    plan = api.get_plan(256, 64, 4, _lib.C128)
    r = time_launches(lambda: plan.exec(x, out=y), max(args.steps, 50), args.warmup, stream)
    plan.exec(x, out=y)
    torch.cuda.synchronize()
    err = _rel(y.cpu().numpy(), oracle.cdft(x_np, 4))
    fl = flops_5nlogn(256, 64)
    return {"workload": "batch 64 x N=256 complex128, re/im U[-1,1) seed 0, forward, variant 4",
            "kernel": plan.describe(), "avg_ms": round(r["avg_ms"], 5), "median_ms": round(r["median_ms"], 5),
            "min_ms": round(r["min_ms"], 5), "gflops": round(fl / r["avg_ms"] / 1e6, 2),
            "rel_l2_vs_oracle": err, "bound": "latency (0.5 MB moved)"}


def bench_uneven(args, stream):
    """20000 FP32 signals of lengths 2^4..2^16 (seed 2), entries N(0,1) (seed 3),
    variant 4: one fused plan (persistent kernel + long-length classes,
    autotuned, graph-replayed) against gather -> one batched plan per length ->
    scatter (B2) and against one launch per signal (B1)."""
    import numpy as np
    import torch

    import oracle
    from paper_1404_1810_amd import _lib, api, inputs
    t0 = time.time()
    lengths, offsets = inputs.uneven_lengths()
    buf = inputs.uneven_entries(lengths, offsets)
    total = int(offsets[-1])
    log("uneven: %d signals, %d points, generated in %.1f s" % (len(lengths), total, time.time() - t0))
    x = torch.from_numpy(buf).cuda()
    y = torch.empty_like(x)
    mp = api.ManyPlan(lengths, offsets, 4, _lib.C64)
    mp.exec(x, out=y)  # first out-of-place execution autotunes
    torch.cuda.synchronize()
    fused_eager = time_launches(lambda: mp.exec(x, out=y), args.steps, args.warmup, stream)
    fused_graph = time_launches(lambda: mp.exec(x, out=y, graph=True), args.steps, args.warmup, stream)
    # B2: gather by length, batched plan per length, scatter back
    classes = []
    off_t = torch.from_numpy(offsets[:-1])
    for k in np.unique(lengths):
        sel = np.nonzero(lengths == k)[0]
        starts = off_t[torch.from_numpy(sel)]
        idx = (starts[:, None] + torch.arange(int(k))[None, :]).reshape(-1).cuda()
        rows = torch.empty((len(sel), int(k)), dtype=torch.complex64, device="cuda")
        outs = torch.empty_like(rows)
        classes.append((idx, rows, outs, api.get_plan(int(k), len(sel), 4, _lib.C64)))
    y2 = torch.empty_like(x)

    def plain():
        for idx, rows, outs, pl in classes:
            torch.index_select(x, 0, idx, out=rows.view(-1))
            pl.exec(rows, out=outs)
            y2.index_copy_(0, idx, outs.view(-1))
    plain_r = time_launches(plain, max(3, args.steps // 4), 1, stream)
    # B1: one launch per signal (plans cached per length, batch 1)
    singles = [api.get_plan(int(n), 1, 4, _lib.C64) for n in lengths]
    y3 = torch.empty_like(x)

    def per_signal():
        for i, pl in enumerate(singles):
            o, n = int(offsets[i]), int(lengths[i])
            pl.exec(x[o:o + n], out=y3[o:o + n])
    b1 = time_launches(per_signal, 2, 1, stream, floor=False)
    torch.cuda.synchronize()
    yf = y.cpu().numpy()
    # accuracy: fused vs plain (same relations, different kernels) and vs the
    # FP64 oracle on one signal of every length
    err_plain = _rel(yf, y2.cpu().numpy())
    worst = 0.0
    for k in np.unique(lengths):
        i = int(np.nonzero(lengths == k)[0][0])
        o, n = int(offsets[i]), int(lengths[i])
        ref = oracle.cdft(buf[o:o + n].astype(np.complex128)[None, :], 4)[0]
        worst = max(worst, _rel(yf[o:o + n], ref))
    algo = total * 16.0
    return {"workload": "20000 complex64 signals, N=2^k, k uniform on {4..16} (seed 2), entries N(0,1) (seed 3), "
                        "packed, int64 offsets, variant 4",
            "points": total, "plan": mp.describe(),
            "fused_graph_ms": round(fused_graph["avg_ms"], 4), "fused_eager_ms": round(fused_eager["avg_ms"], 4),
            "plain_gather_batched_scatter_ms": round(plain_r["avg_ms"], 4),
            "per_signal_launches_ms": round(b1["avg_ms"], 3),
            "speedup_vs_plain": round(plain_r["avg_ms"] / fused_graph["avg_ms"], 3),
            "speedup_vs_per_signal": round(b1["avg_ms"] / fused_graph["avg_ms"], 2),
            "fused_hbm_gbs": round(algo / fused_graph["avg_ms"] / 1e6, 1),
            "fused_frac_of_peak": round(algo / fused_graph["avg_ms"] / 1e6 / HBM_PEAK_GBS, 4),
            "rel_l2_fused_vs_plain": err_plain, "max_rel_l2_vs_oracle_one_per_length": worst}


def bench_grad(args, stream):
    """Fused loss/gradient: batch 4096 x N=1024 complex64 (x seed 0, W seed 1),
    loss = sum |W * F x|^2, grad = 2 F^H(|W|^2 F x); cold cache (a 512 MB
    scrub between reps, outside the events); also the autograd path and a
    65536-signal batch."""
    import numpy as np
    import torch

    import oracle
    from paper_1404_1810_amd import _lib, api, inputs
    xn, wn = inputs.cfg_grad()
    x = torch.from_numpy(xn).cuda()
    w = torch.from_numpy(wn).cuda()
    plan = api.get_plan(1024, 4096, 4, _lib.C64)
    scrub = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")

    def do_scrub():
        scrub.fill_(1)
    for _ in range(args.warmup):
        plan.power_loss_grad(x, w)
    settle(lambda: plan.power_loss_grad(x, w), stream)
    fused = _event_time(lambda: plan.power_loss_grad(x, w), args.steps, stream, do_scrub)

    def autograd_step():
        xr = x.detach().requires_grad_(True)
        yv = api.amqft(xr, 4)
        loss = (torch.abs(w * yv) ** 2).sum()
        loss.backward()
        return xr.grad
    for _ in range(args.warmup):
        autograd_step()
    settle(autograd_step, stream)
    auto = _event_time(autograd_step, max(3, args.steps // 2), stream, do_scrub)
    loss, g = plan.power_loss_grad(x, w)
    torch.cuda.synchronize()
    # accuracy on 4 signals against the oracle's closed form
    Xo = oracle.cdft(xn[:4].astype(np.complex128), 4)
    go = 2.0 * oracle.cdft_adjoint(np.abs(wn[:4].astype(np.complex128)) ** 2 * Xo, 4)
    lo = (np.abs(wn[:4].astype(np.complex128) * Xo) ** 2).sum(axis=1)
    err_g = _rel(g[:4].cpu().numpy(), go)
    err_l = _rel(loss[:4].cpu().numpy(), lo)
    algo = 4096 * 1024 * 24.0
    out = {"workload": "batch 4096 x N=1024 complex64, x ~ N(0,1) seed 0, W ~ N(0,1) seed 1, "
                       "loss = sum |W F x|^2 and its gradient, variant 4, cold cache",
           "fused_ms": round(fused["avg_ms"], 5), "fused_hbm_gbs": round(algo / fused["avg_ms"] / 1e6, 1),
           "autograd_fwd_bwd_ms": round(auto["avg_ms"], 4),
           "rel_l2_grad_vs_oracle": err_g, "rel_l2_loss_vs_oracle": err_l}
    del x, w
    # large batch for the bandwidth figure (inputs beyond the last-level cache)
    B = 65536
    xl = torch.empty((B, 1024), dtype=torch.complex64, device="cuda")
    wl = torch.empty_like(xl)
    for s0, rows in inputs.chunks("normal", inputs.SEEDS["grad_x"], B, 1024, chunk=4096):
        xl[s0:s0 + len(rows)].copy_(torch.from_numpy(rows.astype(np.complex64)))
    for s0, rows in inputs.chunks("normal", inputs.SEEDS["grad_w"], B, 1024, chunk=4096):
        wl[s0:s0 + len(rows)].copy_(torch.from_numpy(rows.astype(np.complex64)))
    pl = api.get_plan(1024, B, 4, _lib.C64)
    big = time_launches(lambda: pl.power_loss_grad(xl, wl), args.steps, args.warmup, stream)
    algo_l = B * 1024 * 24.0
    out.update({"large_batch": B, "large_fused_ms": round(big["avg_ms"], 4),
                "large_hbm_gbs": round(algo_l / big["avg_ms"] / 1e6, 1),
                "large_frac_of_peak": round(algo_l / big["avg_ms"] / 1e6 / HBM_PEAK_GBS, 4),
                "kernel": pl.describe()})
    return out


def bench_precision(args, stream):
    """1024 x N=2^20, FP16 and BF16 storage of U[-1,1) entries (seed 0; BF16:
    the FP16 values rounded to BF16), FP32 arithmetic, on-the-fly constants,
    all 8 variants: time and GB/s per variant, relative L2 error against the
    FP64 oracle on the same stored input for a few sampled signals."""
    import numpy as np
    import torch

    import oracle
    from paper_1404_1810_amd import _lib, api, inputs
    n = 1 << 20
    B = args.batch if args.batch != 16384 else 1024
    xh = torch.empty((B, n, 2), dtype=torch.float16, device="cuda")
    t0 = time.time()
    for s0 in range(0, B, 8):
        m = min(8, B - s0)
        xh[s0:s0 + m].copy_(torch.from_numpy(inputs.cfg_fp16_rows(m, n, start=s0)))
        if (s0 // 8) % 32 == 31:
            log("precision inputs: %d of %d signals resident (%.0f s)" % (s0 + m, B, time.time() - t0))
    sample = [0, B // 2, B - 1][: min(3, B)]
    out = {}
    for kind, dt, code in (("fp16", torch.float16, _lib.C32H), ("bf16", torch.bfloat16, _lib.C32B)):
        x = xh if dt == torch.float16 else xh.to(dt)
        y = torch.empty_like(x)
        xs = x[sample].float().cpu().numpy()
        xs = xs[..., 0].astype(np.float64) + 1j * xs[..., 1].astype(np.float64)
        ref = oracle.cdft(xs, 2)  # FP64 truth on the stored (quantised) input
        res = {}
        for v in range(1, 9):
            plan = api.Plan(n, B, v, code, _lib.FLAG_ONTHEFLY_CONSTANTS)
            r = time_launches(lambda: plan.exec(x, out=y), max(3, min(20, args.steps // 10)), 2, stream,
                              floor=False)
            got = y[sample].float().cpu().numpy()
            got = got[..., 0].astype(np.float64) + 1j * got[..., 1].astype(np.float64)
            nonfinite = int((~np.isfinite(got)).sum())
            res[str(v)] = {"kernel": plan.describe(), "avg_ms": round(r["avg_ms"], 3),
                           "hbm_gbs": round(B * n * 8.0 / r["avg_ms"] / 1e6, 1),
                           "rel_l2_vs_fp64_oracle": _rel(got, ref) if nonfinite == 0 else None,
                           "nonfinite_outputs": nonfinite}
            log("precision %s variant %d: %.3f ms, rel L2 %s" % (kind, v, r["avg_ms"],
                                                                  res[str(v)]["rel_l2_vs_fp64_oracle"]))
            plan.close()
        out[kind] = res
        del y
        if x is not xh:
            del x
        torch.cuda.empty_cache()
    return {"workload": "batch %d x N=2^20, fp16 storage (and the same values rounded to bf16), re/im U[-1,1) "
                        "seed 0, fp32 arithmetic, on-the-fly constants" % B, "sampled_signals": sample,
            "variants": out}


def bench_fixed(args, stream):
    """Fixed-point AM-QFT (int32 values, Q2.29 constants) on the headline shape:
    variants 1, 3, 5, 7, inputs |x| < 2^12 (inside int32 for all four up to
    N = 2^12 here, wraps counted by the oracle), two sampled signals per
    variant against the fixed-point oracle, bit for bit."""
    import numpy as np
    import torch

    import oracle
    from paper_1404_1810_amd import api, inputs

    n, B = args.n, args.batch
    seed = inputs.SEEDS["fixed_n4096"]
    xh = inputs.int_pairs(seed, B, n, 12)
    x = torch.from_numpy(xh).cuda()
    y = torch.empty_like(x)
    algo = B * n * 16.0
    res = {}
    for v in (1, 3, 5, 7):
        plan = api.get_plan(n, B, v, 4)
        r = time_launches(lambda: plan.exec(x, out=y), args.steps, args.warmup, stream)
        rows = [0, B - 1]
        got = y[rows].cpu().numpy()
        Xr, Xi, wraps = oracle.cdft_fixed(xh[rows, :, 0], xh[rows, :, 1], v)
        exact = bool(np.array_equal(got[..., 0], Xr) and np.array_equal(got[..., 1], Xi))
        res[str(v)] = {"kernel": plan.describe(), "avg_ms": round(r["avg_ms"], 5),
                       "hbm_gbs": round(algo / r["avg_ms"] / 1e6, 1),
                       "frac_of_peak": round(algo / r["avg_ms"] / 1e6 / HBM_PEAK_GBS, 4),
                       "sampled_bit_exact_vs_fixed_oracle": exact, "oracle_wraps": wraps}
        log("fixed point variant %d: avg %.4f ms, %.1f GB/s, bit-exact %s" % (v, r["avg_ms"], algo / r["avg_ms"] / 1e6,
                                                                               exact))
    return {"workload": "batch %d x N=%d int32 (re, im) pairs, entries uniform on [-2^12, 2^12) seed %d, "
                        "Q2.29 constants, forward" % (B, n, seed), "variants": res}


def bench_inplace(args, stream):
    """The large-N path in place against out of place: 256 signals of 2^16
    points (FP32, variant 4, 512 MiB), the same inputs, default workspaces;
    time per launch, workspace bytes, and the relative distance of the two
    outputs."""
    import ctypes

    import torch

    from paper_1404_1810_amd import _lib, api, inputs

    n, B, v = 1 << 16, 256, 4
    seed = inputs.SEEDS["fp32_n4096"]
    x = torch.empty((B, n), dtype=torch.complex64, device="cuda")
    for s0, rows in inputs.chunks("normal", seed, B, n):
        x[s0:s0 + len(rows)].copy_(torch.from_numpy(rows.astype("complex64")))
    algo = B * n * 16.0
    res = {}
    outs = {}
    for name, flags in (("out_of_place", 0), ("in_place", _lib.FLAG_IN_PLACE)):
        plan = api.Plan(n, B, v, _lib.C64, flags)
        ws = ctypes.c_size_t(0)
        _lib.check(_lib.load().amqft_plan_workspace_size(plan.handle, ctypes.byref(ws)), "workspace")
        if flags:
            y = x.clone()
            r = time_launches(lambda: plan.exec(y, out=y), args.steps // 4, args.warmup, stream)
            y.copy_(x)
            plan.exec(y, out=y)
        else:
            y = torch.empty_like(x)
            r = time_launches(lambda: plan.exec(x, out=y), args.steps // 4, args.warmup, stream)
        torch.cuda.synchronize()
        outs[name] = y
        res[name] = {"kernel": plan.describe(), "avg_ms": round(r["avg_ms"], 5),
                     "algorithmic_gbs": round(algo / r["avg_ms"] / 1e6, 1),
                     "workspace_bytes": int(ws.value), "workspace_over_data": round(ws.value / (B * n * 8.0), 4)}
        log("large path %s: avg %.4f ms, %.1f GB/s algorithmic, workspace %.1f MiB"
            % (name, r["avg_ms"], algo / r["avg_ms"] / 1e6, ws.value / 2 ** 20))
        plan.close()
    # the same operations in the same order; the compiler contracts the two
    # kernel instantiations into FMAs differently, so they agree to rounding
    d = torch.linalg.vector_norm(outs["in_place"] - outs["out_of_place"])
    res["rel_l2_in_place_vs_out_of_place"] = float(d / torch.linalg.vector_norm(outs["out_of_place"]))
    return {"workload": "batch %d x N=%d complex64, re/im N(0,1) seed %d, variant %d, forward" % (B, n, seed, v),
            **res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # untimed launches before the time-based warm-up floor of every workload
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
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
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the FP64, uneven-batch and fused-gradient workloads")
    ap.add_argument("--workload", default="headline", choices=["headline", "precision", "inplace"],
                    help="precision: the 2^20-point FP16 accuracy/throughput study instead; inplace: only the "
                         "in-place against out-of-place large-N workload")
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

    if args.workload == "precision":
        stream = torch.cuda.current_stream()
        res = bench_precision(args, stream)
        print(json.dumps({"metric": "fp16 / bf16-storage AM-QFT: GB/s and relative L2 error per variant, N=2^20",
                          "n_gpus": 1, "data": "synthetic", "dtype": "f16 / bf16 storage, f32 arithmetic",
                          "config": {"workload": res["workload"]}, "variants": res["variants"],
                          "sampled_signals": res["sampled_signals"]}), flush=True)
        return

    if args.workload == "inplace":
        res = bench_inplace(args, torch.cuda.current_stream())
        print(json.dumps({"metric": "in-place vs out-of-place large-N AM-QFT: ms per launch and workspace bytes",
                          "n_gpus": 1, "data": "synthetic", "dtype": "f32",
                          "config": {"workload": res.pop("workload")}, **res}), flush=True)
        return

    n, batch = args.n, args.batch
    log("generating %d x %d complex64 (seed %d)" % (batch, n, inputs.SEEDS["fp32_n4096"]))
    t0 = time.time()
    x = torch.empty((batch, n), dtype=torch.complex64, device="cuda")
    head_rows = min(batch, 8192)
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

    # context for the roofline: a plain elementwise copy of the same bytes
    rc = time_launches(lambda: torch.neg(x, out=y), args.steps, args.warmup, stream)
    copy_gbs = algo_bytes / rc["avg_ms"] / 1e6
    log("plain copy of the same bytes (torch.neg): avg %.4f ms, %.1f GB/s" % (rc["avg_ms"], copy_gbs))

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
        "warmup_ms": round(head["warmup_ms"], 1),
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
                     "algorithmic_bytes_per_launch": algo_bytes, "avg_launch_ms": round(head["avg_ms"], 5),
                     "copy_gbs_same_bytes": round(copy_gbs, 1),
                     "frac_of_copy": round(achieved / copy_gbs, 4)},
        "rel_l2_vs_oracle": rel_err,
        "variants": {str(v): {"avg_ms": round(r["avg_ms"], 5),
                              "gflops": round(fl / r["avg_ms"] / 1e6, 1),
                              "hbm_gbs": round(algo_bytes / r["avg_ms"] / 1e6, 1)} for v, r in results.items()},
    }
    if not args.no_extra:
        del x, y
        torch.cuda.empty_cache()
        extra = {}
        log("FP64 latency workload")
        extra["fp64_n256"] = bench_fp64_small(args, stream)
        log("uneven-length workload")
        extra["uneven"] = bench_uneven(args, stream)
        torch.cuda.empty_cache()
        log("fused loss/gradient workload")
        extra["grad"] = bench_grad(args, stream)
        torch.cuda.empty_cache()
        log("fixed-point workload")
        extra["fixed_point"] = bench_fixed(args, stream)
        torch.cuda.empty_cache()
        log("in-place large-N workload")
        extra["in_place"] = bench_inplace(args, stream)
        torch.cuda.empty_cache()
        line["workloads"] = extra
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
