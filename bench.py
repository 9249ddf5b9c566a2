#!/usr/bin/env python3
"""Benchmark of the split-precision MoA inner product on one MI355X.

Workload: (+,*) FP64 inner product of two 8192 x 8192 arrays whose entries are
u * 2^k (u uniform[-1,1], k uniform{-8..8}), computed to FP64 accuracy from
BF16 slices (5 signed 9-bit digits per operand, 15 slice-pair products on the
matrix cores). One step = the whole path on one batch of input: row/column
scans, slicing of A and B, the fused slice-pair product with its exact FP64
fold and descaling. Inputs are resident in HBM before timing starts.

Printed (one JSON line): Gop/s of the split path (2*M*N*K algorithmic ops per
step), the plain FP64 matrix-core kernel on the same inputs for comparison,
the roofline of the dominant kernel (slice-pair product: BF16 MFMA flops per
launch / its average HIP-event duration, against 2516.6 TFLOP/s dense BF16),
and the CPU oracle timed on a bounded sample of rows.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "inner-product Gop/s at 8192^3: split-BF16 vs plain FP64, at ≤1e-12 rel err"
PEAK_BF16_TFLOPS = 2516.6
PEAK_FP64_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "split_gemm_8192_traffic.json")
SPLIT_SRCS = [os.path.join(ROOT, "paper_0907_0792_amd", "csrc", f) for f in ("k_split.hip", "split_gemm.hpp")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in SPLIT_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(launch_flops):
    """HBM bytes per launch of the slice-pair kernel from committed counter runs,
    or None when absent or taken on another version of the kernel."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(a, b, target_s=12.0):
    """The CPU oracle (plain psi-definition FP64 fold, OpenMP) on sampled rows."""
    import numpy as np
    import oracle
    K = a.shape[1]
    N = b.shape[1]
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    # Calibrate on one row per thread (the oracle parallelises over rows).
    rows = list(range(cores))
    t0 = time.perf_counter()
    oracle.inner(a, b, rows=rows)
    t1 = time.perf_counter() - t0
    nrows = max(cores, min(a.shape[0], int(cores * target_s / max(t1, 1e-3)) // cores * cores))
    rng = np.random.default_rng(1234)
    rows = np.sort(rng.choice(a.shape[0], nrows, replace=False))
    t0 = time.perf_counter()
    oracle.inner(a, b, rows=rows)
    dt = time.perf_counter() - t0
    ops = 2.0 * nrows * K * N
    return {"value": ops / dt / 1e9, "unit": "Gop/s", "cores": cores, "kind": "oracle",
            "sample": "%d of 8192 result rows (%.3g ops, %.1f s), plain FP64 fold of the psi definition" %
                      (nrows, ops, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--slices", type=int, default=5)
    ap.add_argument("--plain-reps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1).", flush=True)
        sys.exit(2)

    import numpy as np
    import torch
    import moa_inputs as mi
    import paper_0907_0792_amd as moa

    if args.calibrate_copy:
        # A plain copy of known size: HBM counters of this dispatch scale the
        # counters of the other kernels (bytes counted per byte moved).
        src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: calibration copy of %d bytes x2 done" % src.numel())
        del src, dst

    n = args.size
    S = args.slices
    P = S * (S + 1) // 2
    dev = torch.device("cuda:0")
    log("bench: generating %d^3 inputs" % n)
    a_h, b_h = mi.workload_split(m=n, k=n, n=n)
    a = torch.from_numpy(a_h).to(dev)
    b = torch.from_numpy(b_h).to(dev)
    d = torch.empty((n, n), dtype=torch.float64, device=dev)
    ws_bytes = moa.split_workspace_bytes(a.shape, b.shape, "bf16", S)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        moa.split_prepare(a, b, ws, "bf16", S)
        if ev is not None:
            ev[1].record()
        moa.split_multiply(a.shape, b.shape, d, ws, "bf16", S)
        if ev is not None:
            ev[2].record()

    log("bench: warmup %d" % args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    log("bench: timing %d steps" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prep_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps
    mult_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps
    ops = 2.0 * n * n * n
    ms_per_step = elapsed * 1e3 / args.steps
    value = ops * args.steps / elapsed / 1e9
    launch_flops = P * ops
    achieved = launch_flops / (mult_ms * 1e-3) / 1e12
    log("bench: split %.3f ms/step (prepare %.3f ms, multiply %.3f ms), %.1f Gop/s" %
        (ms_per_step, prep_ms, mult_ms, value))

    # Plain FP64 matrix-core kernel on the same inputs (the comparison).
    log("bench: plain FP64 x%d" % args.plain_reps)
    dp = torch.empty_like(d)
    moa.inner(a, b, out=dp)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.plain_reps):
        moa.inner(a, b, out=dp)
    e1.record()
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / args.plain_reps
    plain_gops = ops / (plain_ms * 1e-3) / 1e9
    # Relative difference of the two GPU results (normwise, sampled rows).
    rows = torch.arange(0, n, max(1, n // 64), device=dev)
    diff = float(torch.linalg.norm(d[rows] - dp[rows]) / torch.linalg.norm(dp[rows]))
    log("bench: plain %.3f ms, %.1f Gop/s; split/plain %.3fx; rel diff %.2e" %
        (plain_ms, plain_gops, value / plain_gops, diff))
    del dp

    result = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "split-BF16 (+,*) FP64-accuracy inner product, %dx%dx%d, entries u*2^k "
                               "(u~U[-1,1], k~U{-8..8}), %d signed 9-bit slices (%d slice pairs)" % (n, n, n, S, P),
                   "m": n, "k": n, "n": n, "slices": S, "slice_pairs": P},
        "stages_ms": {"prepare": round(prep_ms, 4), "multiply": round(mult_ms, 4)},
        "plain_fp64": {"value": round(plain_gops, 3), "unit": "Gop/s", "ms": round(plain_ms, 4),
                       "frac_fp64_peak": round(plain_gops / 1e3 / PEAK_FP64_TFLOPS, 4)},
        "split_vs_plain": round(value / plain_gops, 4),
        "rel_diff_split_vs_plain": diff,
        "roofline": {"bound": "mfma", "kernel": "k_split_gemm<%d>" % S, "achieved": round(achieved, 2),
                     "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_BF16_TFLOPS, 4),
                     "traffic": traffic_from_profiles(launch_flops)},
    }
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(a_h, b_h)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
