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
and the oracle leg: the CPU oracle timed on a bounded sample of rows, and the
normwise / max-norm / componentwise error of the BF16, INT8 and plain FP64
results against the oracle's compensated product on 16 sampled rows.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Other rows of the hot path are measured with --workload (one JSON line each,
same fields, their own roofline): plain64 (FP64 (+,*) 8192^3), rank5 (FP64
(+,*) <64 64 32 256>.<256 128 64>), tropical (int32 (max,+) 2048^3), outer
(FP32 (-) <512 512> o <64 64>), batch (10,000 uneven FP32 products, one graph
launch), grad (FP32 forward + backward <32 128 512>.<512 64 64>), small
(FP64 512^3 plus the <32 32> o <16 16> outer product), skinny (the paper's
own FP64 4 x 128 . 128 x 2^22 product, HBM-bound), skinny_sweep (the same for m = 1..4
and n = 2^16..2^22, the analogue of the paper's timing curves), axes (FP64 <16 2048 512>
. <16 2048 512> contracted over axes (1, 1), read in place), fewcols (int32
(max,+) 65536 x 4096 . 4096 x 8, wavefront-reduced fold).
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
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# Non-packed 32-bit VALU: 256 CUs x 64 lanes x 2.4 GHz.
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
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


def oracle_errors(a, b, results, rows):
    """Error of each GPU result (host copies of the sampled rows) against the
    oracle's compensated FP64 product (Dot2) on the same rows: normwise (the
    gate), max-norm and componentwise (|A||B| scale)."""
    import oracle
    ref = oracle.inner_dot2(a, b, rows=rows)
    scale = oracle.abs_product(a, b, rows=rows)
    out = {}
    for name, got in results.items():
        out[name] = {"normwise": oracle.normwise_error(got, ref), "maxnorm": oracle.maxnorm_error(got, ref),
                     "componentwise": oracle.componentwise_error(got, ref, scale)}
    return out


def cpu_oracle_small_single_thread():
    """The oracle on the FP64 512^3 product with one thread (the paper's
    sequential mode), in a child process so OpenMP starts with one thread."""
    import subprocess
    code = ("import json, sys, time; sys.path.insert(0, %r); import moa_inputs as mi, oracle; "
            "a, b, _, _ = mi.workload_small_mixed(); oracle.inner(a[:8], b); t = time.perf_counter(); "
            "oracle.inner(a, b); dt = time.perf_counter() - t; "
            "print(json.dumps({'value': 2.0 * 512 ** 3 / dt / 1e9, 'unit': 'Gop/s', 'ms': dt * 1e3, "
            "'cores': 1, 'kind': 'oracle', 'sample': 'FP64 512^3, whole product, one thread'}))" % ROOT)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=300)
    if r.returncode != 0:
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def _time_events(fn, steps, warmup):
    """Average ms of fn() over `steps` runs, HIP events on the current stream."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return e0.elapsed_time(e1) / steps, wall


def other_workload(args):
    """One JSON line for a non-headline row of the hot path."""
    import numpy as np
    import torch
    import moa_inputs as mi
    import paper_0907_0792_amd as moa
    dev = torch.device("cuda:0")
    w = args.workload
    base = {"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "data": "synthetic"}

    def put(x):
        return torch.from_numpy(np.asarray(x, order="C")).to(dev)

    if w in ("plain64", "rank5", "small"):
        if w == "plain64":
            a_h, b_h = mi.workload_split(m=args.size, k=args.size, n=args.size)
            desc = "FP64 (+,*) %d^3, entries u*2^k" % args.size
        elif w == "rank5":
            a_h, b_h = mi.workload_rank_general_f64()
            desc = "FP64 (+,*) <64 64 32 256> . <256 128 64> -> <64 64 32 128 64>, U[-1,1]"
        else:
            a_h, b_h, oa_h, ob_h = mi.workload_small_mixed()
            desc = "FP64 (+,*) 512^3 plus FP64 (*) outer <32 32> o <16 16>, U[-1,1]"
        a, b = put(a_h), put(b_h)
        out = torch.empty(moa.inner_shape(a.shape, b.shape), dtype=torch.float64, device=dev)
        M = int(np.prod(a_h.shape[:-1]))
        K = a_h.shape[-1]
        N = int(np.prod(b_h.shape[1:]))
        if w == "small":
            oa, ob = put(oa_h), put(ob_h)
            oc = torch.empty(tuple(oa.shape) + tuple(ob.shape), dtype=torch.float64, device=dev)
            fn = lambda: (moa.inner(a, b, out=out), moa.outer(oa, ob, "mul", out=oc))
        else:
            fn = lambda: moa.inner(a, b, out=out)
        ms, wall = _time_events(fn, args.steps, args.warmup)
        flops = 2.0 * M * N * K
        t = flops / (ms * 1e-3) / 1e12
        return dict(base, metric="inner-product Gop/s (%s)" % w, value=round(flops / (ms * 1e-3) / 1e9, 3),
                    unit="Gop/s", ms_per_step=round(ms, 4), dtype="f64",
                    config={"workload": desc, "m": M, "k": K, "n": N},
                    roofline={"bound": "mfma", "kernel": "k_gemm<double>", "achieved": round(t, 3),
                              "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": round(t / PEAK_FP64_TFLOPS, 4),
                              "traffic": None})
    if w == "axes":
        a_h, b_h = mi.workload_axes()
        a, b = put(a_h), put(b_h)
        M = a_h.shape[0] * a_h.shape[2]
        K = a_h.shape[1]
        N = b_h.shape[0] * b_h.shape[2]
        out = torch.empty(moa.inner_axes_shape(a.shape, 1, b.shape, 1), dtype=torch.float64, device=dev)
        ms, wall = _time_events(lambda: moa.inner_axes(a, b, (1, 1), out=out), args.steps, args.warmup)
        # Same M x K . K x N with plain layouts, for the cost of the strided views.
        ap, bp = a.reshape(M, K), b.reshape(K, N)
        outp = torch.empty((M, N), dtype=torch.float64, device=dev)
        ms_plain, _ = _time_events(lambda: moa.inner(ap, bp, out=outp), args.steps, args.warmup)
        flops = 2.0 * M * N * K
        t = flops / (ms * 1e-3) / 1e12
        return dict(base, metric="inner-product Gop/s (any-axis contraction)", value=round(flops / (ms * 1e-3) / 1e9, 3),
                    unit="Gop/s", ms_per_step=round(ms, 4), dtype="f64", plain_layout_ms=round(ms_plain, 4),
                    config={"workload": "FP64 (+,*) <16 2048 512> . <16 2048 512> over axes (1, 1) -> "
                                        "<16 512 16 512>, U[-1,1]", "m": M, "k": K, "n": N},
                    roofline={"bound": "mfma", "kernel": "k_gemm<double, TA=1, TB=0, 4x4, GEN=1>", "achieved": round(t, 3),
                              "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": round(t / PEAK_FP64_TFLOPS, 4),
                              "traffic": None})
    if w == "fewcols":
        a_h, b_h = mi.workload_fewcols()
        a, b = put(a_h), put(b_h)
        m, k, n = a_h.shape[0], a_h.shape[1], b_h.shape[1]
        out = torch.empty((m, n), dtype=torch.int32, device=dev)
        ms, wall = _time_events(lambda: moa.inner(a, b, "max", "add", out=out), args.steps, args.warmup)
        nbytes = 4.0 * (m * k + k * n + m * n)
        gbs = nbytes / (ms * 1e-3) / 1e9
        return dict(base, metric="few-column inner product GB/s", value=round(gbs, 2), unit="GB/s",
                    ms_per_step=round(ms, 4), dtype="int32", gops=round(2.0 * m * k * n / (ms * 1e-3) / 1e9, 2),
                    config={"workload": "int32 (max,+) %d x %d . %d x %d (wavefront-reduced fold over l)"
                                        % (m, k, k, n), "m": m, "k": k, "n": n},
                    roofline={"bound": "hbm", "kernel": "k_fewcols<int, max, add, NC=8>", "achieved": round(gbs, 2),
                              "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                              "traffic": None})
    if w == "skinny":
        a_h, b_h = mi.workload_skinny()
        a, b = put(a_h), put(b_h)
        m, k, n = a_h.shape[0], a_h.shape[1], b_h.shape[1]
        out = torch.empty((m, n), dtype=torch.float64, device=dev)
        ms, wall = _time_events(lambda: moa.inner(a, b, out=out), args.steps, args.warmup)
        nbytes = 8.0 * (k * n + m * n + m * k)
        gbs = nbytes / (ms * 1e-3) / 1e9
        return dict(base, metric="few-row inner product GB/s", value=round(gbs, 2), unit="GB/s",
                    ms_per_step=round(ms, 4), dtype="f64",
                    gops=round(2.0 * m * k * n / (ms * 1e-3) / 1e9, 2),
                    config={"workload": "FP64 (+,*) %d x %d . %d x %d (the paper's m x 128 . 128 x n matrix product)"
                                        % (m, k, k, n), "m": m, "k": k, "n": n},
                    roofline={"bound": "hbm", "kernel": "k_skinny<double, add, mul, MR=%d, R=4>" % m, "achieved": round(gbs, 2),
                              "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                              "traffic": None})
    if w == "skinny_sweep":
        # The paper's experiment shape (Section II.B): m x 128 . 128 x n for
        # m = 1..4 and growing n, as GB/s against the HBM roofline.
        rows = []
        for lg in (16, 18, 20, 22):
            n = 1 << lg
            a_h, b_h = mi.workload_skinny(m=4, n=n)
            a4, b = put(a_h), put(b_h)
            for m in (1, 2, 3, 4):
                a = a4[:m].contiguous()
                out = torch.empty((m, n), dtype=torch.float64, device=dev)
                ms, _ = _time_events(lambda: moa.inner(a, b, out=out), args.steps, args.warmup)
                nbytes = 8.0 * (128 * n + m * n + m * 128)
                rows.append({"m": m, "n": n, "ms": round(ms, 4), "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1),
                             "Gflop/s": round(2.0 * m * 128 * n / (ms * 1e-3) / 1e9, 1)})
            del a4, b, a, out
        best = max(r["GB/s"] for r in rows)
        return dict(base, metric="few-row inner product GB/s (sweep)", value=best, unit="GB/s",
                    ms_per_step=rows[-1]["ms"], dtype="f64",
                    config={"workload": "FP64 (+,*) m x 128 . 128 x n, m = 1..4, n = 2^16..2^22, U[-1,1]"},
                    sweep=rows,
                    roofline={"bound": "hbm", "kernel": "k_skinny<double, add, mul>", "achieved": best,
                              "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(best / PEAK_HBM_GBS, 4),
                              "traffic": None})
    if w == "tropical":
        a_h, b_h = mi.workload_tropical()
        a, b = put(a_h), put(b_h)
        out = torch.empty((2048, 2048), dtype=torch.int32, device=dev)
        ms, wall = _time_events(lambda: moa.inner(a, b, "max", "add", out=out), args.steps, args.warmup)
        terms = 2048.0 ** 3
        ops = 2 * terms  # one add and one max per term
        t = ops / (ms * 1e-3) / 1e12
        return dict(base, metric="tropical (max,+) inner product Gop/s", value=round(ops / (ms * 1e-3) / 1e9, 3),
                    unit="Gop/s", ms_per_step=round(ms, 4), dtype="i32",
                    config={"workload": "int32 (max,+) 2048^3, U{-1000..1000}", "m": 2048, "k": 2048, "n": 2048},
                    roofline={"bound": "alu", "kernel": "k_simt_inner<int,max,add,4,4>", "achieved": round(t, 3),
                              "peak": round(PEAK_VALU_TOPS, 2), "unit": "Tlane-op/s",
                              "frac": round(t / PEAK_VALU_TOPS, 4), "traffic": None})
    if w == "outer":
        a_h, b_h = mi.workload_outer_f32()
        a, b = put(a_h), put(b_h)
        out = torch.empty((512, 512, 64, 64), dtype=torch.float32, device=dev)
        ms, wall = _time_events(lambda: moa.outer(a, b, "sub", out=out), args.steps, args.warmup)
        nbytes = out.numel() * 4 + (a.numel() + b.numel()) * 4
        gbs = nbytes / (ms * 1e-3) / 1e9
        return dict(base, metric="outer product GB/s", value=round(gbs, 2), unit="GB/s", ms_per_step=round(ms, 4),
                    dtype="f32", config={"workload": "FP32 (-) outer <512 512> o <64 64> -> 2^30 elements"},
                    roofline={"bound": "hbm", "kernel": "k_outer_vec<float,sub>", "achieved": round(gbs, 2),
                              "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                              "traffic": None})
    if w == "batch":
        # The tile table is autotuned on this GPU first (outside the timed region).
        table = moa.batch_autotune(torch.float32)
        probs = mi.batch_problems(mi.rng_for(mi.BATCH), 10000)
        As = [put(p.a) for p in probs]
        Bs = [put(p.b) for p in probs]
        Ds = [torch.empty(moa.inner_shape(p.shape_a, p.shape_b), device=dev) for p in probs]
        bt = moa.Batch(As, Bs, Ds)
        ms, wall = _time_events(bt.run, args.steps, args.warmup)
        items, launches = bt.info()
        flops = sum(2.0 * np.prod(p.a.shape) * np.prod(p.b.shape[1:]) for p in probs)
        nbytes = sum(4.0 * (p.a.size + p.b.size + np.prod(p.a.shape[:-1]) * np.prod(p.b.shape[1:])) for p in probs)
        gbs = nbytes / (ms * 1e-3) / 1e9
        bt.close()
        return dict(base, metric="batched inner products Gop/s", value=round(flops / (ms * 1e-3) / 1e9, 3),
                    unit="Gop/s", ms_per_step=round(ms, 4), dtype="f32",
                    config={"workload": "10,000 uneven FP32 (+,*) products, one persistent graph launch, "
                                        "autotuned tile table",
                            "tile_table": table.strip().splitlines(),
                            "problems": len(probs), "work_items": items, "launches": launches,
                            "flops": flops, "bytes": nbytes},
                    roofline={"bound": "hbm", "kernel": "k_batch<float>", "achieved": round(gbs, 2),
                              "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                              "traffic": None})
    if w == "grad":
        a_h, b_h, g_h = mi.workload_grad()
        a = put(a_h).requires_grad_(True)
        b = put(b_h).requires_grad_(True)
        g = put(g_h)

        def fb():
            a.grad = None
            b.grad = None
            d = moa.moa_inner(a, b)
            d.backward(g)
        ms, wall = _time_events(fb, args.steps, args.warmup)
        flops = 3 * 2.0 * (32 * 128) * 512 * (64 * 64)
        t = flops / (ms * 1e-3) / 1e12
        return dict(base, metric="forward+backward Gop/s", value=round(flops / (ms * 1e-3) / 1e9, 3), unit="Gop/s",
                    ms_per_step=round(ms, 4), dtype="f32",
                    config={"workload": "FP32 (+,*) <32 128 512> . <512 64 64>, forward + dA + dB"},
                    roofline={"bound": "mfma", "kernel": "k_gemm<float>", "achieved": round(t, 3),
                              "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(t / PEAK_FP32_TFLOPS, 4),
                              "traffic": None})
    raise ValueError(w)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--slices", type=int, default=5)
    ap.add_argument("--plain-reps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="split",
                    choices=["split", "plain64", "rank5", "tropical", "outer", "batch", "grad", "small", "skinny", "skinny_sweep",
                             "axes", "fewcols"])
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

    if args.workload != "split":
        print(json.dumps(other_workload(args)), flush=True)
        return

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

    # The INT8-slice variant on the same inputs (7 slices of 7-bit digits).
    S8 = 7
    ws8 = torch.empty(moa.split_workspace_bytes(a.shape, b.shape, "int8", S8), dtype=torch.uint8, device=dev)
    d8 = torch.empty_like(d)

    def step8(ev=None):
        if ev is not None:
            ev[0].record()
        moa.split_prepare(a, b, ws8, "int8", S8)
        if ev is not None:
            ev[1].record()
        moa.split_multiply(a.shape, b.shape, d8, ws8, "int8", S8)
        if ev is not None:
            ev[2].record()

    for _ in range(max(1, args.warmup)):
        step8()
    torch.cuda.synchronize()
    evs8 = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        step8(evs8[i])
    torch.cuda.synchronize()
    el8 = time.perf_counter() - t0
    mult8 = sum(e[1].elapsed_time(e[2]) for e in evs8) / args.steps
    prep8 = sum(e[0].elapsed_time(e[1]) for e in evs8) / args.steps
    diff8 = float(torch.linalg.norm(d8[rows] - dp[rows]) / torch.linalg.norm(dp[rows]))
    # Host copies of seeded sample rows of the three results, for the oracle
    # leg's error report (after every timed region).
    err_rows = np.sort(np.random.default_rng(4321).choice(n, 16, replace=False))
    er = torch.from_numpy(err_rows).to(dev)
    sampled = {"split_bf16": d[er].cpu().numpy(), "split_int8": d8[er].cpu().numpy(),
               "plain_fp64": dp[er].cpu().numpy()}
    int8_ops = S8 * (S8 + 1) // 2 * ops / (mult8 * 1e-3) / 1e12
    split_int8 = {"value": round(ops * args.steps / el8 / 1e9, 3), "unit": "Gop/s",
                  "ms_per_step": round(el8 * 1e3 / args.steps, 4),
                  "stages_ms": {"prepare": round(prep8, 4), "multiply": round(mult8, 4)},
                  "slices": S8, "slice_pairs": S8 * (S8 + 1) // 2, "rel_diff_vs_plain": diff8,
                  "product_kernel_tops": round(int8_ops, 2), "frac_int8_peak": round(int8_ops / 5033.2, 4)}
    log("bench: int8 split %.3f ms/step, %.1f Gop/s, rel diff %.2e" %
        (split_int8["ms_per_step"], split_int8["value"], diff8))

    # The FP8 (E4M3) slice variant on the same inputs (10 slices of 5-bit digits).
    SF = 10
    wsf = torch.empty(moa.split_workspace_bytes(a.shape, b.shape, "fp8", SF), dtype=torch.uint8, device=dev)
    df = torch.empty_like(d)

    def stepf(ev=None):
        if ev is not None:
            ev[0].record()
        moa.split_prepare(a, b, wsf, "fp8", SF)
        if ev is not None:
            ev[1].record()
        moa.split_multiply(a.shape, b.shape, df, wsf, "fp8", SF)
        if ev is not None:
            ev[2].record()

    for _ in range(max(1, args.warmup)):
        stepf()
    torch.cuda.synchronize()
    evsf = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        stepf(evsf[i])
    torch.cuda.synchronize()
    elf = time.perf_counter() - t0
    multf = sum(e[1].elapsed_time(e[2]) for e in evsf) / args.steps
    prepf = sum(e[0].elapsed_time(e[1]) for e in evsf) / args.steps
    difff = float(torch.linalg.norm(df[rows] - dp[rows]) / torch.linalg.norm(dp[rows]))
    f8_tflops = SF * (SF + 1) // 2 * ops / (multf * 1e-3) / 1e12
    split_fp8 = {"value": round(ops * args.steps / elf / 1e9, 3), "unit": "Gop/s",
                 "ms_per_step": round(elf * 1e3 / args.steps, 4),
                 "stages_ms": {"prepare": round(prepf, 4), "multiply": round(multf, 4)},
                 "slices": SF, "slice_pairs": SF * (SF + 1) // 2, "rel_diff_vs_plain": difff,
                 "product_kernel_tflops": round(f8_tflops, 2), "frac_fp8_peak": round(f8_tflops / 5033.2, 4)}
    log("bench: fp8 split %.3f ms/step, %.1f Gop/s, rel diff %.2e" %
        (split_fp8["ms_per_step"], split_fp8["value"], difff))
    sampled["split_fp8"] = df[er].cpu().numpy()
    del wsf, df
    del d8, ws8

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
        "split_int8": split_int8,
        "split_fp8": split_fp8,
        "rel_diff_split_vs_plain": diff,
        "roofline": {"bound": "mfma", "kernel": "k_split_gemm<%d>" % S, "achieved": round(achieved, 2),
                     "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_BF16_TFLOPS, 4),
                     "traffic": traffic_from_profiles(launch_flops)},
    }
    if not args.no_cpu_baseline:
        # The oracle leg: the oracle timed on the host cores, and the error of
        # every result against it on the sampled rows.
        log("bench: error against the oracle on %d sampled rows" % len(err_rows))
        errs = oracle_errors(a_h, b_h, sampled, err_rows)
        bound = 1e-12
        ok = all(errs[k]["normwise"] <= bound for k in ("split_bf16", "split_int8", "split_fp8"))
        result["error_vs_oracle"] = dict(errs, reference="oracle Dot2 (compensated FP64)",
                                         rows=len(err_rows), bound_normwise=bound, within_bound=ok)
        if not ok:
            log("bench: WARNING: a split result exceeds the %.0e normwise bound: %s" % (bound, errs))
        log("bench: CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(a_h, b_h)
        result["cpu_oracle_512_one_thread"] = cpu_oracle_small_single_thread()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
