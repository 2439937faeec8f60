#!/usr/bin/env python3
"""Benchmark of the FP8 GEMM hot path on one MI355X.

A step is one dense FP8 GEMM C = A B at M = N = K = 8192 (E4M3 x E4M3,
per-row A and per-column B descales, FP32 accumulation, BF16 output) on
operands already resident in HBM; `value` is its throughput in TFLOP/s
(2 M N K per step).  The same JSON line carries:
  - roofline: the GEMM kernel's own average duration from HIP events on the
    stream it is launched on, against the MI355X dense FP8 peak;
  - cpu_baseline: the CPU oracle timed on a block of rows of the same GEMM;
  - extra: the 2:4 GEMM on the same shape (dense-equivalent TFLOP/s), the
    quantize and prune passes (GB/s), and, unless --quick, the skinny shapes,
    the grouped GEMM and the served request stream.
Only one GPU is supported: --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP8_TFLOPS = 5000.0          # MI355X dense FP8 MFMA
PEAK_FP8_SPARSE_TFLOPS = 10000.0  # 2:4 dense-equivalent
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_events(fn, iters, stream):
    """Average milliseconds per call of fn, from HIP events on `stream`."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(iters):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / iters


def make_operands(lib, M, N, K, seed, fa=0, fb=0):
    """Quantized operands built on the device by the library's own quantize."""
    import torch
    from paper_2602_10262_amd import synth
    xa = torch.from_numpy(synth.normal_outliers(seed, (M, K))).cuda()
    xb = torch.from_numpy(synth.normal_outliers(seed + 1, (N, K))).cuda()
    qa, _, da = lib.fp8_quantize(xa, fa, lib.FP8_SCALE_ROW)
    qb, _, db = lib.fp8_quantize(xb, fb, lib.FP8_SCALE_ROW)
    torch.cuda.synchronize()
    return xa, xb, qa, da, qb, db


def cpu_baseline(M, N, K, target_s=12.0):
    """The oracle (plain C, FP64, all host threads) on a block of rows of the
    same GEMM; throughput scaled to TFLOP/s of the full-shape metric."""
    import oracle as orc
    from paper_2602_10262_amd import synth
    nt = os.cpu_count() or 1
    rows = max(1, nt)
    xb = synth.normal_outliers(1, (N, K))
    qb, _, db = orc.quantize(xb, orc.E4M3, True)
    done_rows, spent = 0, 0.0
    while True:
        xa = synth.normal_outliers(0, (rows, K))
        qa, _, da = orc.quantize(xa, orc.E4M3, True)
        t0 = time.perf_counter()
        orc.gemm(qa, orc.E4M3, qb, orc.E4M3, da, db, nthreads=nt)
        dt = time.perf_counter() - t0
        done_rows, spent = rows, dt
        if dt * 2 > target_s or rows >= M:
            break
        rows = min(M, int(rows * max(2.0, target_s / max(dt, 1e-3) * 0.8)))
    tflops = 2.0 * done_rows * N * K / spent / 1e12
    return {"value": tflops, "unit": "TFLOP/s", "cores": nt, "kind": "oracle",
            "sample": f"{done_rows} of {M} rows of the {M}x{N}x{K} GEMM (FP64, exact decode), {spent:.1f} s"}


def bench_sparse(lib, qa, da, qb, db, iters, warmup, stream):
    import torch
    M, K = qa.shape
    N = qb.shape[0]
    values, meta, _ = lib.fp8_sparse24_prune_compress(qa, 0, with_mask=False)
    c = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")
    fn = lambda: lib.fp8_sparse24_gemm(values, meta, qb, lib.FP8_SPARSE_A, da, db, c=c, stream=stream)
    for _ in range(warmup):
        fn()
    ms = time_events(fn, iters, stream)
    prune_ms = time_events(lambda: lib.fp8_sparse24_prune_compress(qa, 0, with_mask=False, stream=stream), 10, stream)
    pruned = lib.fp8_sparse24_decompress(values, meta, K)
    cd = torch.empty_like(c)
    fnd = lambda: lib.fp8_gemm(pruned, qb, da, db, c=cd, stream=stream)
    for _ in range(warmup):
        fnd()
    ms_dense_pruned = time_events(fnd, iters, stream)
    flops = 2.0 * M * N * K
    return {
        "shape": [M, N, K],
        "sparse_ms": ms, "sparse_tflops_dense_equiv": flops / ms / 1e9,
        "sparse_frac_of_2to4_peak": flops / ms / 1e9 / PEAK_FP8_SPARSE_TFLOPS,
        "dense_on_pruned_ms": ms_dense_pruned, "speedup_vs_dense": ms_dense_pruned / ms,
        "prune_compress_ms": prune_ms, "prune_gbs": (M * K * (1 + 0.5 + 0.125)) / prune_ms / 1e6,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--quick", action="store_true", help="headline GEMM, 2:4 and quantize only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tune", action="store_true", help="use the library's default plan")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (see DESIGN.md, sharding)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2602_10262_amd as lib
    lib.load()
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    M = N = K = args.size
    log(f"bench: dense FP8 GEMM {M}x{N}x{K}")
    xa, xb, qa, da, qb, db = make_operands(lib, M, N, K, 0)
    c = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")
    gargs = lib.gemm_args(qa, qb, da, db, c)
    tuned = None
    if not args.no_tune:
        (tile, split), us = lib.fp8_tune_gemm(gargs, iters=5, stream=stream)
        tuned = {"tile": tile, "split_k": split, "us": us}
        log(f"tuned plan: tile {tile} split {split} {us:.1f} us")
    plan_tile, plan_split = lib.fp8_gemm_plan_resolve(gargs)
    ws = None
    step = lambda: lib.fp8_gemm(qa, qb, da, db, c=c, ws=ws, stream=stream)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = e0.elapsed_time(e1) / args.steps
    ms_per_step = 1000.0 * wall / args.steps
    flops = 2.0 * M * N * K
    value = flops / (ms_per_step * 1e-3) / 1e12
    achieved = flops / (kernel_ms * 1e-3) / 1e12
    log(f"dense: {ms_per_step:.3f} ms/step wall, {kernel_ms:.3f} ms by events -> {achieved:.1f} TFLOP/s")

    extra = {"plan": {"tile": plan_tile, "split_k": plan_split}, "tuned": tuned}
    # quantize pass (per-row, A operand): 4 B read + 1 B written per element
    qms = time_events(lambda: lib.fp8_quantize(xa, 0, lib.FP8_SCALE_ROW, stream=stream), 10, stream)
    extra["quantize_per_row"] = {"ms": qms, "gbs": M * K * 5 / qms / 1e6}
    extra["sparse24"] = bench_sparse(lib, qa, da, qb, db, max(5, args.steps // 2), 3, stream)
    log(f"2:4: {extra['sparse24']['sparse_tflops_dense_equiv']:.1f} TFLOP/s dense-equivalent, "
        f"{extra['sparse24']['speedup_vs_dense']:.2f}x vs dense on the pruned matrix")
    del xa, xb

    out = {
        "metric": "FP8 TFLOP/s (% of peak) dense vs 2:4 sparse; grouped-serving p50/p99 latency",
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp8_e4m3 x fp8_e4m3 -> fp32 accumulate",
        "data": "synthetic: N(0,1) with 1% +-20 sigma outliers, per-row/column amax scales",
        "config": {"workload": f"dense FP8 GEMM {M}x{N}x{K}, E4M3 x E4M3, per-row A / per-column B "
                               "descales, FP32 accumulate, BF16 out", "M": M, "N": N, "K": K,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP8_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP8_TFLOPS, "traffic": None},
        "extra": extra,
    }
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(M, N, K)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
