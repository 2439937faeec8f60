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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dense_gemm_8192_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2602_10262_amd", "csrc", f)
                  for f in ("gemm_tile.hpp", "gemm_launch.hpp", "gemm.hip")]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the headline GEMM from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's
    reading for a copy of known size), or None when that summary is missing
    or was taken from different kernel sources."""
    try:
        kv = dict(line.split(":", 1) for line in open(TRAFFIC_FILE) if ":" in line and not line.startswith("#"))
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        if kv.get("kernel_source_sha1") != kernel_source_hash():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


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


def cpu_baseline(M, N, K, target_s=20.0):
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


def overlap_fraction(spans):
    """Share of the makespan during which at least two of the (start, end)
    intervals are active: the paper's overlap efficiency (Sec. 4.2), here over
    the streams' busy spans (each stream runs its kernels back to back)."""
    if len(spans) < 2:
        return 0.0
    ev = sorted([(s, 1) for s, _ in spans] + [(e, -1) for _, e in spans])
    t0 = min(s for s, _ in spans)
    t1 = max(e for _, e in spans)
    active, last, both = 0, t0, 0.0
    for t, d in ev:
        if active >= 2:
            both += t - last
        active += d
        last = t
    return both / (t1 - t0) if t1 > t0 else 0.0


def fp8_plan_sweep(lib, fn_plan, stream, candidates):
    """The fastest FP8-MFMA plan of `candidates` for fn_plan(plan)."""
    best = None
    for pl in candidates:
        try:
            fn_plan(pl)
        except lib.Fp8Error:
            continue
        ms = time_events(lambda: fn_plan(pl), 10, stream)
        if best is None or ms < best[1]:
            best = (pl, ms)
    return best


def bench_ace(lib, base, sizes=(256, 512, 2048), iters=100, counts=(1, 2, 4, 8), pairs_with=(512, 1024, 2048)):
    """Concurrent-stream study (the paper's ACE study, Sec. 6): at each size,
    `n` streams each run `iters` back-to-back GEMMs (dense, 2:4 on A, or half
    of the streams each), every stream's GEMMs captured once into a HIP graph
    so the host launch rate does not limit what the device overlaps.  The
    GEMMs run FP8-MFMA plans (the path this study is about; below K = 3584
    the library's own default is the exact-sum path) picked by a small sweep.
    Per stream: device time from its first kernel to its last (events on the
    stream).  Reported per (size, mode, n): makespan, aggregate TFLOP/s,
    speedup (the streams' one-stream times, summed, over the makespan),
    overlap (share of the makespan with at least two streams busy), the
    coefficient of variation of the stream times and both fairness measures.
    Co-run pairs (occupancy fragmentation, Sec. 6.3): a 512^3 stream beside a
    stream of S^3 GEMMs sized to the same one-stream time."""
    import torch
    from paper_2602_10262_amd import synth
    nmax = max(counts)
    streams = [torch.cuda.Stream() for _ in range(nmax)]
    res = {"iters_per_stream": iters, "launch": "one HIP graph per stream", "sizes": {}}
    ops = {}

    def operands(size):
        if size in ops:
            return ops[size]
        M = N = K = size
        xa = torch.from_numpy(synth.normal_outliers(7, (M, K))).cuda()
        xb = torch.from_numpy(synth.normal_outliers(8, (N, K))).cuda()
        qa, _, da = lib.fp8_quantize(xa, 0, lib.FP8_SCALE_ROW, stream=base)
        qb, _, db = lib.fp8_quantize(xb, 0, lib.FP8_SCALE_ROW, stream=base)
        va, ma, _ = lib.fp8_sparse24_prune_compress(qa, 0, with_mask=False, stream=base)
        torch.cuda.synchronize()
        cands = [(t, s) for t in (0, 3, 7, 8, 13, 19) for s in (1, 2, 4)]
        c0 = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")
        dplan = fp8_plan_sweep(lib, lambda pl: lib.fp8_gemm(qa, qb, da, db, c=c0, plan=pl, stream=base), base, cands)[0]
        splan = fp8_plan_sweep(lib, lambda pl: lib.fp8_sparse24_gemm(va, ma, qb, lib.FP8_SPARSE_A, da, db, c=c0,
                                                                     plan=pl, stream=base), base, cands)[0]
        outs = [torch.empty((M, N), dtype=torch.bfloat16, device="cuda") for _ in range(nmax)]
        ws = [torch.empty(4 * M * N * 4, dtype=torch.uint8, device="cuda") for _ in range(nmax)]
        ops[size] = dict(qa=qa, qb=qb, da=da, db=db, va=va, ma=ma, dplan=dplan, splan=splan, outs=outs, ws=ws)
        return ops[size]

    def gemm(size, sparse, i, st):
        o = operands(size)
        if sparse:
            lib.fp8_sparse24_gemm(o["va"], o["ma"], o["qb"], lib.FP8_SPARSE_A, o["da"], o["db"], c=o["outs"][i],
                                  plan=o["splan"], ws=o["ws"][i], stream=st)
        else:
            lib.fp8_gemm(o["qa"], o["qb"], o["da"], o["db"], c=o["outs"][i], plan=o["dplan"], ws=o["ws"][i], stream=st)

    def capture(size, sparse, i, n_iter):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=streams[i]):
            for _ in range(n_iter):
                gemm(size, sparse, i, streams[i])
        return g

    def run(graphs):
        """graphs[i] runs on stream i; returns per-stream (start, end) in ms from a common event."""
        n = len(graphs)
        start = torch.cuda.Event(enable_timing=True)
        begins = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
        ends = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
        start.record(base)
        for i in range(n):
            streams[i].wait_event(start)
            begins[i].record(streams[i])
            with torch.cuda.stream(streams[i]):
                graphs[i].replay()
            ends[i].record(streams[i])
        torch.cuda.synchronize()
        return [(start.elapsed_time(b), start.elapsed_time(e)) for b, e in zip(begins, ends)]

    def stats(spans, alone):
        t = [e - s for s, e in spans]
        mk = max(e for _, e in spans) - min(s for s, _ in spans)
        mean = sum(t) / len(t)
        sd = (sum((x - mean) ** 2 for x in t) / len(t)) ** 0.5
        return {"makespan_ms": mk, "speedup": sum(alone) / mk, "overlap": overlap_fraction(spans),
                "cv": sd / mean, "fairness_range": 1.0 - (max(t) - min(t)) / mean, "fairness_minmax": min(t) / max(t),
                "stream_ms": t}

    for size in sizes:
        o = operands(size)
        flops = 2.0 * size ** 3
        # each stream's graph checked once against the eager GEMM, bit for bit
        ref = {}
        for sparse in (False, True):
            gemm(size, sparse, 0, base)
            torch.cuda.synchronize()
            ref[sparse] = o["outs"][0].clone()
        graphs = {}
        for mode in ("dense", "sparse", "mixed"):
            for i in range(nmax):
                sparse = mode == "sparse" or (mode == "mixed" and i % 2 == 1)
                g = capture(size, sparse, i, iters)
                o["outs"][i].zero_()
                with torch.cuda.stream(streams[i]):
                    g.replay()
                torch.cuda.synchronize()
                if not torch.equal(o["outs"][i], ref[sparse]):
                    raise RuntimeError(f"graph replay differs from the eager GEMM ({size}, {mode}, stream {i})")
                graphs[(mode, i)] = g
        alone = {}
        for mode in ("dense", "sparse"):
            run([graphs[(mode, 0)]])
            sp = run([graphs[(mode, 0)]])[0]
            alone[mode] = sp[1] - sp[0]
        sres = {"plans": {"dense": list(o["dplan"]), "sparse": list(o["splan"])},
                "one_stream_ms": dict(alone), "modes": {}}
        for mode in ("dense", "sparse", "mixed"):
            rows = []
            for n in counts:
                kinds = ["sparse" if (mode == "sparse" or (mode == "mixed" and i % 2 == 1)) else "dense"
                         for i in range(n)]
                spans = run([graphs[(mode, i)] for i in range(n)])
                row = stats(spans, [alone[k] for k in kinds])
                row.update({"streams": n, "tflops": n * iters * flops / (row["makespan_ms"] * 1e-3) / 1e12})
                rows.append(row)
            sres["modes"][mode] = rows
        res["sizes"][str(size)] = sres
        log(f"  ace {size}^3: " + "; ".join(
            f"{m} " + ", ".join(f"{r['streams']}s x{r['speedup']:.2f} ov {r['overlap']:.2f}" for r in rows)
            for m, rows in sres["modes"].items()))
        del graphs
    # co-run pairs: 512^3 beside S^3 of about the same one-stream time
    if 512 in sizes:
        pres = []
        g512 = capture(512, False, 0, iters)
        run([g512])
        sp = run([g512])[0]
        t512 = sp[1] - sp[0]
        for S in pairs_with:
            operands(S)
            probe = capture(S, False, 1, 10)
            run([probe])
            sp = run([probe])[0]
            per = (sp[1] - sp[0]) / 10
            n_it = max(1, int(round(t512 / per)))
            gS = capture(S, False, 1, n_it)
            run([gS])
            spS = run([gS])[0]
            tS = spS[1] - spS[0]
            spans = run([g512, gS])
            row = stats(spans, [t512, tS])
            row.update({"pair": f"512^3 x {iters} with {S}^3 x {n_it}",
                        "slowdown_512": (spans[0][1] - spans[0][0]) / t512,
                        "slowdown_other": (spans[1][1] - spans[1][0]) / tS})
            pres.append(row)
            del gS, probe
        res["pairs"] = pres
        log("  ace pairs: " + "; ".join(f"{r['pair']}: x{r['speedup']:.2f} fair {r['fairness_minmax']:.2f}"
                                        for r in pres))
    return res


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
    # both sides pruned: the weight rows too; dense on the two pruned matrices
    vw, mw, _ = lib.fp8_sparse24_prune_compress(qb, 0, with_mask=False)
    pruned_w = lib.fp8_sparse24_decompress(vw, mw, K)
    fnb = lambda: lib.fp8_sparse24_both_gemm(values, meta, vw, mw, da, db, c=c, stream=stream)
    for _ in range(warmup):
        fnb()
    ms_both = time_events(fnb, iters, stream)
    fnbd = lambda: lib.fp8_gemm(pruned, pruned_w, da, db, c=cd, stream=stream)
    for _ in range(warmup):
        fnbd()
    ms_both_dense = time_events(fnbd, iters, stream)
    both_plan = lib.fp8_sparse24_both_gemm_plan_resolve(
        lib.sparse24_both_args(values, meta, vw, mw, da, db, c))
    flops = 2.0 * M * N * K
    return {
        "shape": [M, N, K],
        "sparse_ms": ms, "sparse_tflops_dense_equiv": flops / ms / 1e9,
        "sparse_frac_of_2to4_peak": flops / ms / 1e9 / PEAK_FP8_SPARSE_TFLOPS,
        "dense_on_pruned_ms": ms_dense_pruned, "speedup_vs_dense": ms_dense_pruned / ms,
        "prune_compress_ms": prune_ms, "prune_gbs": (M * K * (1 + 0.5 + 0.125)) / prune_ms / 1e6,
        "both_sides": {"ms": ms_both, "plan": list(both_plan), "tflops_dense_equiv": flops / ms_both / 1e9,
                       "dense_on_both_pruned_ms": ms_both_dense, "speedup_vs_dense": ms_both_dense / ms_both},
    }


def bench_mixed(lib, stream, M=4096, H=2048, n_chains=8, streams=4):
    """Mixed-precision sequence: the FP32 / FP16 / BF16 GEMMs alone at H^3,
    then n_chains chains of FP32 -> FP16 -> FP8 stages (M x H each) under the
    three schedules of the chain executor."""
    import torch
    res = {"gemm": [], "chains": {}}
    g = torch.Generator(device="cuda").manual_seed(3)
    for name, dt in (("f32", torch.float32), ("f16", torch.float16), ("bf16", torch.bfloat16)):
        a = torch.randn((4096, 4096), generator=g, device="cuda").to(dt)
        b = torch.randn((4096, 4096), generator=g, device="cuda").to(dt)
        c = torch.empty((4096, 4096), dtype=torch.float32, device="cuda")
        lib.fp8_hp_gemm(a, b, c=c, stream=stream)
        ms = time_events(lambda: lib.fp8_hp_gemm(a, b, c=c, stream=stream), 10, stream)
        peak = 157.3 if name == "f32" else 2500.0
        tf = 2.0 * 4096 ** 3 / (ms * 1e-3) / 1e12
        res["gemm"].append({"type": name, "shape": [4096, 4096, 4096], "ms": ms, "tflops": tf,
                            "frac_of_peak": tf / peak})
        del a, b, c
    stages, keep = [], []
    for p, dt in ((lib.FP8_STAGE_F32, torch.float32), (lib.FP8_STAGE_F16, torch.float16), (lib.FP8_STAGE_FP8, None)):
        w = torch.randn((H, H), generator=g, device="cuda") / H ** 0.5
        if p == lib.FP8_STAGE_FP8:
            q, _, d = lib.fp8_quantize(w, 0, lib.FP8_SCALE_ROW, stream=stream)
            stages.append((p, q, d))
        else:
            stages.append((p, w.to(dt), None))
    torch.cuda.synchronize()
    ch = lib.Chain(stages, M, H, n_chains, max_streams=streams)
    for c in range(n_chains):
        ch.tensor(c, 0).copy_(torch.randn((M, H), generator=g, device="cuda"))
    torch.cuda.synchronize()
    res["chains"]["config"] = {"M": M, "H": H, "n_chains": n_chains, "streams": streams,
                               "stages": ["f32", "f16", "fp8"]}
    for name, sched, ns in (("serial", lib.FP8_CHAIN_SERIAL, 1), ("in_phase", lib.FP8_CHAIN_IN_PHASE, streams),
                            ("staggered", lib.FP8_CHAIN_STAGGERED, streams)):
        ch.run(sched, ns)   # warm-up
        runs = [ch.run(sched, ns) for _ in range(3)]
        best = min(runs, key=lambda r: r["makespan_ms"])
        res["chains"][name] = best
    ch.close()
    return res


PEAK_BF16_TFLOPS = 2500.0   # dense 16-bit MFMA peak of MI355X (the exact-sum tiles run the BF16 MFMA)


def bench_exact(lib, stream, iters=20):
    """The exact-sum tiles (K below 3584: FP8 decoded exactly to BF16 and
    summed on the BF16 MFMA): the default plan and each exact tile, dense and
    2:4 (A side, on the pruned A), against the BF16 roofline."""
    import torch
    from paper_2602_10262_amd import synth
    out = []
    exact_tiles = [t for t in range(lib.fp8_num_tiles()) if lib.fp8_tile_info(t)["exact"]]
    for (M, N, K) in ((1024, 1024, 1024), (2048, 2048, 2048), (3072, 3072, 3072), (8192, 8192, 2048)):
        xa = torch.from_numpy(synth.normal_outliers(7, (M, K))).cuda()
        xb = torch.from_numpy(synth.normal_outliers(8, (N, K))).cuda()
        qa, _, da = lib.fp8_quantize(xa, 0, lib.FP8_SCALE_ROW, stream=stream)
        qb, _, db = lib.fp8_quantize(xb, 0, lib.FP8_SCALE_ROW, stream=stream)
        del xa, xb
        values, meta, _ = lib.fp8_sparse24_prune_compress(qa, 0, with_mask=False, stream=stream)
        pruned = lib.fp8_sparse24_decompress(values, meta, K)
        c = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")
        flops = 2.0 * M * N * K
        row = {"M": M, "N": N, "K": K,
               "default_plan": lib.fp8_gemm_plan_resolve(lib.gemm_args(pruned, qb, da, db, c)), "tiles": {}}
        for _ in range(20):   # clocks up before the first timed plan
            lib.fp8_gemm(pruned, qb, da, db, c=c, stream=stream)
        for plan in [None] + [(t, 1) for t in exact_tiles]:
            key = "default" if plan is None else str(plan[0])
            dense = lambda: lib.fp8_gemm(pruned, qb, da, db, c=c, plan=plan, stream=stream)
            sparse = lambda: lib.fp8_sparse24_gemm(values, meta, qb, lib.FP8_SPARSE_A, da, db, c=c, plan=plan,
                                                   stream=stream)
            r = {}
            for name, f in (("dense", dense), ("sparse", sparse)):
                for _ in range(3):
                    f()
                ms = time_events(f, iters, stream)
                r[name + "_tflops"] = flops / ms / 1e9
                r[name + "_frac_of_bf16_peak"] = r[name + "_tflops"] / PEAK_BF16_TFLOPS
            row["tiles"][key] = r
        out.append(row)
        del qa, qb, values, meta, pruned, c
        torch.cuda.empty_cache()
    return out


def bench_batching(lib, stream, batch_sizes=(4, 8, 16, 32), seeds=(0, 1, 2)):
    """Should the server batch the requests it admits together into one
    grouped launch?  For batches of B requests drawn from the served workload
    (M log-uniform on [1, 8192], N and K from {2048, 4096, 8192, 14336}, half
    with 2:4 weights), each request's activations are quantized per token and
    multiplied by its weight, either (a) as the server does it: one quantize +
    GEMM per request, requests spread round robin over 4 streams; or (b)
    quantize per request on one stream, then one persistent grouped launch of
    the batch (plan built beforehand; its host-side build time is reported
    apart)."""
    import ctypes
    import torch
    from paper_2602_10262_amd import synth
    sizes = [2048, 4096, 8192, 14336]
    L = lib.load()
    streams = [torch.cuda.Stream() for _ in range(4)]
    weights = {}

    def weight(N, K, sp):
        key = (N, K, sp)
        if key not in weights:
            w = torch.randn((N, K), device="cuda")
            qw, _, dw = lib.fp8_quantize(w, 0, lib.FP8_SCALE_ROW)
            del w
            if sp:
                v, m, _ = lib.fp8_sparse24_prune_compress(qw, 0, with_mask=False)
                weights[key] = (v, m, dw)
            else:
                weights[key] = (qw, None, dw)
        return weights[key]

    out = []
    for B in batch_sizes:
        row = {"batch": B, "per_request_4_streams_ms": [], "grouped_ms": [], "plan_build_us": []}
        for seed in seeds:
            rng = np.random.default_rng(1000 * B + seed)
            gen = torch.Generator(device="cuda").manual_seed(1000 * B + seed)
            Ms = synth.log_uniform_int(rng, 1, 8192, B)
            reqs = []
            for i in range(B):
                M, N, K = int(Ms[i]), int(rng.choice(sizes)), int(rng.choice(sizes))
                sp = bool(rng.integers(0, 2))
                x = torch.rand((M, K), device="cuda", generator=gen) * 2.0 - 1.0
                q = torch.empty((M, K), dtype=torch.uint8, device="cuda")
                sc = torch.empty(M, dtype=torch.float32, device="cuda")
                dc = torch.empty(M, dtype=torch.float32, device="cuda")
                c = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")
                w, meta, dw = weight(N, K, sp)
                if sp:
                    args = lib.sparse24_args(w, meta, q, lib.FP8_SPARSE_B, dc, dw, c)
                    ws, nb = lib._workspace("fp8_sparse24_gemm_workspace_size", ctypes.byref(args), None, "cuda")
                    prob = lib.sparse_weight_problem(q, w, meta, dc, dw, c)
                    fn = L.fp8_sparse24_gemm
                else:
                    args = lib.gemm_args(q, w, dc, dw, c)
                    ws, nb = lib._workspace("fp8_gemm_workspace_size", ctypes.byref(args), None, "cuda")
                    prob = lib.dense_problem(q, w, dc, dw, c)
                    fn = L.fp8_gemm
                reqs.append((x, q, sc, dc, c, args, ws, nb, fn, prob))
            torch.cuda.synchronize()

            def per_request():
                for i, (x, q, sc, dc, c, args, ws, nb, fn, _) in enumerate(reqs):
                    st = streams[i % 4]
                    lib.fp8_quantize(x, 0, lib.FP8_SCALE_ROW, q=q, scale=sc, descale=dc, stream=st)
                    fn(ctypes.byref(args), None, None if ws is None else ws.data_ptr(), nb, st.cuda_stream)

            def span(fn_issue):
                e0 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for st in streams:
                    st.wait_event(e0)
                fn_issue()
                ends = []
                for st in streams:
                    e = torch.cuda.Event(enable_timing=True)
                    e.record(st)
                    ends.append(e)
                torch.cuda.synchronize()
                return max(e0.elapsed_time(e) for e in ends)

            t0 = time.perf_counter()
            plan = lib.GroupedPlan([r[9] for r in reqs], use_graph=True)
            row["plan_build_us"].append((time.perf_counter() - t0) * 1e6)

            def grouped():
                st = streams[0]
                for (x, q, sc, dc, *_r) in reqs:
                    lib.fp8_quantize(x, 0, lib.FP8_SCALE_ROW, q=q, scale=sc, descale=dc, stream=st)
                plan.run(st)

            span(per_request)
            span(grouped)
            row["per_request_4_streams_ms"].append(min(span(per_request) for _ in range(3)))
            row["grouped_ms"].append(min(span(grouped) for _ in range(3)))
            plan.close()
            del reqs
        row["per_request_median_ms"] = float(np.median(row["per_request_4_streams_ms"]))
        row["grouped_median_ms"] = float(np.median(row["grouped_ms"]))
        row["grouped_speedup"] = row["per_request_median_ms"] / row["grouped_median_ms"]
        out.append(row)
    return out


def bench_encode(lib, stream, sizes=(256, 512, 2048, 8192)):
    """The 2:4 encode step (the overhead the paper measures apart from the
    GEMM): FP32 -> codes -> pruned and compressed, per-row scales, as two
    launches (quantize, then prune) and as the fused pass; one side and both
    sides (two operands of the same size)."""
    import torch
    out = []
    for S in sizes:
        g = torch.Generator(device="cuda").manual_seed(S)
        x = torch.randn((S, S), dtype=torch.float32, device="cuda", generator=g)
        q, _, _ = lib.fp8_quantize(x, 0, lib.FP8_SCALE_ROW, stream=stream)
        # one untimed call of each kernel first (the first launch loads the code)
        lib.fp8_sparse24_prune_compress(q, 0, with_mask=False, stream=stream)
        lib.fp8_quantize_prune24(x, 0, lib.FP8_SCALE_ROW, with_mask=False, stream=stream)
        n = 50 if S <= 2048 else 20
        t_q = time_events(lambda: lib.fp8_quantize(x, 0, lib.FP8_SCALE_ROW, stream=stream), n, stream)
        t_p = time_events(lambda: lib.fp8_sparse24_prune_compress(q, 0, with_mask=False, stream=stream), n, stream)
        t_f = time_events(lambda: lib.fp8_quantize_prune24(x, 0, lib.FP8_SCALE_ROW, with_mask=False, stream=stream),
                          n, stream)
        elems = S * S
        out.append({"rows": S, "K": S, "quantize_us": t_q * 1e3, "prune_us": t_p * 1e3,
                    "quantize_then_prune_us": (t_q + t_p) * 1e3, "fused_us": t_f * 1e3,
                    "fused_gbs": elems * (4 + 0.5 + 0.125) / t_f / 1e6,
                    "both_sides_fused_us": 2 * t_f * 1e3})
        del x, q
    return out


def bench_shape(lib, M, N, K, fa, stream, iters=20, tune=True, rotate=1, sparse_too=True):
    """One shape of the sweep: tuned dense and 2:4 (on the identical pruned A)
    timings; B rotated over `rotate` copies so large caches cannot hold it."""
    import torch
    from paper_2602_10262_amd import synth
    xa = torch.from_numpy(synth.normal_outliers(7, (M, K))).cuda()
    qa, _, da = lib.fp8_quantize(xa, fa, lib.FP8_SCALE_ROW)
    del xa
    xb = torch.from_numpy(synth.normal_outliers(8, (N, K))).cuda()
    qb, _, db = lib.fp8_quantize(xb, 0, lib.FP8_SCALE_ROW)
    del xb
    bs = [qb] + [qb.clone() for _ in range(rotate - 1)]
    c = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")
    res = {"M": M, "N": N, "K": K, "a_fmt": "E5M2" if fa else "E4M3"}
    flops = 2.0 * M * N * K
    byts = M * K + N * K + 2 * M * N
    # dense on the pruned A (the same matrix the 2:4 kernel sees)
    values, meta, _ = lib.fp8_sparse24_prune_compress(qa, fa, with_mask=False)
    pruned = lib.fp8_sparse24_decompress(values, meta, K)
    gargs = lib.gemm_args(pruned, qb, da, db, c, fa, 0)
    if tune and sparse_too:
        # dense on the pruned A against 2:4 on A: both tuned, record kept by the library
        sargs0 = lib.sparse24_args(values, meta, qb, lib.FP8_SPARSE_A, da, db, c, fa, 0)
        res["breakeven_A"] = lib.fp8_tune_sparse_vs_dense(sargs0, gargs, iters=3, stream=stream)
    elif tune:
        lib.fp8_tune_gemm(gargs, iters=3, stream=stream)
    it = [0]

    def dense():
        lib.fp8_gemm(pruned, bs[it[0] % rotate], da, db, fa, 0, c=c, stream=stream)
        it[0] += 1
    for _ in range(3):
        dense()
    ms = time_events(dense, iters, stream)
    res["dense_ms"] = ms
    res["dense_tflops"] = flops / ms / 1e9
    res["dense_frac_peak"] = res["dense_tflops"] / PEAK_FP8_TFLOPS
    res["dense_gbs"] = byts / ms / 1e6
    res["plan"] = lib.fp8_gemm_plan_resolve(gargs)
    if sparse_too:
        sargs = lib.sparse24_args(values, meta, qb, lib.FP8_SPARSE_A, da, db, c, fa, 0)
        if tune:
            lib.fp8_tune_sparse24_gemm(sargs, iters=3, stream=stream)

        def sparse():
            lib.fp8_sparse24_gemm(values, meta, bs[it[0] % rotate], lib.FP8_SPARSE_A, da, db, fa, 0, c=c,
                                  stream=stream)
            it[0] += 1
        for _ in range(3):
            sparse()
        sms = time_events(sparse, iters, stream)
        res["sparse_ms"] = sms
        res["sparse_tflops_dense_equiv"] = flops / sms / 1e9
        res["sparse_frac_2to4_peak"] = res["sparse_tflops_dense_equiv"] / PEAK_FP8_SPARSE_TFLOPS
        res["speedup_2to4_vs_dense"] = ms / sms
        # weight-side 2:4 (the serving form): C = A x B' with B compressed
        wv, wm, _ = lib.fp8_sparse24_prune_compress(qb, 0, with_mask=False)
        wargs = lib.sparse24_args(wv, wm, qa, lib.FP8_SPARSE_B, da, db, c, 0, fa)
        if tune:
            wpruned = lib.fp8_sparse24_decompress(wv, wm, K)
            res["breakeven_B"] = lib.fp8_tune_sparse_vs_dense(wargs, lib.gemm_args(qa, wpruned, da, db, c, fa, 0),
                                                              iters=3, stream=stream)
        wms = time_events(lambda: lib.fp8_sparse24_gemm(wv, wm, qa, lib.FP8_SPARSE_B, da, db, 0, fa, c=c,
                                                        stream=stream), iters, stream)
        res["weight_sparse_ms"] = wms
        res["speedup_weight_2to4_vs_dense"] = ms / wms
    return res


def bench_grouped(lib, stream, seed=0, count=64):
    """64 transformer-shaped problems in one persistent launch (graph
    replay) against 64 plain launches of the same problems on one stream."""
    import torch
    from paper_2602_10262_amd import synth
    rng = np.random.default_rng(seed)
    pairs = [(4096, 4096), (14336, 4096), (4096, 14336), (12288, 4096)]
    Ms = synth.log_uniform_int(rng, 1, 4096, count)
    nk = [pairs[i] for i in rng.integers(0, 4, count)]
    sparse = np.zeros(count, bool)
    sparse[rng.permutation(count)[: count // 2]] = True
    probs, keep, plain = [], [], []
    flops = 0.0
    wbytes = 0
    L = lib.load()
    sh = stream.cuda_stream
    import ctypes
    for i in range(count):
        M, (N, K) = int(Ms[i]), nk[i]
        xa = torch.from_numpy(synth.normal_outliers(1000 + i, (M, K))).cuda()
        qa, _, da = lib.fp8_quantize(xa, 0, lib.FP8_SCALE_ROW)
        w = torch.randn((N, K), device="cuda")
        qw, _, dw = lib.fp8_quantize(w, 0, lib.FP8_SCALE_ROW)
        del w, xa
        c = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")
        if sparse[i]:
            v, m, _ = lib.fp8_sparse24_prune_compress(qw, 0, with_mask=False)
            probs.append(lib.sparse_weight_problem(qa, v, m, da, dw, c))
            args = lib.sparse24_args(v, m, qa, lib.FP8_SPARSE_B, da, dw, c)
            ws, nb = lib._workspace("fp8_sparse24_gemm_workspace_size", ctypes.byref(args), None, "cuda")
            plain.append((L.fp8_sparse24_gemm, args, ws, nb))
            keep.append((qa, v, m, da, dw, c, ws))
            wbytes += N * K * 5 // 8
        else:
            probs.append(lib.dense_problem(qa, qw, da, dw, c))
            args = lib.gemm_args(qa, qw, da, dw, c)
            ws, nb = lib._workspace("fp8_gemm_workspace_size", ctypes.byref(args), None, "cuda")
            plain.append((L.fp8_gemm, args, ws, nb))
            keep.append((qa, qw, da, dw, c, ws))
            wbytes += N * K
        flops += 2.0 * M * N * K
    torch.cuda.synchronize()
    refs = [(fn, ctypes.byref(a), None if ws is None else ws.data_ptr(), nb) for fn, a, ws, nb in plain]

    def run_plain():
        for fn, a, w, nb in refs:
            fn(a, None, w, nb, sh)
    res = {"problems": count, "flops": flops, "weight_bytes": wbytes,
           "M": {"min": int(Ms.min()), "median": int(np.median(Ms)), "max": int(Ms.max())},
           "sparse_problems": int(sparse.sum())}
    # plain per-problem launches, issued straight through the C ABI
    run_plain()
    plain_ms = time_events(run_plain, 5, stream)
    res["plain_ms"] = plain_ms
    res["plain_tflops"] = flops / plain_ms / 1e9
    # the library's grouped tuner picks the tile; the plan then replays from a HIP graph
    tile, tune_us = lib.fp8_grouped_tune(probs, iters=5, stream=stream)
    res["tuner"] = {"tile": tile, "median_us": tune_us}
    plan = lib.GroupedPlan(probs, tile=tile, use_graph=True)
    plan.run(stream)
    ms = time_events(lambda: plan.run(stream), 5, stream)
    res["grouped_tile"] = tile
    res["grouped_info"] = plan.info()
    plan.close()
    default_plan = lib.GroupedPlan(probs, use_graph=True)
    default_plan.run(stream)
    res["default_tile"] = default_plan.info()["tile"]
    res["default_ms"] = time_events(lambda: default_plan.run(stream), 5, stream)
    default_plan.close()
    res["grouped_ms"] = ms
    res["grouped_tflops"] = flops / ms / 1e9
    res["speedup_vs_plain"] = plain_ms / ms
    # rooflines of the drawn instance: each problem alone at its own bound,
    # and all of them overlapped
    f_g = 2.0 * Ms * np.array([n for n, _ in nk]) * np.array([k for _, k in nk])
    peak = np.where(sparse, PEAK_FP8_SPARSE_TFLOPS, PEAK_FP8_TFLOPS) * 1e12
    b_g = np.array([M * K + (N * K * 5 // 8 if sp else N * K) + 2 * M * N
                    for M, (N, K), sp in zip(Ms, nk, sparse)], dtype=np.float64)
    res["serial_roofline_ms"] = float(np.sum(np.maximum(f_g / peak, b_g / (PEAK_HBM_GBS * 1e9)))) * 1e3
    res["overlapped_roofline_ms"] = float(max(np.sum(f_g / peak), np.sum(b_g) / (PEAK_HBM_GBS * 1e9))) * 1e3
    return res


def bench_served(lib, n_requests=20000, seed=0, rates=(0.5, 1.0, 1.5), budgets=(2 << 30,), streams=4, slots=64):
    """Poisson stream of dense / 2:4 GEMM requests through the server on
    `streams` streams against the same arrivals served one at a time.
    Request r writes output slot r % slots; before it is submitted, the
    request that last used that slot has completed (slots exceeds the number
    of requests in flight), so no two live requests share an output."""
    import torch
    from paper_2602_10262_amd import synth
    rng = np.random.default_rng(seed)
    sizes = [2048, 4096, 8192, 14336]
    Mmax = 8192
    # resident weights: one per (N, K, dense | 2:4)
    weights = {}
    for N in sizes:
        for K in sizes:
            w = torch.randn((N, K), device="cuda")
            qw, _, dw = lib.fp8_quantize(w, 0, lib.FP8_SCALE_ROW)
            del w
            v, m, _ = lib.fp8_sparse24_prune_compress(qw, 0, with_mask=False)
            weights[(N, K)] = (qw, v, m, dw)
    pools = {K: torch.from_numpy(synth.uniform(seed, K, (Mmax, K))).cuda() for K in sizes}
    out_slots = [torch.empty(Mmax * max(sizes), dtype=torch.bfloat16, device="cuda") for _ in range(slots)]
    torch.cuda.synchronize()   # the server's streams are not ordered after torch's
    Ms = synth.log_uniform_int(rng, 1, Mmax, n_requests)
    Ns = rng.choice(sizes, n_requests)
    Ks = rng.choice(sizes, n_requests)
    sp = rng.random(n_requests) < 0.5
    offs = [int(rng.integers(0, Mmax - M + 1)) for M in Ms]
    flops = float(np.sum(2.0 * Ms * Ns * Ks))

    def run(arrivals, nstreams, max_inflight, budget=budgets[0]):
        srv = lib.Server(budget, nstreams, max_inflight)
        ids = {}
        for (N, K), (qw, v, m, dw) in weights.items():
            ids[(N, K, False)] = srv.register_weight(qw, None, dw, N, K)
            ids[(N, K, True)] = srv.register_weight(v, m, dw, N, K)
        t0 = srv.now() + 0.05
        tickets = []
        for r in range(n_requests):
            M, N, K = int(Ms[r]), int(Ns[r]), int(Ks[r])
            x_ptr = pools[K].data_ptr() + offs[r] * K * 4
            if r >= slots:
                # the slot's previous request must be done before its output is reused
                srv.wait(tickets[r - slots], -1)
            tickets.append(srv.submit(M, ids[(N, K, bool(sp[r]))], x_ptr=x_ptr,
                                      c_ptr=out_slots[r % slots].data_ptr(),
                                      arrival_time_s=t0 + float(arrivals[r])))
        srv.drain()
        st = srv.stats()
        srv.close()
        return st

    # serial capacity: all requests present at once, one at a time
    cap = run(np.zeros(n_requests), 1, 1)
    mu = n_requests / cap["span_s"]
    res = {"requests": n_requests, "flops": flops, "serial_capacity_req_s": mu,
           "serial_capacity_tflops": cap["tflops"], "streams": streams, "budgets_bytes": list(budgets), "rates": []}
    # per-stream busy-time balance under least-loaded placement (the streams
    # carry different work, so this is a load-balance figure, not the paper's
    # fairness over equal per-stream workloads, which the ACE study reports)
    keys = ("p50_ms", "p99_ms", "mean_ms", "tflops", "stream_cv", "peak_inflight", "peak_bytes", "done")
    for f in rates:
        lam = f * mu
        arr = synth.poisson_arrivals(np.random.default_rng(seed + 1), lam, n_requests)
        serial = run(arr, 1, 1)
        row = {"load": f, "rate_req_s": lam, "serial": {k: serial[k] for k in keys}, "served": {}}
        for budget in budgets:
            served = run(arr, streams, 4 * streams, budget)
            row["served"][str(budget >> 30) + "GiB"] = {k: served[k] for k in keys}
            log(f"served load {f} budget {budget >> 30} GiB: p50 {served['p50_ms']:.2f} ms p99 "
                f"{served['p99_ms']:.2f} ms {served['tflops']:.0f} TF/s | serial p50 {serial['p50_ms']:.2f} "
                f"p99 {serial['p99_ms']:.2f} {serial['tflops']:.0f} TF/s")
        res["rates"].append(row)
    return res


def bench_ubench(lib, stream):
    """Matrix-core and LDS microbenchmarks (the paper's Sec. 5 MFMA study on
    gfx950): throughput against resident waves per CU, dependent-issue
    latency, LDS read bandwidth."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    iters = 2000
    out = {"cus": cus, "throughput": [], "latency": [], "lds": [],
           "sclk_ghz_under_mfma_load": lib.fp8_ubench_clock(20000, stream)}
    for kind, (name, mnk) in lib.UBENCH_KINDS.items():
        for waves in (1, 2, 4, 8, 16):
            chains = 8 if kind in (0, 2) else 4
            ms = lib.fp8_ubench_mfma(kind, waves, chains, iters, stream)
            n_instr = cus * waves * chains * iters
            out["throughput"].append({"instr": name, "waves_per_cu": waves, "chains": chains,
                                      "tflops_dense_equiv": 2.0 * mnk * n_instr / (ms * 1e-3) / 1e12,
                                      "ns_per_instr_per_wave": ms * 1e6 / (chains * iters)})
        ms = lib.fp8_ubench_mfma(kind, 1, 1, iters, stream)
        out["latency"].append({"instr": name, "ns_dependent_issue": ms * 1e6 / iters})
    for waves in (1, 4, 8, 16):
        ms = lib.fp8_ubench_lds(waves, 4096, stream)
        nbytes = cus * waves * 64 * 16 * 4096
        out["lds"].append({"waves_per_cu": waves, "tbs": nbytes / (ms * 1e-3) / 1e12})
    # every swizzle of a compressed (64-byte) row that XORs row bits into the
    # chunk index, on the compressed-fragment read: time relative to a linear
    # read of the same bytes (about 1: conflict-free, about 1.7: 2-way)
    lin = [16 * l for l in range(64)]
    lib.fp8_ubench_lds_offsets(lin, 8, 16, stream)
    t_lin = min(lib.fp8_ubench_lds_offsets(lin, 8, 2048, stream) for _ in range(3))
    sweep = {}
    for m0 in range(16):
        for m1 in range(16):
            def h(r):
                return (bin(m0 & r).count("1") & 1) | ((bin(m1 & r).count("1") & 1) << 1)
            offs = [(l & 15) * 64 + (((l >> 4) ^ h(l & 15)) << 4) for l in range(64)]
            sweep[(m0, m1)] = min(lib.fp8_ubench_lds_offsets(offs, 8, 2048, stream) for _ in range(2)) / t_lin
    vals = sorted(sweep.values())
    out["compressed_swizzle_sweep"] = {
        "candidates": len(vals), "conflict_free": sum(v < 1.3 for v in vals),
        "two_way": sum(1.3 <= v < 2.5 for v in vals), "four_way": sum(v >= 2.5 for v in vals),
        "library_swizzle_rel_time": sweep[(2, 8)], "previous_swizzle_rel_time": sweep[(10, 4)],
        "unswizzled_rel_time": sweep[(0, 0)]}
    # the address patterns of the GEMM fragment reads, 8 waves per CU
    out["lds_patterns"] = []
    for pat, name in lib.LDS_PATTERNS.items():
        ms = lib.fp8_ubench_lds_pattern(pat, 8, 4096, stream)
        per_lane = {4: 4, 6: 8}.get(pat, 16)
        nbytes = cus * 8 * 64 * per_lane * 4096
        out["lds_patterns"].append({"pattern": name, "tbs": nbytes / (ms * 1e-3) / 1e12,
                                    "ns_per_instr_per_wave": ms * 1e6 / 4096})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--quick", action="store_true", help="headline GEMM, 2:4 and quantize only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tune", action="store_true", help="use the library's default plan")
    ap.add_argument("--sweep", action="store_true", help="also the square and skinny sweep with 2:4 break-even")
    ap.add_argument("--requests", type=int, default=20000, help="served stream length")
    ap.add_argument("--served-sweep", action="store_true",
                    help="served stream at 0.25..2.0 x serial capacity and 1, 2, 8 GiB budgets")
    ap.add_argument("--ace-only", action="store_true", help="only the concurrent-stream study (for counter runs)")
    ap.add_argument("--ubench-only", action="store_true", help="only the matrix-core and LDS microbenchmarks")
    ap.add_argument("--mixed-only", action="store_true", help="only the mixed-precision GEMMs and chains")
    ap.add_argument("--batching-only", action="store_true", help="only the per-request vs grouped batch study")
    ap.add_argument("--exact-only", action="store_true", help="only the exact-sum tiles (K below 3584)")
    ap.add_argument("--served-only", action="store_true",
                    help="only the served stream (with --served-sweep: all rates and budgets)")
    ap.add_argument("--out", default=None, help="also write the JSON line to this file")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only launch the headline GEMM and its 2:4 form 3 times each and a 1 GiB device copy "
                         "(for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the GEMM would shard by "
              "columns of B with no exchange; that is not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2602_10262_amd as lib
    lib.load()
    torch.cuda.init()
    # a stream of our own: the grouped leg captures a HIP graph on it
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    M = N = K = args.size
    if args.ace_only or args.ubench_only or args.mixed_only or args.batching_only or args.served_only or args.exact_only:
        if args.exact_only:
            res = {"exact": bench_exact(lib, stream)}
        elif args.served_only:
            if args.served_sweep:
                res = {"served": bench_served(lib, n_requests=args.requests,
                                              rates=(0.25, 0.5, 0.75, 1.0, 1.25, 1.5, 2.0),
                                              budgets=(1 << 30, 2 << 30, 8 << 30))}
            else:
                res = {"served": bench_served(lib, n_requests=args.requests)}
        elif args.batching_only:
            res = {"batching": bench_batching(lib, stream)}
        elif args.ace_only:
            res = {"ace": bench_ace(lib, stream)}
        elif args.ubench_only:
            res = {"ubench": bench_ubench(lib, stream)}
        else:
            res = {"mixed": bench_mixed(lib, stream)}
        print(json.dumps(res), flush=True)
        return
    if args.traffic_probe:
        xa, xb, qa, da, qb, db = make_operands(lib, M, N, K, 0)
        c = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")
        for _ in range(3):
            lib.fp8_gemm(qa, qb, da, db, c=c, stream=stream)
        # the 2:4 GEMM of the same shape (A pruned), on its default plan
        va, ma, _ = lib.fp8_sparse24_prune_compress(qa, 0, with_mask=False, stream=stream)
        for _ in range(3):
            lib.fp8_sparse24_gemm(va, ma, qb, lib.FP8_SPARSE_A, da, db, c=c, stream=stream)
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"traffic probe done; kernel_source_sha1: {kernel_source_hash()}", flush=True)
        return
    log(f"bench: dense FP8 GEMM {M}x{N}x{K}")
    xa, xb, qa, da, qb, db = make_operands(lib, M, N, K, 0)
    c = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")
    gargs = lib.gemm_args(qa, qb, da, db, c)
    # The headline runs the library's default plan for the shape (what a
    # caller gets without tuning), so the same kernel is the one the
    # rocprofv3 summaries and the traffic counters describe; the autotuner's
    # pick is timed separately below.
    lib.fp8_tune_cache_clear()
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

    tuned = None
    if not args.no_tune:
        (tile, split), us = lib.fp8_tune_gemm(gargs, iters=5, stream=stream)
        # a split-K plan takes its workspace from torch's caching allocator
        tms = time_events(lambda: lib.fp8_gemm(qa, qb, da, db, c=c, plan=(tile, split), stream=stream),
                          max(5, args.steps // 2), stream)
        tuned = {"tile": tile, "split_k": split, "ms": tms, "tflops": flops / (tms * 1e-3) / 1e12}
        log(f"tuned plan: tile {tile} split {split}: {tms:.3f} ms -> {tuned['tflops']:.1f} TFLOP/s")
        lib.fp8_tune_cache_clear()
    extra = {"plan": {"tile": plan_tile, "split_k": plan_split}, "tuned": tuned}
    # quantize pass (per-row, A operand): 4 B read + 1 B written per element
    lib.fp8_quantize(xa, 0, lib.FP8_SCALE_ROW, stream=stream)   # first launch loads the kernel
    qms = time_events(lambda: lib.fp8_quantize(xa, 0, lib.FP8_SCALE_ROW, stream=stream), 20, stream)
    extra["quantize_per_row"] = {"ms": qms, "gbs": M * K * 5 / qms / 1e6}
    extra["sparse24"] = bench_sparse(lib, qa, da, qb, db, max(5, args.steps // 2), 3, stream)
    extra["ubench"] = bench_ubench(lib, stream)
    extra["encode"] = bench_encode(lib, stream)
    extra["exact"] = bench_exact(lib, stream)
    log(f"2:4: {extra['sparse24']['sparse_tflops_dense_equiv']:.1f} TFLOP/s dense-equivalent, "
        f"{extra['sparse24']['speedup_vs_dense']:.2f}x vs dense on the pruned matrix")
    del xa, xb, c
    torch.cuda.empty_cache()

    if not args.quick:
        # 256^3: uniform [-1, 1) inputs, per-tensor 448/amax scales, FP32 out
        from paper_2602_10262_amd import synth
        x1 = torch.from_numpy(synth.uniform(0, 0, (256, 256))).cuda()
        y1 = torch.from_numpy(synth.uniform(0, 1, (256, 256))).cuda()
        q1, _, d1 = lib.fp8_quantize(x1, 0, lib.FP8_SCALE_TENSOR, stream=stream)
        r1, _, e1 = lib.fp8_quantize(y1, 0, lib.FP8_SCALE_TENSOR, stream=stream)
        c1 = torch.empty((256, 256), dtype=torch.float32, device="cuda")
        ms1 = time_events(lambda: lib.fp8_gemm(q1, r1, d1, e1, c=c1, stream=stream), 200, stream)
        extra["gemm_256"] = {"us": ms1 * 1e3, "tflops": 2.0 * 256 ** 3 / (ms1 * 1e-3) / 1e12,
                             "plan": list(lib.fp8_gemm_plan_resolve(lib.gemm_args(q1, r1, d1, e1, c1)))}
        log(f"256^3 per-tensor FP32 out: {ms1 * 1e3:.2f} us per launch")
        log("grouped: 64 problems ...")
        extra["grouped"] = bench_grouped(lib, stream)
        log(f"grouped {extra['grouped']['grouped_tflops']:.0f} TF/s vs plain {extra['grouped']['plain_tflops']:.0f}")
        torch.cuda.empty_cache()
        log("concurrent streams (512^3) ...")
        extra["ace"] = bench_ace(lib, stream)
        torch.cuda.empty_cache()
        log("mixed-precision chains ...")
        extra["mixed"] = bench_mixed(lib, stream)
        torch.cuda.empty_cache()
        log("batching admitted requests ...")
        extra["batching"] = bench_batching(lib, stream)
        torch.cuda.empty_cache()
        log("served stream ...")
        if args.served_sweep:
            extra["served"] = bench_served(lib, n_requests=args.requests,
                                           rates=(0.25, 0.5, 0.75, 1.0, 1.25, 1.5, 2.0),
                                           budgets=(1 << 30, 2 << 30, 8 << 30))
        else:
            extra["served"] = bench_served(lib, n_requests=args.requests)
        torch.cuda.empty_cache()
        # skinny shapes of the sweep (HBM-bound), B rotated past the caches
        extra["skinny"] = [bench_shape(lib, m, 8192, 8192, 0, stream, rotate=5) for m in (16, 64, 256)]
    if args.sweep:
        sweep = []
        for S in (1024, 2048, 4096, 8192, 16384):
            for fa in (0, 1):
                log(f"sweep {S}^3 fa={fa}")
                sweep.append(bench_shape(lib, S, S, S, fa, stream))
                torch.cuda.empty_cache()
        for m in (16, 64, 256):
            sweep.append(bench_shape(lib, m, 8192, 8192, 1, stream, rotate=5))
        sweep.append(bench_shape(lib, 512, 2048, 1024, 0, stream))
        extra["sweep"] = sweep
        # the dense-vs-2:4 records the library's tuner kept for these shapes
        extra["breakeven_records"] = lib.fp8_tune_breakeven_records()
        lib.fp8_tune_cache_save(os.path.join(ROOT, "gpurun_out", "tune_cache.jsonl")) if os.path.isdir(
            os.path.join(ROOT, "gpurun_out")) else None

    sclk = extra["ubench"]["sclk_ghz_under_mfma_load"]
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
                     "frac": achieved / PEAK_FP8_TFLOPS, "traffic": measured_traffic() if M == 8192 else None,
                     # the peak assumes 2.4 GHz; the engine clock this GPU showed under an MFMA load
                     # (s_memtime against the constant-rate wall clock), and the fraction of the
                     # peak scaled to that clock
                     "sclk_ghz_mfma_load": sclk,
                     "frac_at_that_sclk": achieved / (PEAK_FP8_TFLOPS * sclk / 2.4) if sclk else None},
        "extra": extra,
    }
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(M, N, K)
    line = json.dumps(out)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    print(line, flush=True)


if __name__ == "__main__":
    main()
