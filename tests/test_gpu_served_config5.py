"""The serving runtime at the served workload's full sizes: a seeded sample of
200 requests (tokens log-uniform on [1, 8192], N and K from {2048, 4096, 8192,
14336}, half dense and half 2:4 on the weight side, uniform activations,
N(0,1) weights) runs as one mix on 4 streams under a 2 GiB transient budget.
Each result meets the bound against the oracle on sampled outputs and equals,
bit for bit, the same request run alone."""
import numpy as np
import pytest

import oracle as orc
from paper_2602_10262_amd import synth
from tests.helpers import dev, host, log

pytestmark = pytest.mark.gpu

SIZES = [2048, 4096, 8192, 14336]


def test_served_sample_full_sizes_oracle_and_alone(gpu):
    import torch
    rng = np.random.default_rng(2024)
    n = 200
    Ms = synth.log_uniform_int(rng, 1, 8192, n)
    Ns = rng.choice(SIZES, n)
    Ks = rng.choice(SIZES, n)
    sparse = rng.random(n) < 0.5
    # weights: one per (N, K); the 2:4 weight is the pruned dense one
    W = {}
    for wi, (N, K) in enumerate(sorted({(int(a), int(b)) for a, b in zip(Ns, Ks)})):
        xw = synth.normal_outliers(9000 + wi, (N, K), p_outlier=0.0)
        qw, _, dw = orc.quantize(xw, orc.E4M3, True)
        del xw
        v, m, _, pw = orc.prune24(qw, orc.E4M3)
        W[(N, K)] = dict(qw=qw, dw=dw, pw=pw, d_qw=dev(qw), d_v=dev(v), d_m=dev(m), d_dw=dev(dw))
    log(f"served sample: {n} requests, {len(W)} weight shapes, tokens median {int(np.median(Ms))} max {Ms.max()}")

    def make_server(streams, inflight):
        srv = gpu.Server(2 << 30, streams, inflight)
        ids = {}
        for key, w in W.items():
            ids[(key, False)] = srv.register_weight(w["d_qw"], None, w["d_dw"], key[0], key[1])
            ids[(key, True)] = srv.register_weight(w["d_v"], w["d_m"], w["d_dw"], key[0], key[1])
        return srv, ids

    xs, outs, samples = [], [], []
    for r in range(n):
        M, N, K = int(Ms[r]), int(Ns[r]), int(Ks[r])
        x = synth.uniform(31, 100000 + r, (M, K))
        xs.append(dev(x))
        outs.append(torch.full((M, N), float("nan"), dtype=torch.bfloat16, device="cuda"))
        # sampled outputs: 60 random positions and the four corners; the
        # oracle needs only their rows (quantization is per row)
        srng = np.random.default_rng(r)
        ii = np.concatenate([srng.integers(0, M, 60), [0, 0, M - 1, M - 1]])
        jj = np.concatenate([srng.integers(0, N, 60), [0, N - 1, 0, N - 1]])
        rows, inv = np.unique(ii, return_inverse=True)
        samples.append((rows, x[rows].copy(), inv, jj))
        del x
    torch.cuda.synchronize()   # inputs and outputs ready before the server's streams see them
    srv, ids = make_server(4, 0)
    tickets = [srv.submit(int(Ms[r]), ids[((int(Ns[r]), int(Ks[r])), bool(sparse[r]))], xs[r], outs[r])
               for r in range(n)]
    for t in tickets:
        assert srv.wait(t, 120_000_000) == gpu.FP8_OK
    st = srv.stats()
    srv.close()
    log(f"mix: done {st['done']} peak in flight {st['peak_inflight']} peak bytes {st['peak_bytes']}")
    assert st["done"] == n and st["failed"] == 0

    alone_srv, alone_ids = make_server(1, 1)
    worst = 0.0
    for r in range(n):
        M, N, K = int(Ms[r]), int(Ns[r]), int(Ks[r])
        key = (N, K)
        c = torch.full((M, N), float("nan"), dtype=torch.bfloat16, device="cuda")
        torch.cuda.synchronize()
        t = alone_srv.submit(M, alone_ids[(key, bool(sparse[r]))], xs[r], c)
        assert alone_srv.wait(t, 120_000_000) == gpu.FP8_OK
        assert torch.equal(c.view(torch.int16), outs[r].view(torch.int16)), f"request {r} alone != in mix"
        # oracle on sampled outputs: it quantizes the sampled rows of the same
        # FP32 activations itself (per-row scales, so rows are independent)
        rows, xrows, inv, jj = samples[r]
        qa, _, da = orc.quantize(xrows, orc.E4M3, True)
        wq = W[key]["pw"] if sparse[r] else W[key]["qw"]
        cref, sabs = orc.gemm_at(qa, orc.E4M3, wq, orc.E4M3, da, W[key]["dw"], inv, jj)
        ii = rows[inv]
        got = host(outs[r].view(-1)[torch.from_numpy(ii * N + jj).cuda()])
        res = orc.check(got, cref, sabs, K, orc.OUT_BF16)
        worst = max(worst, res["max_ratio"])
        assert res["ok"], (r, M, N, K, bool(sparse[r]), res)
        if r % 25 == 0:
            log(f"  request {r}: M={M} N={N} K={K} sparse={bool(sparse[r])} max_ratio={res['max_ratio']:.3e}")
    alone_srv.close()
    log(f"served sample: all {n} alone == in mix; worst max_ratio {worst:.3e}")
