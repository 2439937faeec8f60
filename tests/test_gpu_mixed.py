"""GPU parity of the FP32 / FP16 / BF16 GEMMs (the higher-precision stages of
the mixed-precision sequence) against the FP64 oracle, and of the chain
executor: every stage of every chain against the oracle on the stage's own
GPU input, results identical under every schedule."""
import numpy as np
import pytest

import oracle as orc
from paper_2602_10262_amd import synth
from tests.helpers import dev, host, log

pytestmark = pytest.mark.gpu

OUT = {"f32": orc.OUT_F32, "bf16": orc.OUT_BF16, "f16": orc.OUT_F16}


def _dtypes():
    import torch
    return {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}


def _padded(x, dtype):
    """A CUDA tensor of dtype holding x, with a 16-byte-multiple row stride."""
    import torch
    rows, K = x.shape
    es = torch.tensor([], dtype=dtype).element_size()
    ld = (K * es + 15) // 16 * 16 // es
    t = torch.zeros((rows, ld), dtype=dtype, device="cuda")
    t[:, :K] = torch.from_numpy(np.ascontiguousarray(x)).cuda().to(dtype)
    return t[:, :K]


def _values(t) -> np.ndarray:
    """Exact FP64 values of a CUDA tensor."""
    import torch
    return t.to(torch.float64).cpu().numpy()


@pytest.mark.parametrize("M,N,K", [(64, 64, 64), (77, 45, 200), (130, 260, 384), (300, 17, 1000), (1, 256, 512),
                                   (513, 129, 136), (40, 300, 3600), (256, 256, 4096)])
@pytest.mark.parametrize("ab", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("out", ["f32", "bf16", "f16"])
def test_hp_gemm_parity(gpu, M, N, K, ab, out):
    import torch
    dt = _dtypes()
    xa = synth.normal_outliers(M + K, (M, K))
    xb = synth.normal_outliers(N + 2 * K, (N, K))
    a = _padded(xa, dt[ab])
    b = _padded(xb, dt[ab])
    rng = np.random.default_rng(M * N)
    sa = rng.uniform(0.5, 2.0, M).astype(np.float32)
    sb = rng.uniform(0.5, 2.0, N).astype(np.float32)
    log(f"hp gemm {ab}->{out} M={M} N={N} K={K}")
    c = gpu.fp8_hp_gemm(a, b, dev(sa), dev(sb), out_dtype=dt[out])
    torch.cuda.synchronize()
    cref, sabs = orc.gemm_real(_values(a), _values(b), sa, sb)
    res = orc.check(_values(c), cref, sabs, K, OUT[out])
    log(f"  max_ratio={res['max_ratio']:.3e} normwise={res['normwise']:.3e}")
    assert res["ok"], res


@pytest.mark.parametrize("ab", ["f32", "f16", "bf16"])
def test_hp_gemm_all_ones_and_identity_exact(gpu, ab):
    import torch
    dt = _dtypes()
    K = 1000
    c = gpu.fp8_hp_gemm(_padded(np.ones((33, K), np.float32), dt[ab]), _padded(np.ones((17, K), np.float32), dt[ab]))
    torch.cuda.synchronize()
    assert bool(torch.all(c == K))
    x = synth.normal_outliers(3, (40, 64)).astype(np.float32)
    a = _padded(x, dt[ab])
    c = gpu.fp8_hp_gemm(a, _padded(np.eye(64, dtype=np.float32), dt[ab]))
    torch.cuda.synchronize()
    assert np.array_equal(_values(c), _values(a))


def test_fp8_gemm_fp16_output(gpu):
    """The FP8 GEMM's epilogue stores FP16 (RNE) within the FP16 bound."""
    import torch
    from tests.helpers import operands, codes_with_pad
    qa, da, qb, db = operands(96, 80, 4096, 5, "normal", 0, 0, True)
    c = gpu.fp8_gemm(codes_with_pad(96, 4096, qa), codes_with_pad(80, 4096, qb), dev(da), dev(db),
                     out_dtype=torch.float16)
    torch.cuda.synchronize()
    cref, sabs = orc.gemm(qa, 0, qb, 0, da, db)
    assert orc.check(_values(c), cref, sabs, 4096, orc.OUT_F16)["ok"]


STAGES = [("f32", 384), ("f16", 256), ("fp8", 320), ("bf16", 192), ("f32", 128)]
PREC = {"f32": 0, "f16": 1, "bf16": 2, "fp8": 3}


def _make_chain(gpu, M, in_width, n_chains, streams):
    import torch
    dt = _dtypes()
    stages, host_w = [], []
    k = in_width
    for s, (p, n) in enumerate(STAGES):
        w = synth.normal_outliers(100 + s, (n, k)).astype(np.float32) / np.sqrt(k)
        if p == "fp8":
            q, _, d = orc.quantize(w, 0, True)
            wt, sc = dev(q), dev(d)
            host_w.append((q, d))
        else:
            wt, sc = _padded(w, dt[p]), None
            host_w.append((_values(wt), None))
        stages.append((PREC[p], wt, sc))
        k = n
    ch = gpu.Chain(stages, M, in_width, n_chains, max_streams=streams)
    for c in range(n_chains):
        x = synth.normal_outliers(200 + c, (M, in_width)).astype(np.float32)
        ch.tensor(c, 0).copy_(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    return ch, host_w


def _check_chain(ch, host_w, M):
    """Every stage of every chain against the oracle on its GPU input."""
    for c in range(ch.n_chains):
        for s, (p, n) in enumerate(STAGES):
            x = _values(ch.tensor(c, s))
            y = _values(ch.tensor(c, s + 1))
            nxt = STAGES[s + 1][0] if s + 1 < len(STAGES) else "f32"
            out = OUT["f32"] if nxt in ("f32", "fp8") else OUT[nxt]
            K = x.shape[1]
            if p == "fp8":
                q, _, d = orc.quantize(x.astype(np.float32), 0, True)
                wq, wd = host_w[s]
                cref, sabs = orc.gemm(q, 0, wq, 0, d, wd)
            else:
                cref, sabs = orc.gemm_real(x, host_w[s][0])
            res = orc.check(y, cref, sabs, K, out)
            assert res["ok"], (c, s, p, res)


def test_chain_stages_against_oracle_and_schedules_agree(gpu):
    import torch
    M, in_width, n_chains = 200, 512, 3
    ch, host_w = _make_chain(gpu, M, in_width, n_chains, streams=3)
    outs = {}
    for sched, streams in [(gpu.FP8_CHAIN_SERIAL, 1), (gpu.FP8_CHAIN_IN_PHASE, 3), (gpu.FP8_CHAIN_STAGGERED, 3)]:
        st = ch.run(sched, streams)
        log(f"chain schedule={sched} streams={streams}: {st}")
        assert st["makespan_ms"] > 0 and st["stage_count"]["f32"] == 2 * n_chains
        outs[sched] = [ch.tensor(c, len(STAGES)).clone() for c in range(n_chains)]
        torch.cuda.synchronize()
    for c in range(n_chains):
        assert torch.equal(outs[0][c], outs[1][c]) and torch.equal(outs[0][c], outs[2][c])
    _check_chain(ch, host_w, M)
    ch.close()


def test_chain_rejects_bad_stages(gpu):
    import torch
    w = torch.zeros((64, 100), dtype=torch.float32, device="cuda")
    with pytest.raises(gpu.Fp8Error):
        gpu.Chain([(gpu.FP8_STAGE_FP8, torch.zeros((64, 100), dtype=torch.uint8, device="cuda"), None)], 8, 100, 1)
    with pytest.raises(gpu.Fp8Error):
        gpu.Chain([(7, w, None)], 8, 100, 1)


@pytest.mark.parametrize("tile_rows", [64, 128, 256])
@pytest.mark.parametrize("ab", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("M,N,K", [(300, 200, 1000), (513, 257, 136), (40, 600, 3600), (77, 300, 1001)])
def test_hp_gemm_every_tile(gpu, tile_rows, ab, M, N, K):
    """Each tile of the FP32 / 16-bit GEMM (64 x 64 and 128 x 128 on 256-byte
    LDS rows, 256 x 256 with 8 waves on 128-byte rows) on ragged shapes."""
    import torch
    dt = _dtypes()
    xa = synth.normal_outliers(M + 3 * K, (M, K))
    xb = synth.normal_outliers(N + 5 * K, (N, K))
    a, b = _padded(xa, dt[ab]), _padded(xb, dt[ab])
    c = gpu.fp8_hp_gemm(a, b, out_dtype=torch.float32, tile_rows=tile_rows)
    torch.cuda.synchronize()
    cref, sabs = orc.gemm_real(_values(a), _values(b))
    res = orc.check(_values(c), cref, sabs, K, orc.OUT_F32)
    log(f"hp tile {tile_rows} {ab} {M}x{N}x{K}: max_ratio={res['max_ratio']:.3e}")
    assert res["ok"], res


@pytest.mark.parametrize("ab", ["f32", "bf16"])
def test_hp_gemm_4096_sampled_rows(gpu, ab):
    """4096^3 on the default (256 x 256) tile: sampled rows against the oracle."""
    import torch
    dt = _dtypes()
    M = N = K = 4096
    g = torch.Generator(device="cuda").manual_seed(7)
    a = torch.randn((M, K), generator=g, device="cuda").to(dt[ab])
    b = torch.randn((N, K), generator=g, device="cuda").to(dt[ab])
    c = gpu.fp8_hp_gemm(a, b, out_dtype=torch.float32)
    torch.cuda.synchronize()
    rows = [0, 1, 255, 256, 2047, 4095]
    cref, sabs = orc.gemm_real(_values(a[rows]), _values(b))
    res = orc.check(_values(c[rows]), cref, sabs, K, orc.OUT_F32)
    assert res["ok"], res
