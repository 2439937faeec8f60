"""GPU parity: quantization codes/scales and 2:4 prune/compress must equal the
oracle bit for bit."""
import numpy as np
import pytest

import oracle as orc
from paper_2602_10262_amd import synth
from tests.helpers import dev, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fmt", [0, 1])
@pytest.mark.parametrize("per_row", [False, True])
@pytest.mark.parametrize("shape,dist", [((256, 256), "uniform"), ((37, 53), "normal"), ((1, 16), "normal"),
                                        ((300, 1000), "normal"), ((5, 4096), "uniform"), ((3, 8192), "normal"),
                                        ((2, 12288), "normal"), ((2, 16384), "uniform"), ((2, 16400), "normal")])
def test_quantize_bit_exact(gpu, fmt, per_row, shape, dist):
    import torch
    rows, cols = shape
    x = synth.uniform(3, 7, shape) if dist == "uniform" else synth.normal_outliers(4, shape)
    # give the host array a 4-float aligned row stride on the device
    ld = (cols + 3) // 4 * 4
    xd = torch.zeros((rows, ld), dtype=torch.float32, device="cuda")
    xd[:, :cols] = dev(x)
    q, s, d = gpu.fp8_quantize(xd[:, :cols], fmt, gpu.FP8_SCALE_ROW if per_row else gpu.FP8_SCALE_TENSOR)
    torch.cuda.synchronize()
    qo, so, do = orc.quantize(x, fmt, per_row)
    log(f"quantize fmt={fmt} per_row={per_row} shape={shape}")
    assert np.array_equal(q.cpu().numpy(), qo)
    assert np.array_equal(s.cpu().numpy().view(np.uint32), so.view(np.uint32))
    assert np.array_equal(d.cpu().numpy().view(np.uint32), do.view(np.uint32))


@pytest.mark.parametrize("fmt", [0, 1])
def test_encoder_exhaustive_over_rounding_range(gpu, fmt):
    """Every FP32 bit pattern whose binade lies in [2^-20, 2^17] (all the
    values where FP8 rounding happens, for both formats), plus a stratified
    sample of the rest of the positive and negative ranges.  Each row starts
    with +inf, so its amax is infinite and the scale is exactly 1: the codes are
    the encoder's output for the raw values."""
    import torch
    lo = (127 - 20) << 23
    n_total = 38 << 23
    row = 1 << 22
    for start in range(0, n_total, row * 8):
        n = min(row * 8, n_total - start)
        nrows = n // row
        bits = torch.arange(lo + start, lo + start + n, dtype=torch.int64, device="cuda").to(torch.int32)
        x = torch.zeros((nrows, row + 4), dtype=torch.float32, device="cuda")
        x[:, 0] = float("inf")
        x[:, 1:row + 1] = bits.view(torch.float32).reshape(nrows, row)
        q, s, d = gpu.fp8_quantize(x, fmt, gpu.FP8_SCALE_ROW)
        got = q[:, 1:row + 1].reshape(-1).cpu().numpy()
        want = orc.encode_range(fmt, lo + start, n)
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, (fmt, hex(lo + start + int(bad[0])), got[bad[0]], want[bad[0]])
        assert torch.all(s == 1.0)
    rng = np.random.default_rng(fmt)
    sample = rng.integers(0, 1 << 32, 1 << 22, dtype=np.uint64).astype(np.uint32)
    xs = sample.view(np.float32)
    x = torch.zeros((1, sample.size + 4), dtype=torch.float32, device="cuda")
    x[0, 0] = float("inf")
    x[0, 1:sample.size + 1] = dev(xs)
    q, _, _ = gpu.fp8_quantize(x, fmt, gpu.FP8_SCALE_ROW)
    got = q[0, 1:sample.size + 1].cpu().numpy()
    want = orc.encode(fmt, xs[:20000])
    assert np.array_equal(got[:20000], want)
    log(f"encoder fmt={fmt}: {n_total} patterns + sample equal")


def _prune_input(seed, rows, K, fmt, kind):
    rng = np.random.default_rng(seed)
    t = orc.decode_table(fmt)
    finite = np.flatnonzero(np.isfinite(t)).astype(np.uint8)
    if kind == "ties":          # few distinct magnitudes: many ties
        pool = np.array([0x00, 0x80, 0x38, 0xB8, 0x40, 0xC0], np.uint8)
        return rng.choice(pool, size=(rows, K))
    if kind == "specials":      # include NaN / infinity codes
        return rng.integers(0, 256, size=(rows, K)).astype(np.uint8)
    return rng.choice(finite, size=(rows, K))


@pytest.mark.parametrize("fmt", [0, 1])
@pytest.mark.parametrize("rows,K", [(64, 256), (3, 8), (17, 40), (5, 264), (129, 1024)])
@pytest.mark.parametrize("kind", ["random", "ties", "specials"])
def test_prune_bit_exact(gpu, fmt, rows, K, kind):
    import torch
    x = _prune_input(rows * 7 + K, rows, K, fmt, kind)
    ld = (K + 15) // 16 * 16
    xd = torch.zeros((rows, ld), dtype=torch.uint8, device="cuda")
    xd[:, :K] = dev(x)
    values, meta, mask = gpu.fp8_sparse24_prune_compress(xd[:, :K], fmt)
    pruned = gpu.fp8_sparse24_decompress(values, meta, K)
    torch.cuda.synchronize()
    v, m, k, p = orc.prune24(x, fmt)
    log(f"prune fmt={fmt} rows={rows} K={K} kind={kind}")
    assert np.array_equal(values.cpu().numpy(), v)
    assert np.array_equal(meta.cpu().numpy(), m)
    assert np.array_equal(mask.cpu().numpy(), k)
    assert np.array_equal(pruned.cpu().numpy(), p)


def test_prune_full_size_bit_exact(gpu):
    """A 16384 x 16384 E4M3 matrix (the largest A of the square sweep): prune on the
    GPU, compare sampled rows with the oracle and check the invariants on all."""
    import torch
    rows = K = 16384
    x = torch.randint(0, 256, (rows, K), dtype=torch.uint8, device="cuda")
    x[(x & 0x7F) == 0x7F] = 0     # no NaN codes
    values, meta, mask = gpu.fp8_sparse24_prune_compress(x, 0)
    torch.cuda.synchronize()
    # every group keeps exactly two
    bits = torch.stack([(mask >> b) & 1 for b in range(8)], dim=-1).reshape(rows, K // 4, 4)
    assert bool(torch.all(bits.sum(-1) == 2))
    sel = [0, 1, 4095, 8191, 12345, rows - 1]
    xh = x[sel].cpu().numpy()
    v, m, k, _ = orc.prune24(xh, 0)
    assert np.array_equal(values[sel].cpu().numpy(), v)
    assert np.array_equal(meta[sel].cpu().numpy(), m)
    assert np.array_equal(mask[sel].cpu().numpy(), k)


@pytest.mark.parametrize("fmt", [0, 1])
@pytest.mark.parametrize("per_row", [False, True])
@pytest.mark.parametrize("shape,dist", [((256, 256), "uniform"), ((37, 56), "normal"), ((1, 8), "normal"),
                                        ((300, 1000), "normal"), ((5, 4096), "uniform"), ((3, 8200), "normal"),
                                        ((2, 12288), "normal"), ((2, 16384), "uniform"), ((2, 16392), "normal")])
def test_quantize_prune_fused_bit_exact(gpu, fmt, per_row, shape, dist):
    """The one-pass encode equals the oracle's quantize followed by its 2:4
    prune: codes of the survivors, metadata, mask and scales bit for bit
    (K % 16 == 8 rows end in a half unit; K > 16384 takes the two-read form)."""
    import torch
    rows, K = shape
    x = synth.uniform(5, 9, shape) if dist == "uniform" else synth.normal_outliers(6, shape)
    ld = (K + 3) // 4 * 4
    xd = torch.zeros((rows, ld), dtype=torch.float32, device="cuda")
    xd[:, :K] = dev(x)
    kind = gpu.FP8_SCALE_ROW if per_row else gpu.FP8_SCALE_TENSOR
    values, meta, mask, s, d = gpu.fp8_quantize_prune24(xd[:, :K], fmt, kind)
    torch.cuda.synchronize()
    qo, so, do = orc.quantize(x, fmt, per_row)
    v, m, k, _ = orc.prune24(qo, fmt)
    log(f"quantize+prune fmt={fmt} per_row={per_row} shape={shape}")
    assert np.array_equal(values.cpu().numpy(), v)
    assert np.array_equal(meta.cpu().numpy(), m)
    assert np.array_equal(mask.cpu().numpy(), k)
    assert np.array_equal(s.cpu().numpy().view(np.uint32), so.view(np.uint32))
    assert np.array_equal(d.cpu().numpy().view(np.uint32), do.view(np.uint32))


@pytest.mark.parametrize("per_row", [False, True])
def test_quantize_prune_fused_full_size(gpu, per_row):
    """8192 x 8192 (the headline operand): the fused pass equals quantize then
    prune on the GPU bit for bit, and sampled rows equal the oracle's."""
    import torch
    rows = K = 8192
    g = torch.Generator(device="cuda").manual_seed(11)
    x = torch.randn((rows, K), dtype=torch.float32, device="cuda", generator=g)
    kind = gpu.FP8_SCALE_ROW if per_row else gpu.FP8_SCALE_TENSOR
    values, meta, mask, s, d = gpu.fp8_quantize_prune24(x, 0, kind)
    q, s2, d2 = gpu.fp8_quantize(x, 0, kind)
    v2, m2, k2 = gpu.fp8_sparse24_prune_compress(q, 0)
    torch.cuda.synchronize()
    assert torch.equal(values, v2) and torch.equal(meta, m2) and torch.equal(mask, k2)
    assert torch.equal(s.view(torch.int32), s2.view(torch.int32))
    assert torch.equal(d.view(torch.int32), d2.view(torch.int32))
    sel = [0, 1, 4095, rows - 1]
    xh = x[sel].cpu().numpy()
    if per_row:
        qo, so, _ = orc.quantize(xh, 0, True)
        assert np.array_equal(s[sel].cpu().numpy().view(np.uint32), so.view(np.uint32))
    else:
        # the per-tensor scale of the whole matrix applied to the sampled rows
        qo = orc.encode(0, (xh * s.cpu().numpy()[0]).astype(np.float32).ravel()).reshape(xh.shape)
    vo, mo, ko, _ = orc.prune24(qo, 0)
    assert np.array_equal(values[sel].cpu().numpy(), vo)
    assert np.array_equal(meta[sel].cpu().numpy(), mo)
    assert np.array_equal(mask[sel].cpu().numpy(), ko)
