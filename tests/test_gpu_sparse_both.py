"""GPU parity of the both-sides 2:4 GEMM (activations and weight both pruned
and compressed) against the FP64 oracle on the two pruned matrices, strict
elementwise bound."""
import numpy as np
import pytest

import oracle as orc
from tests.helpers import check_gemm, check_gemm_sampled, dev, log, operands

pytestmark = pytest.mark.gpu

BOTH_TILES = (0, 3, 11, 12, 25, 26, 27)


def _both(gpu, M, N, K, seed, fa, bf16, plan=None):
    import torch
    qa, da, qb, db = operands(M, N, K, seed, "normal", fa, 0, True)
    va, ma, _, pa = orc.prune24(qa, fa)
    vw, mw, _, pw = orc.prune24(qb, 0)
    c = gpu.fp8_sparse24_both_gemm(dev(va), dev(ma), dev(vw), dev(mw), dev(da), dev(db), fa, 0,
                                   torch.bfloat16 if bf16 else torch.float32, plan=plan)
    torch.cuda.synchronize()
    return c, pa, pw, da, db


@pytest.mark.parametrize("M,N,K", [(64, 64, 128), (77, 45, 200), (130, 260, 384), (16, 512, 1024), (257, 33, 1032),
                                   (300, 130, 4096), (40, 300, 3600), (16, 1024, 4096), (1, 256, 512)])
@pytest.mark.parametrize("fa", [0, 1])
@pytest.mark.parametrize("bf16", [False, True])
def test_both_sides_default_plan(gpu, M, N, K, fa, bf16):
    """Default plan (exact-sum tiles below K = 3584, the FP8 SMFMAC with the
    weight expanded in-kernel above; the weight takes the compressed slot when
    A has fewer than 64 rows)."""
    log(f"both sides M={M} N={N} K={K} fa={fa} bf16={bf16}")
    c, pa, pw, da, db = _both(gpu, M, N, K, 41 + K % 7, fa, bf16)
    check_gemm(c, pa, fa, pw, 0, da, db, bf16, f"both {M}x{N}x{K}")


@pytest.mark.parametrize("tile", BOTH_TILES)
@pytest.mark.parametrize("split", [1, 3])
def test_both_sides_every_tile(gpu, tile, split):
    M, N, K = 150, 200, 4096
    log(f"both sides tile={tile} split={split}")
    c, pa, pw, da, db = _both(gpu, M, N, K, 43, 0, False, plan=(tile, split))
    check_gemm(c, pa, 0, pw, 0, da, db, False, f"both tile {tile} split {split}")


def test_both_sides_ragged_k_on_fp8_tile(gpu):
    """K % 128 != 0 on an FP8 tile: the byte-exact loader of both operands."""
    M, N, K = 96, 80, 3720
    c, pa, pw, da, db = _both(gpu, M, N, K, 44, 0, False, plan=(0, 1))
    check_gemm(c, pa, 0, pw, 0, da, db, False, "both ragged K")


def test_both_sides_rejects_tiles_without_kernel(gpu):
    import torch
    n = gpu.fp8_num_tiles()
    qa, da, qb, db = operands(64, 64, 256, 45, "normal", 0, 0, True)
    va, ma, _, _ = orc.prune24(qa, 0)
    vw, mw, _, _ = orc.prune24(qb, 0)
    for tile in range(n):
        if tile in BOTH_TILES:
            continue
        with pytest.raises(gpu.Fp8Error):
            gpu.fp8_sparse24_both_gemm(dev(va), dev(ma), dev(vw), dev(mw), dev(da), dev(db), plan=(tile, 1))
    torch.cuda.synchronize()


def test_both_sides_full_size_sampled(gpu):
    """8192^3 with both operands pruned by the fused quantize+prune pass,
    default plan, BF16 out: sampled outputs against the oracle on the oracle's
    own quantization and pruning of the same FP32 data."""
    import torch
    from paper_2602_10262_amd import synth
    M = N = K = 8192
    xa = synth.normal_outliers(51, (M, K))
    xb = synth.normal_outliers(52, (N, K))
    va_d, ma_d, _, _, da_d = gpu.fp8_quantize_prune24(dev(xa), 0, gpu.FP8_SCALE_ROW, with_mask=False)
    vw_d, mw_d, _, _, db_d = gpu.fp8_quantize_prune24(dev(xb), 0, gpu.FP8_SCALE_ROW, with_mask=False)
    log("both sides 8192^3")
    c = gpu.fp8_sparse24_both_gemm(va_d, ma_d, vw_d, mw_d, da_d, db_d, out_dtype=torch.bfloat16)
    torch.cuda.synchronize()
    qa, _, da = orc.quantize(xa, 0, True)
    qb, _, db = orc.quantize(xb, 0, True)
    va, ma, _, pa = orc.prune24(qa, 0)
    vw, mw, _, pw = orc.prune24(qb, 0)
    assert np.array_equal(va_d.cpu().numpy(), va) and np.array_equal(mw_d.cpu().numpy(), mw)
    check_gemm_sampled(c, pa, 0, pw, 0, da, db, True, what="both sides 8192^3")
