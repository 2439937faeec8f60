"""The allocation-free GEMM entry point: through the C ABI, its results equal
fp8_gemm's with the same plan (bit for bit, and within the oracle bound on
sampled outputs), on two calls in a row with the second input smaller, and
plans whose split-K partial sums exceed the fixed scratch are refused."""
import numpy as np
import pytest

import oracle as orc
from paper_2602_10262_amd import synth
from tests.helpers import check_gemm_sampled, dev, log

pytestmark = pytest.mark.gpu


def _operands(M, N, K, seed):
    xa = synth.normal_outliers(seed, (M, K))
    xb = synth.normal_outliers(seed + 1, (N, K))
    qa, _, da = orc.quantize(xa, orc.E4M3, True)
    qb, _, db = orc.quantize(xb, orc.E4M3, True)
    return qa, da, qb, db


@pytest.mark.parametrize("plan", [(4, 4), (7, 3), None])
def test_noalloc_matches_fp8_gemm_twice_second_smaller(gpu, plan):
    import torch
    for M, N, K, seed in [(64, 4096, 8192, 41), (16, 2048, 4096, 43)]:
        qa, da, qb, db = _operands(M, N, K, seed)
        a, b, sa, sb = dev(qa), dev(qb), dev(da), dev(db)
        ref = gpu.fp8_gemm(a, b, sa, sb, out_dtype=torch.bfloat16, plan=plan)
        c = torch.full((M, N), float("nan"), dtype=torch.bfloat16, device="cuda")
        torch.cuda.synchronize()
        gpu.fp8_gemm_noalloc(a, b, sa, sb, c=c, plan=plan)
        torch.cuda.synchronize()
        log(f"noalloc M={M} N={N} K={K} plan={plan} resolved={gpu.fp8_gemm_plan_resolve(gpu.gemm_args(a, b, sa, sb, c), plan)}")
        assert torch.equal(c.view(torch.int16), ref.view(torch.int16)), (M, N, K, plan)
        check_gemm_sampled(c, qa, orc.E4M3, qb, orc.E4M3, da, db, True, n=1024, what=f"noalloc {M}x{N}x{K}")


def test_noalloc_refuses_partial_sums_beyond_scratch(gpu):
    import torch
    M = N = 2048
    K = 4096
    a = torch.zeros((M, K), dtype=torch.uint8, device="cuda")
    b = torch.zeros((N, K), dtype=torch.uint8, device="cuda")
    one = torch.ones(1, dtype=torch.float32, device="cuda")
    c = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")
    # 8 splits x 2048 x 2048 x 4 bytes = 128 MiB > the fixed scratch
    assert 8 * M * N * 4 > gpu.fp8_noalloc_scratch_bytes()
    with pytest.raises(gpu.Fp8Error) as e:
        gpu.fp8_gemm_noalloc(a, b, one, one, c=c, plan=(0, 8))
    assert e.value.status == 4
