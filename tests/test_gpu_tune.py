"""The autotuner on the GPU: the plan it keeps is one the library can run,
belongs to the accumulation class K asks for (exact sums below K = 3584),
answers later plan lookups, and computes a result inside the oracle bound;
the dense-vs-2:4 record names plans of the right kind and consistent times."""
import numpy as np
import pytest

import oracle as orc
from tests.helpers import check_gemm, codes_with_pad, dev, log, operands

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("M,N,K", [(256, 512, 4096), (96, 384, 1024)])
def test_tuned_plan_is_valid_cached_and_correct(gpu, M, N, K):
    import torch
    qa, da, qb, db = operands(M, N, K, 41, "normal", 0, 0, True)
    a, b = codes_with_pad(M, K, qa), codes_with_pad(N, K, qb)
    c = torch.empty((M, N), dtype=torch.float32, device="cuda")
    args = gpu.gemm_args(a, b, dev(da), dev(db), c)
    gpu.fp8_tune_cache_clear()
    try:
        (tile, split), us = gpu.fp8_tune_gemm(args, iters=2)
        log(f"tuned {M}x{N}x{K}: tile {tile} split {split} {us:.1f} us")
        info = gpu.fp8_tile_info(tile)
        assert info["dense"] and split >= 1 and us > 0
        assert bool(info["exact"]) == (K < 3584)
        # the cache answers the default-plan lookup from now on
        assert gpu.fp8_gemm_plan_resolve(args) == (tile, split)
        c2 = gpu.fp8_gemm(a, b, dev(da), dev(db), out_dtype=torch.float32)
        torch.cuda.synchronize()
        check_gemm(c2, qa, 0, qb, 0, da, db, False, f"tuned plan {M}x{N}x{K}")
    finally:
        gpu.fp8_tune_cache_clear()


def test_sparse_vs_dense_record(gpu):
    import torch
    M, N, K = 512, 512, 4096
    qa, da, qb, db = operands(M, N, K, 43, "normal", 0, 0, True)
    va, ma, _, pa = orc.prune24(qa, 0)
    b = codes_with_pad(N, K, qb)
    c = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")
    dargs = gpu.gemm_args(codes_with_pad(M, K, pa), b, dev(da), dev(db), c)
    sargs = gpu.sparse24_args(dev(va), dev(ma), b, gpu.FP8_SPARSE_A, dev(da), dev(db), c)
    gpu.fp8_tune_cache_clear()
    try:
        rec = gpu.fp8_tune_sparse_vs_dense(sargs, dargs, iters=2)
        log(f"break-even record: {rec}")
        assert (rec["M"], rec["N"], rec["K"], rec["side"]) == (M, N, K, "A")
        assert gpu.fp8_tile_info(rec["dense_plan"][0])["dense"]
        assert gpu.fp8_tile_info(rec["sparse_plan"][0])["sparse"]
        assert rec["dense_us"] > 0 and rec["sparse_us"] > 0
        assert rec["use_sparse"] == (rec["sparse_us"] < rec["dense_us"])
        assert any((r["M"], r["N"], r["K"]) == (M, N, K) for r in gpu.fp8_tune_breakeven_records())
        # the 2:4 product on the tuned sparse plan is still inside the bound
        cs = gpu.fp8_sparse24_gemm(dev(va), dev(ma), b, gpu.FP8_SPARSE_A, dev(da), dev(db),
                                   out_dtype=torch.float32, plan=tuple(rec["sparse_plan"]))
        torch.cuda.synchronize()
        check_gemm(cs, pa, 0, qb, 0, da, db, False, "tuned 2:4 plan")
    finally:
        gpu.fp8_tune_cache_clear()
