"""GPU parity of the dense and 2:4 FP8 GEMMs against the FP64 oracle:
|C - C_ref| <= 4 K 2^-24 S_abs elementwise for FP32 output, plus one BF16
rounding step for BF16 output."""
import numpy as np
import pytest

import oracle as orc
from tests.helpers import check_gemm, check_gemm_sampled, codes_with_pad, dev, host, log, operands

pytestmark = pytest.mark.gpu


def _run_dense(gpu, qa, qb, da, db, fa, fb, bf16, plan=None):
    import torch
    M, K = qa.shape
    N = qb.shape[0]
    a = codes_with_pad(M, K, qa)
    b = codes_with_pad(N, K, qb)
    c = gpu.fp8_gemm(a, b, dev(da), dev(db), fa, fb, torch.bfloat16 if bf16 else torch.float32, plan=plan)
    torch.cuda.synchronize()
    return c


def test_256_cube_uniform_per_tensor_fp32(gpu):
    """M = N = K = 256, uniform[-1, 1) inputs, per-tensor 448/amax scales,
    E4M3 x E4M3, FP32 output."""
    qa, da, qb, db = operands(256, 256, 256, 0, "uniform", 0, 0, False)
    log("256^3 E4M3 uniform inputs, per-tensor scales, FP32 out")
    c = _run_dense(gpu, qa, qb, da, db, 0, 0, False)
    check_gemm(c, qa, 0, qb, 0, da, db, False, "256^3")


@pytest.mark.parametrize("M,N,K", [(1, 1, 16), (77, 45, 200), (130, 260, 384), (300, 17, 1000), (16, 640, 1024),
                                   (513, 129, 136), (64, 64, 4096), (96, 80, 128), (200, 100, 512), (40, 300, 3600)])
@pytest.mark.parametrize("fa", [0, 1])
@pytest.mark.parametrize("bf16", [False, True])
def test_dense_ragged_shapes(gpu, M, N, K, fa, bf16):
    """N(0,1) + 1% 20-sigma outliers at every K, default plan, strict bound."""
    qa, da, qb, db = operands(M, N, K, 1, "normal", fa, 0, True)
    log(f"dense M={M} N={N} K={K} fa={fa} bf16={bf16}")
    c = _run_dense(gpu, qa, qb, da, db, fa, 0, bf16)
    check_gemm(c, qa, fa, qb, 0, da, db, bf16, f"{M}x{N}x{K}")


NUM_TILES = 32   # tile configurations the library exports (fp8_num_tiles)
# FP8 decoded to BF16 and summed on the BF16 MFMA: 25-27 through registers
# (any K), 28-30 on the LDS-DMA ring (K % 16 == 0, or % 128 with a 2:4
# operand; any other K runs on tile 27); dense and 2:4 alike
EXACT_TILES = (25, 26, 27, 28, 29, 30)


def test_tile_table_size(gpu):
    assert gpu.load().fp8_num_tiles() == NUM_TILES


@pytest.mark.parametrize("tile", list(range(NUM_TILES)))
@pytest.mark.parametrize("split", [1, 3])
def test_every_tile_and_split(gpu, tile, split):
    M, N, K = 200, 300, 640
    qa, da, qb, db = operands(M, N, K, 2, "normal", 0, 0, True)
    log(f"tile={tile} split={split}")
    if not gpu.fp8_tile_info(tile)["dense"]:
        # 2:4-only tile: a dense plan is rejected before any launch
        with pytest.raises(gpu.Fp8Error):
            _run_dense(gpu, qa, qb, da, db, 0, 0, False, plan=(tile, split))
        return
    c = _run_dense(gpu, qa, qb, da, db, 0, 0, False, plan=(tile, split))
    check_gemm(c, qa, 0, qb, 0, da, db, False, f"tile {tile} split {split}")


@pytest.mark.parametrize("tile", list(range(NUM_TILES)))
@pytest.mark.parametrize("split", [1, 2])
def test_every_tile_partial_last_k_step(gpu, tile, split):
    """K a multiple of 16 but not of 128: the last K step of the last split is
    partial, so its chunks past K must read as zero (the DMA tiles fetch them
    from past the buffer range; the register tiles select zero)."""
    M, N, K = 70, 90, 656
    qa, da, qb, db = operands(M, N, K, 21, "normal", 0, 0, True)
    log(f"tile={tile} split={split} K={K}")
    if not gpu.fp8_tile_info(tile)["dense"]:
        return   # 2:4-only tile (its dense rejection is tested above)
    c = _run_dense(gpu, qa, qb, da, db, 0, 0, False, plan=(tile, split))
    check_gemm(c, qa, 0, qb, 0, da, db, False, f"tile {tile} split {split} K {K}")


def test_both_e5m2_operands(gpu):
    qa, da, qb, db = operands(96, 80, 512, 3, "normal", 1, 1, True)
    c = _run_dense(gpu, qa, qb, da, db, 1, 1, True)
    check_gemm(c, qa, 1, qb, 1, da, db, True, "E5M2 x E5M2")


def test_all_ones_exact(gpu):
    import torch
    for K in (128, 1000, 8192):
        qa = np.full((64, K), 0x38, np.uint8)
        qb = np.full((48, K), 0x38, np.uint8)
        one = np.ones(1, np.float32)
        c = _run_dense(gpu, qa, qb, one, one, 0, 0, False)
        assert torch.all(c == float(K)), K


def test_identity_exact(gpu):
    K = 256
    rng = np.random.default_rng(0)
    qa = rng.integers(0, 256, (40, K)).astype(np.uint8)
    qa[(qa & 0x7F) == 0x7F] = 0
    eye = np.where(np.eye(K, dtype=bool), 0x38, 0).astype(np.uint8)
    one = np.ones(1, np.float32)
    c = _run_dense(gpu, qa, eye, one, one, 0, 0, False)
    assert np.array_equal(host(c), orc.decode(0, qa).astype(np.float32))


def test_deterministic_reruns(gpu):
    import torch
    qa, da, qb, db = operands(300, 200, 2048, 5, "normal", 0, 0, True)
    c1 = _run_dense(gpu, qa, qb, da, db, 0, 0, False, plan=(0, 4))
    c2 = _run_dense(gpu, qa, qb, da, db, 0, 0, False, plan=(0, 4))
    assert torch.equal(c1, c2)


# ---------------------------------------------------------------- 2:4 ----

def _sparse_case(M, N, K, seed, fa=0):
    return operands(M, N, K, seed, "normal", fa, 0, True)


@pytest.mark.parametrize("M,N,K", [(64, 64, 128), (77, 45, 200), (130, 260, 384), (16, 512, 1024), (257, 33, 1032)])
@pytest.mark.parametrize("bf16", [False, True])
def test_sparse_A(gpu, M, N, K, bf16):
    import torch
    qa, da, qb, db = _sparse_case(M, N, K, 11)
    va, ma, _, pa = orc.prune24(qa, 0)
    log(f"sparse A M={M} N={N} K={K} bf16={bf16}")
    values = dev(va)
    meta = dev(ma)
    b = codes_with_pad(N, K, qb)
    c = gpu.fp8_sparse24_gemm(values, meta, b, gpu.FP8_SPARSE_A, dev(da), dev(db), 0, 0,
                              torch.bfloat16 if bf16 else torch.float32)
    torch.cuda.synchronize()
    check_gemm(c, pa, 0, qb, 0, da, db, bf16, "sparse A")
    # dense on the identical pruned matrix
    cd = _run_dense(gpu, pa, qb, da, db, 0, 0, bf16)
    check_gemm(cd, pa, 0, qb, 0, da, db, bf16, "dense on pruned A")


@pytest.mark.parametrize("M,N,K", [(64, 64, 128), (1, 256, 512), (45, 77, 200), (300, 130, 1024), (16, 4096, 1024)])
@pytest.mark.parametrize("bf16", [False, True])
def test_sparse_B_weight(gpu, M, N, K, bf16):
    import torch
    qa, da, qb, db = _sparse_case(M, N, K, 12)
    vw, mw, _, pw = orc.prune24(qb, 0)       # weight: N x K rows
    log(f"sparse B M={M} N={N} K={K} bf16={bf16}")
    a = codes_with_pad(M, K, qa)
    c = gpu.fp8_sparse24_gemm(dev(vw), dev(mw), a, gpu.FP8_SPARSE_B, dev(da), dev(db), 0, 0,
                              torch.bfloat16 if bf16 else torch.float32)
    torch.cuda.synchronize()
    check_gemm(c, qa, 0, pw, 0, da, db, bf16, "sparse B")


@pytest.mark.parametrize("tile", list(range(NUM_TILES)))
def test_sparse_every_tile(gpu, tile):
    import torch
    M, N, K = 150, 200, 512
    qa, da, qb, db = _sparse_case(M, N, K, 13)
    va, ma, _, pa = orc.prune24(qa, 0)
    if not gpu.fp8_tile_info(tile)["sparse"]:
        # dense-only tile: the plan is rejected before any launch
        with pytest.raises(gpu.Fp8Error):
            gpu.fp8_sparse24_gemm(dev(va), dev(ma), codes_with_pad(N, K, qb), gpu.FP8_SPARSE_A, dev(da), dev(db),
                                  plan=(tile, 2))
        return
    c = gpu.fp8_sparse24_gemm(dev(va), dev(ma), codes_with_pad(N, K, qb), gpu.FP8_SPARSE_A, dev(da), dev(db),
                              plan=(tile, 2))
    torch.cuda.synchronize()
    check_gemm(c, pa, 0, qb, 0, da, db, False, f"sparse tile {tile}")


def test_sparse_e5m2_activation(gpu):
    import torch
    M, N, K = 64, 96, 256
    qa, da, qb, db = _sparse_case(M, N, K, 14, fa=1)
    va, ma, _, pa = orc.prune24(qa, 1)
    c = gpu.fp8_sparse24_gemm(dev(va), dev(ma), codes_with_pad(N, K, qb), gpu.FP8_SPARSE_A, dev(da), dev(db), 1, 0)
    torch.cuda.synchronize()
    check_gemm(c, pa, 1, qb, 0, da, db, False, "sparse E5M2 A")


# ---------------------------------------------------- full-size samples ----

@pytest.mark.parametrize("M,N,K,fa", [(8192, 8192, 8192, 0), (8192, 8192, 8192, 1), (16, 8192, 8192, 0),
                                      (256, 8192, 8192, 1), (16384, 16384, 16384, 0), (16384, 16384, 16384, 1)])
def test_full_size_sampled(gpu, M, N, K, fa):
    """The benchmark's shapes with the benchmark's default plan: sampled
    outputs against the oracle, N(0,1) + 1% 20-sigma outliers, per-row and
    per-column scales, BF16 output."""
    import torch
    from paper_2602_10262_amd import synth
    xa = synth.normal_outliers(21, (M, K))
    xb = synth.normal_outliers(22, (N, K))
    qa_d, _, da_d = gpu.fp8_quantize(dev(xa), fa, gpu.FP8_SCALE_ROW)
    qb_d, _, db_d = gpu.fp8_quantize(dev(xb), 0, gpu.FP8_SCALE_ROW)
    log(f"full size {M}x{N}x{K} fa={fa}")
    c = gpu.fp8_gemm(qa_d, qb_d, da_d, db_d, fa, 0, torch.bfloat16)
    torch.cuda.synchronize()
    # the oracle's inputs are its own quantization of the same FP32 data
    qa, _, da = orc.quantize(xa, fa, True)
    qb, _, db = orc.quantize(xb, 0, True)
    assert np.array_equal(qa_d.cpu().numpy(), qa) and np.array_equal(qb_d.cpu().numpy(), qb)
    check_gemm_sampled(c, qa, fa, qb, 0, da, db, True, what=f"{M}x{N}x{K}")


@pytest.mark.parametrize("S", [8192, 16384])
def test_full_size_sparse_sampled(gpu, S):
    """2:4 (A pruned) at the sweep's large squares on the default plan."""
    import torch
    from paper_2602_10262_amd import synth
    M = N = K = S
    log(f"full size sparse {S}^3")
    xa = synth.normal_outliers(31, (M, K))
    xb = synth.normal_outliers(32, (N, K))
    qa_d, _, da_d = gpu.fp8_quantize(dev(xa), 0, gpu.FP8_SCALE_ROW)
    qb_d, _, db_d = gpu.fp8_quantize(dev(xb), 0, gpu.FP8_SCALE_ROW)
    values, meta, _ = gpu.fp8_sparse24_prune_compress(qa_d, 0, with_mask=False)
    c = gpu.fp8_sparse24_gemm(values, meta, qb_d, gpu.FP8_SPARSE_A, da_d, db_d, out_dtype=torch.bfloat16)
    torch.cuda.synchronize()
    qa, _, da = orc.quantize(xa, 0, True)
    qb, _, db = orc.quantize(xb, 0, True)
    _, _, _, pa = orc.prune24(qa, 0)
    check_gemm_sampled(c, pa, 0, qb, 0, da, db, True, what=f"sparse {S}^3")


# ------------------------------------------- MFMA in-instruction precision ---

def _run_a_sparse_or_dense(gpu, qa, da, qb, db, sparse, plan):
    if sparse:
        va, ma, _, pa = orc.prune24(qa, 0)
        c = gpu.fp8_sparse24_gemm(dev(va), dev(ma), codes_with_pad(qb.shape[0], qb.shape[1], qb), gpu.FP8_SPARSE_A,
                                  dev(da), dev(db), plan=plan)
        return c, pa
    c = gpu.fp8_gemm(codes_with_pad(qa.shape[0], qa.shape[1], qa), codes_with_pad(qb.shape[0], qb.shape[1], qb),
                     dev(da), dev(db), plan=plan)
    return c, qa


SMALL_K = [(77, 45, 200), (513, 129, 136), (64, 64, 128), (130, 260, 384), (200, 100, 512)]


@pytest.mark.parametrize("M,N,K", SMALL_K)
@pytest.mark.parametrize("sparse", [False, True])
def test_small_k_outliers_strict_bound_default_plan(gpu, M, N, K, sparse):
    """Small K, N(0,1) + 1% 20-sigma outliers, the library's own plan (the
    exact-sum tiles below K = 3584): the strict elementwise bound."""
    import torch
    qa, da, qb, db = operands(M, N, K, 17, "normal", 0, 0, True)
    c, qa_eff = _run_a_sparse_or_dense(gpu, qa, da, qb, db, sparse, None)
    torch.cuda.synchronize()
    check_gemm(c, qa_eff, 0, qb, 0, da, db, False, f"default plan {M}x{N}x{K} sparse={sparse}")


@pytest.mark.parametrize("tile", EXACT_TILES)
@pytest.mark.parametrize("M,N,K", [(513, 129, 136), (77, 45, 200), (33, 70, 8200)])
def test_exact_tiles_strict_bound_any_k(gpu, tile, M, N, K):
    """The exact-sum tiles meet the strict bound at any K, split or not."""
    import torch
    qa, da, qb, db = operands(M, N, K, 19, "normal", 1, 0, True)
    for split in (1, 3):
        c = _run_dense(gpu, qa, qb, da, db, 1, 0, False, plan=(tile, split))
        check_gemm(c, qa, 1, qb, 0, da, db, False, f"exact tile {tile} split {split} {M}x{N}x{K}")


@pytest.mark.parametrize("tile", EXACT_TILES)
@pytest.mark.parametrize("M,N,K", [(150, 77, 2064), (97, 130, 1280), (260, 33, 136)])
@pytest.mark.parametrize("sparse", [False, True])
def test_exact_tiles_fast_and_byte_loaders(gpu, tile, M, N, K, sparse):
    """Both loaders of the exact-sum tiles: buffer loads when K is a multiple
    of 16 (dense) or 128 (compressed), the byte-exact loader otherwise; ragged
    M and N, padded rows, split or not, against the strict bound."""
    import torch
    qa, da, qb, db = operands(M, N, K, 23, "normal", 0, 0, True)
    if sparse and not gpu.fp8_tile_info(tile)["sparse"]:
        # dense-only exact tile: a 2:4 plan is rejected before any launch
        with pytest.raises(gpu.Fp8Error):
            _run_a_sparse_or_dense(gpu, qa, da, qb, db, True, (tile, 1))
        return
    for split in (1, 3):
        log(f"exact loaders tile={tile} {M}x{N}x{K} sparse={sparse} split={split}")
        c, qa_eff = _run_a_sparse_or_dense(gpu, qa, da, qb, db, sparse, (tile, split))
        torch.cuda.synchronize()
        check_gemm(c, qa_eff, 0, qb, 0, da, db, False, f"exact tile {tile} {M}x{N}x{K} sparse={sparse} split={split}")


@pytest.mark.parametrize("M,N,K", [(2048, 2048, 2048), (4096, 1536, 1024), (1024, 1024, 1024), (8192, 8192, 2048)])
@pytest.mark.parametrize("sparse", [False, True])
def test_exact_default_plan_sampled(gpu, M, N, K, sparse):
    """The library's own plan below K = 3584 at sweep sizes (many tiles of
    the exact-sum kernels), dense and 2:4 on A: sampled outputs against the
    strict bound."""
    import torch
    qa, da, qb, db = operands(M, N, K, 29, "normal", 0, 0, True)
    log(f"exact default plan {M}x{N}x{K} sparse={sparse}")
    if sparse:
        va, ma, _, pa = orc.prune24(qa, 0)
        c = gpu.fp8_sparse24_gemm(dev(va), dev(ma), codes_with_pad(N, K, qb), gpu.FP8_SPARSE_A, dev(da), dev(db),
                                  out_dtype=torch.bfloat16)
        qa = pa
    else:
        c = _run_dense(gpu, qa, qb, da, db, 0, 0, True)
    torch.cuda.synchronize()
    check_gemm_sampled(c, qa, 0, qb, 0, da, db, True, what=f"exact default plan {M}x{N}x{K} sparse={sparse}")


@pytest.mark.parametrize("tile", [28, 29, 30])
def test_exact_dma_tiles_weight_side(gpu, tile):
    """2:4 weight (B side) on the exact-sum DMA tiles, split or not."""
    import torch
    M, N, K = 130, 300, 1280
    qa, da, qb, db = _sparse_case(M, N, K, 31)
    vw, mw, _, pw = orc.prune24(qb, 0)
    for split in (1, 3):
        log(f"exact dma weight side tile={tile} split={split}")
        c = gpu.fp8_sparse24_gemm(dev(vw), dev(mw), codes_with_pad(M, K, qa), gpu.FP8_SPARSE_B, dev(da), dev(db),
                                  plan=(tile, split))
        torch.cuda.synchronize()
        check_gemm(c, qa, 0, pw, 0, da, db, False, f"exact dma weight side tile {tile} split {split}")


def _fp8_mfma_envelope(qa, da, qb, db, K):
    """The FP8 MFMA's measured error model: within each run of eight
    consecutive k (starting at multiples of 8) the products are aligned to the
    largest exponent sum of the run and about fourteen bits below it are kept,
    so each run loses less than 7 * 2^-13 of its largest product; 2^-12 per
    run leaves a factor of 8 / 7 of margin."""
    va, vb = orc.decode(0, qa), orc.decode(0, qb)
    pad = (-K) % 8
    pa = np.pad(va, ((0, 0), (0, pad)))
    pb = np.pad(vb, ((0, 0), (0, pad)))
    ga = pa.reshape(pa.shape[0], -1, 8)
    gb = pb.reshape(pb.shape[0], -1, 8)
    # max over each run of |a_ik b_jk|, summed over runs
    runmax = np.max(np.abs(ga[:, None, :, :] * gb[None, :, :, :]), axis=3).sum(axis=2)
    return 2.0 ** -12 * runmax * np.abs(da[:, None] * db[None, :])


@pytest.mark.parametrize("M,N,K", SMALL_K)
@pytest.mark.parametrize("sparse", [False, True])
def test_fp8_mfma_tile_error_model_small_k(gpu, M, N, K, sparse):
    """An FP8-MFMA tile forced at small K on outlier data: its error stays
    inside 4 K 2^-24 S_abs plus the measured in-instruction truncation term,
    which is what keeps such K on the exact-sum tiles by default (the plain
    bound is reported, not asserted, for these forced plans)."""
    import torch
    qa, da, qb, db = operands(M, N, K, 17, "normal", 0, 0, True)
    c, qa_eff = _run_a_sparse_or_dense(gpu, qa, da, qb, db, sparse, (0, 1))
    torch.cuda.synchronize()
    cref, sabs = orc.gemm(qa_eff, 0, qb, 0, da, db)
    err = np.abs(host(c).astype(np.float64) - cref)
    fp32_bound = orc.bound(sabs, cref, K, orc.OUT_F32)
    envelope = fp32_bound + _fp8_mfma_envelope(qa_eff, da, qb, db, K)
    log(f"FP8 tile 0 M={M} N={N} K={K} sparse={sparse}: max err/bound={np.max(err / fp32_bound):.3f} "
        f"max err/envelope={np.max(err / envelope):.3f}")
    assert np.all(err <= envelope)


# ------------------------------------------------------ device validator ---

@pytest.mark.parametrize("bf16", [False, True])
def test_device_validator_agrees_with_oracle_check(gpu, bf16):
    """fp8_validate (FP64 reduction on the GPU) reports the same maximum error,
    maximum ratio to the bound, normwise error and count over the bound as the
    oracle's CPU check of the same result; a planted error is counted by both."""
    import torch
    M, N, K = 300, 200, 1000
    qa, da, qb, db = operands(M, N, K, 23, "normal", 0, 0, True)
    c = _run_dense(gpu, qa, qb, da, db, 0, 0, bf16)
    cref, sabs = orc.gemm(qa, 0, qb, 0, da, db)
    out_t = orc.OUT_BF16 if bf16 else orc.OUT_F32
    for planted in (False, True):
        if planted:
            # push a few outputs far outside their bound
            c.view(-1)[torch.tensor([0, 777, M * N - 1], device="cuda")] += 1.0
            torch.cuda.synchronize()
        ref = orc.check(host(c), cref, sabs, K, out_t)
        got = gpu.fp8_validate(c, dev(cref), dev(sabs), K)
        torch.cuda.synchronize()
        b = orc.bound(sabs, cref, K, out_t)
        over = int(np.sum(np.abs(host(c).astype(np.float64) - cref) > b))
        log(f"validator bf16={bf16} planted={planted}: gpu {got} cpu {ref} over {over}")
        assert got["over"] == over
        assert got["ok"] == ref["ok"] == (not planted)
        assert np.isclose(got["max_abs_err"], ref["max_abs_err"], rtol=1e-12, atol=0)
        assert np.isclose(got["max_ratio"], ref["max_ratio"], rtol=1e-12, atol=0)
        assert np.isclose(got["normwise"], ref["normwise"], rtol=1e-9, atol=0)
