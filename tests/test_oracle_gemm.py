"""Pins for the oracle's FP64 GEMM (dense and 2:4) and for the acceptance
bound used against the GPU results."""
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle as orc
from paper_2602_10262_amd import synth

TORCH_DT = {orc.E4M3: torch.float8_e4m3fn, orc.E5M2: torch.float8_e5m2}


def _lib_decode(fmt, codes):
    """Decode through torch's float8 dtypes (independent of the oracle)."""
    t = torch.from_numpy(np.ascontiguousarray(codes, dtype=np.uint8))
    return t.view(TORCH_DT[fmt]).to(torch.float64).numpy()


def _finite_codes(fmt, rng, shape):
    t = orc.decode_table(fmt)
    return rng.choice(np.flatnonzero(np.isfinite(t)).astype(np.uint8), size=shape)


@pytest.mark.parametrize("fa,fb", [(orc.E4M3, orc.E4M3), (orc.E5M2, orc.E4M3)])
def test_all_code_pairs_1x1x1(fa, fb):
    a = np.arange(256, dtype=np.uint8).repeat(256).reshape(256 * 256, 1)
    b = np.tile(np.arange(256, dtype=np.uint8), 256).reshape(256 * 256, 1)
    va, vb = _lib_decode(fa, a[:, 0]), _lib_decode(fb, b[:, 0])
    with np.errstate(invalid="ignore"):
        want = va * vb
    # each pair is its own 1x1x1 product: row p of A with column p of B
    idx = np.arange(256 * 256)
    c, s = orc.gemm_at(a, fa, b, fb, 1.0, 1.0, idx, idx)
    nan = np.isnan(want)
    assert np.array_equal(nan, np.isnan(c))
    assert np.array_equal(c[~nan], want[~nan])


@pytest.mark.parametrize("fa,fb", [(orc.E4M3, orc.E4M3), (orc.E5M2, orc.E4M3)])
def test_tiny_against_exact_rationals(fa, fb):
    rng = np.random.default_rng(2)
    for trial in range(30):
        M, N, K = rng.integers(1, 9, 3)
        a = _finite_codes(fa, rng, (M, K))
        b = _finite_codes(fb, rng, (N, K))
        da = (rng.random(M) + 0.5).astype(np.float32)
        db = (rng.random(N) + 0.5).astype(np.float32)
        if trial % 3 == 0:
            da, db = da[:1], db[:1]
        c, s = orc.gemm(a, fa, b, fb, da, db, nthreads=2)
        va, vb = _lib_decode(fa, a), _lib_decode(fb, b)
        for i in range(M):
            for j in range(N):
                exact = sum(Fraction(va[i, k]) * Fraction(vb[j, k]) for k in range(K))
                exact_abs = sum(abs(Fraction(va[i, k]) * Fraction(vb[j, k])) for k in range(K))
                sa = Fraction(float(da[i if da.size > 1 else 0]))
                sb = Fraction(float(db[j if db.size > 1 else 0]))
                ref = exact * sa * sb
                # two FP64 scale products: within 2 ulp relative; the sum itself
                # is exact for these K
                assert abs(Fraction(c[i, j]) - ref) <= abs(ref) * Fraction(2, 2 ** 52)
                assert abs(Fraction(s[i, j]) - exact_abs * sa * sb) <= exact_abs * sa * sb * Fraction(2, 2 ** 52)


def test_all_ones_gives_K():
    for fmt, one in ((orc.E4M3, 0x38), (orc.E5M2, 0x3C)):
        for K in (1, 7, 128, 4096):
            a = np.full((3, K), one, np.uint8)
            b = np.full((5, K), one, np.uint8)
            c, s = orc.gemm(a, fmt, b, fmt, 1.0, 1.0, nthreads=1)
            assert np.all(c == K) and np.all(s == K)


@pytest.mark.parametrize("fmt", [orc.E4M3, orc.E5M2])
def test_identity_B(fmt):
    rng = np.random.default_rng(4)
    K = 16
    a = _finite_codes(fmt, rng, (6, K))
    one = 0x38 if fmt == orc.E4M3 else 0x3C
    eye = np.where(np.eye(K, dtype=bool), one, 0).astype(np.uint8)
    da = np.float32(0.375)
    db = np.float32(3.0)
    c, _ = orc.gemm(a, fmt, eye, orc.E4M3 if fmt == orc.E4M3 else orc.E5M2, da, db, nthreads=1)
    assert np.array_equal(c, _lib_decode(fmt, a) * float(da) * float(db))


def test_power_of_two_scales_are_exact():
    rng = np.random.default_rng(5)
    a = _finite_codes(orc.E4M3, rng, (8, 64))
    b = _finite_codes(orc.E4M3, rng, (9, 64))
    c1, s1 = orc.gemm(a, 0, b, 0, 1.0, 1.0, nthreads=1)
    da = (2.0 ** rng.integers(-10, 10, 8)).astype(np.float32)
    db = (2.0 ** rng.integers(-10, 10, 9)).astype(np.float32)
    c2, s2 = orc.gemm(a, 0, b, 0, da, db, nthreads=1)
    assert np.array_equal(c2, c1 * da[:, None] * db[None, :])


def test_row_blocks_and_sampled_entries_agree_with_full():
    rng = np.random.default_rng(6)
    a = _finite_codes(orc.E4M3, rng, (37, 96))
    b = _finite_codes(orc.E4M3, rng, (29, 96))
    da = rng.random(37).astype(np.float32)
    db = rng.random(29).astype(np.float32)
    c, s = orc.gemm(a, 0, b, 0, da, db, nthreads=3)
    c2, s2 = orc.gemm(a, 0, b, 0, da, db, rows=(10, 20), nthreads=4)
    assert np.array_equal(c[10:20], c2[10:20])
    ii = rng.integers(0, 37, 100)
    jj = rng.integers(0, 29, 100)
    c3, s3 = orc.gemm_at(a, 0, b, 0, da, db, ii, jj)
    assert np.array_equal(c3, c[ii, jj]) and np.array_equal(s3, s[ii, jj])


def test_sparse_equals_dense_on_pruned():
    """dense GEMM on the pruned matrix equals a direct sum over the compressed
    values gathered by the metadata indices (an independent formula)."""
    rng = np.random.default_rng(8)
    M, N, K = 12, 10, 64
    x = synth.normal_outliers(8, (M, K))
    qa, sa, da = orc.quantize(x, orc.E4M3, True)
    qb, sb, db = orc.quantize(synth.normal_outliers(9, (N, K)), orc.E4M3, True)
    values, meta, mask, pruned = orc.prune24(qa, orc.E4M3)
    c_dense, _ = orc.gemm(pruned, 0, qb, 0, da, db, nthreads=2)
    c_decomp, _ = orc.gemm(orc.decompress24(values, meta, K), 0, qb, 0, da, db, nthreads=2)
    assert np.array_equal(c_dense, c_decomp)
    va = _lib_decode(orc.E4M3, values).reshape(M, K // 4, 2)
    vb = _lib_decode(orc.E4M3, qb)
    nib = np.stack([meta & 0xF, meta >> 4], axis=-1).reshape(M, K // 4)
    idx = np.stack([nib & 3, nib >> 2], axis=-1) + 4 * np.arange(K // 4)[None, :, None]
    direct = np.zeros((M, N))
    for i in range(M):
        for j in range(N):
            direct[i, j] = np.sum(va[i] * vb[j][idx[i]])
    direct = direct * da[:, None].astype(np.float64) * db[None, :].astype(np.float64)
    assert np.array_equal(direct, c_dense)


# ------------------------------------------------------------- validator ----

def _case(fa=orc.E4M3, M=64, N=48, K=512, seed=0):
    xa = synth.normal_outliers(seed, (M, K))
    xb = synth.normal_outliers(seed + 1, (N, K))
    qa, _, da = orc.quantize(xa, fa, True)
    qb, _, db = orc.quantize(xb, orc.E4M3, True)
    return qa, qb, da, db


def _fp32_gemm(qa, fa, qb, fb, da, db):
    """A faithful FP32-accumulating GEMM on the decoded values (what a correct
    device kernel does), used to exercise the bound."""
    va = orc.decode(fa, qa).astype(np.float32)
    vb = orc.decode(fb, qb).astype(np.float32)
    acc = np.zeros((va.shape[0], vb.shape[0]), np.float32)
    for k in range(va.shape[1]):
        acc += np.outer(va[:, k], vb[:, k]).astype(np.float32)
    return (acc * da[:, None]) * db[None, :]


def _bf16_rne(x):
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16).astype(np.uint16)
    return orc.bf16_to_f64(r)


def _bf16_trunc(x):
    return orc.bf16_to_f64((np.asarray(x, np.float32).view(np.uint32) >> 16).astype(np.uint16))


def test_validator_accepts_correct_fp32_and_bf16():
    qa, qb, da, db = _case()
    cref, sabs = orc.gemm(qa, 0, qb, 0, da, db)
    c = _fp32_gemm(qa, 0, qb, 0, da, db)
    assert orc.check(c, cref, sabs, 512, orc.OUT_F32)["ok"]
    assert orc.check(_bf16_rne(c), cref, sabs, 512, orc.OUT_BF16)["ok"]


def test_validator_rejects_mutants():
    qa, qb, da, db = _case()
    K = qa.shape[1]
    cref, sabs = orc.gemm(qa, 0, qb, 0, da, db)
    good = _fp32_gemm(qa, 0, qb, 0, da, db)
    # a dropped K block of 128
    q2 = qa.copy()
    q2[:, 128:256] = 0
    dropped = _fp32_gemm(q2, 0, qb, 0, da, db)
    assert not orc.check(dropped, cref, sabs, K, orc.OUT_F32)["ok"]
    # a wrong scale (one ulp-scale error of 2^-10 relative on a row)
    da2 = da.copy()
    da2[3] *= np.float32(1 + 2.0 ** -10)
    assert not orc.check(_fp32_gemm(qa, 0, qb, 0, da2, db), cref, sabs, K, orc.OUT_F32)["ok"]
    # operands decoded in the wrong format
    assert not orc.check(_fp32_gemm(qa, 1, qb, 0, da, db), cref, sabs, K, orc.OUT_F32)["ok"]
    # BF16 by truncation instead of round to nearest even
    assert not orc.check(_bf16_trunc(good), cref, sabs, K, orc.OUT_BF16)["ok"]
    # an off-by-one transposition of the output
    assert not orc.check(np.roll(good, 1, axis=1), cref, sabs, K, orc.OUT_F32)["ok"]
