"""Pins for the oracle's real-valued FP64 GEMM (the FP32 and 16-bit stages of
the mixed-precision sequence) and for the FP16-output acceptance bound."""
from fractions import Fraction

import numpy as np
import pytest

import oracle as orc


def _exact(a, b, sa, sb):
    """Exact rational C and S_abs (scales applied as in the definition)."""
    M, K = a.shape
    N = b.shape[0]
    c = np.zeros((M, N))
    s = np.zeros((M, N))
    for i in range(M):
        for j in range(N):
            tot = sum(Fraction(float(a[i, k])) * Fraction(float(b[j, k])) for k in range(K))
            ab = sum(abs(Fraction(float(a[i, k])) * Fraction(float(b[j, k]))) for k in range(K))
            si = Fraction(float(sa[i if sa.size > 1 else 0]))
            sj = Fraction(float(sb[j if sb.size > 1 else 0]))
            c[i, j] = float(tot * si * sj)
            s[i, j] = float(ab * abs(si * sj))
    return c, s


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (3, 4, 5), (5, 2, 9), (2, 7, 16)])
def test_tiny_against_exact_rationals(dtype, M, N, K):
    rng = np.random.default_rng(M * 100 + N * 10 + K)
    a = (rng.standard_normal((M, K)) * 2.0 ** rng.integers(-6, 6, (M, K))).astype(dtype)
    b = (rng.standard_normal((N, K)) * 2.0 ** rng.integers(-6, 6, (N, K))).astype(dtype)
    sa = rng.uniform(0.5, 2.0, M).astype(np.float32)
    sb = rng.uniform(0.5, 2.0, N).astype(np.float32)
    c, s = orc.gemm_real(a, b, sa, sb)
    ce, se = _exact(a, b, sa, sb)
    # the FP64 sum errs by at most K 2^-53 S_abs; the scales add two roundings
    tol = (K + 3) * 2.0 ** -53 * se
    assert np.all(np.abs(c - ce) <= tol)
    assert np.allclose(s, se, rtol=2.0 ** -50, atol=0)


def test_all_ones_and_identity():
    K = 37
    c, s = orc.gemm_real(np.ones((3, K), np.float32), np.ones((4, K), np.float32))
    assert np.all(c == K) and np.all(s == K)
    rng = np.random.default_rng(5)
    a = rng.standard_normal((6, 8)).astype(np.float32)
    c, _ = orc.gemm_real(a, np.eye(8, dtype=np.float32))
    assert np.array_equal(c, a.astype(np.float64))


def test_transpose_symmetry_and_power_of_two_scales():
    rng = np.random.default_rng(6)
    a = rng.standard_normal((5, 33)).astype(np.float32)
    b = rng.standard_normal((7, 33)).astype(np.float32)
    c, _ = orc.gemm_real(a, b)
    ct, _ = orc.gemm_real(b, a)
    assert np.array_equal(c, ct.T)
    sa = (2.0 ** rng.integers(-4, 4, 5)).astype(np.float32)
    sb = (2.0 ** rng.integers(-4, 4, 7)).astype(np.float32)
    cs, _ = orc.gemm_real(a, b, sa, sb)
    assert np.array_equal(cs, c * sa[:, None].astype(np.float64) * sb[None, :].astype(np.float64))


def test_agrees_with_fp8_oracle_on_fp8_values():
    """On operands holding FP8 values, the real-valued GEMM equals the
    (separately pinned) FP8 oracle bit for bit: both sums are exact."""
    rng = np.random.default_rng(7)
    t = orc.decode_table(orc.E4M3)
    finite = np.flatnonzero(np.isfinite(t)).astype(np.uint8)
    qa = rng.choice(finite, (9, 200))
    qb = rng.choice(finite, (11, 200))
    da = rng.uniform(0.01, 1, 9).astype(np.float32)
    db = rng.uniform(0.01, 1, 11).astype(np.float32)
    c8, s8 = orc.gemm(qa, orc.E4M3, qb, orc.E4M3, da, db)
    cr, sr = orc.gemm_real(t[qa], t[qb], da, db)
    assert np.array_equal(c8, cr) and np.array_equal(s8, sr)


def test_fp16_output_bound_accepts_rne_rejects_truncation():
    rng = np.random.default_rng(8)
    a = rng.standard_normal((40, 64)).astype(np.float16)
    b = rng.standard_normal((30, 64)).astype(np.float16)
    cref, sabs = orc.gemm_real(a, b)
    rne = cref.astype(np.float16).astype(np.float64)
    assert orc.check(rne, cref, sabs, 64, orc.OUT_F16)["ok"]
    # truncation toward zero to 11 significant bits: off by up to one FP16 ulp
    m, e = np.frexp(cref)
    trunc = np.ldexp(np.trunc(m * 2.0 ** 11) / 2.0 ** 11, e)
    assert not orc.check(trunc, cref, sabs, 64, orc.OUT_F16)["ok"]
    # a dropped K block is rejected
    cref2, _ = orc.gemm_real(a[:, :48], b[:, :48])
    assert not orc.check(cref2.astype(np.float16).astype(np.float64), cref, sabs, 64, orc.OUT_F16)["ok"]
