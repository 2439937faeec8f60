"""Pins for the oracle's amax/scale/quantize and 2:4 prune/compress."""
import os

import numpy as np
import pytest

import oracle as orc
from paper_2602_10262_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "prune24_cases.txt")


# ---------------------------------------------------------------- scale ----

def test_scale_closed_forms():
    assert orc.scale(orc.E4M3, 1.0) == (np.float32(448.0), np.float32(1.0) / np.float32(448.0))
    assert orc.scale(orc.E4M3, 448.0) == (1.0, 1.0)
    assert orc.scale(orc.E5M2, 57344.0) == (1.0, 1.0)
    assert orc.scale(orc.E5M2, 7.0)[0] == np.float32(57344.0) / np.float32(7.0)
    for bad in (0.0, float("inf"), float("nan"), 1e-45):
        assert orc.scale(orc.E4M3, bad) == (1.0, 1.0), bad


@pytest.mark.parametrize("fmt", [orc.E4M3, orc.E5M2])
@pytest.mark.parametrize("per_row", [False, True])
def test_quantize_scale_invariance(fmt, per_row):
    """Scaling x by 2^p leaves every code unchanged and scales d by exactly 2^p."""
    x = synth.normal_outliers(11, (6, 40))
    q0, s0, d0 = orc.quantize(x, fmt, per_row)
    for p in (-7, 3, 20):
        q1, s1, d1 = orc.quantize(x * np.float32(2.0 ** p), fmt, per_row)
        assert np.array_equal(q0, q1)
        assert np.array_equal(d1, d0 * np.float32(2.0 ** p))


@pytest.mark.parametrize("fmt", [orc.E4M3, orc.E5M2])
def test_quantize_per_tensor_equals_encode_of_scaled(fmt):
    x = synth.uniform(0, 5, (8, 24))
    q, s, d = orc.quantize(x, fmt, False)
    amax = np.float32(np.abs(x).max())
    assert s[0] == np.float32(orc.FMAX[fmt]) / amax
    assert d[0] == np.float32(1.0) / s[0]
    assert np.array_equal(q, orc.encode(fmt, (x * s[0]).astype(np.float32)))
    # the largest magnitude lands on the largest finite code
    i = np.unravel_index(np.argmax(np.abs(x)), x.shape)
    assert q[i] & 0x7F == (0x7E if fmt == orc.E4M3 else 0x7B)


@pytest.mark.parametrize("fmt", [orc.E4M3, orc.E5M2])
def test_quantize_per_row_is_tensor_quantize_of_each_row(fmt):
    x = synth.normal_outliers(3, (5, 33))
    q, s, d = orc.quantize(x, fmt, True)
    for r in range(5):
        qr, sr, dr = orc.quantize(x[r:r + 1], fmt, False)
        assert np.array_equal(q[r], qr[0]) and s[r] == sr[0] and d[r] == dr[0]


@pytest.mark.parametrize("fmt", [orc.E4M3, orc.E5M2])
def test_quantize_error_within_half_ulp(fmt):
    """|dec(q) d - x| is at most half a unit in the last FP8 place (relative
    2^-4 for E4M3, 2^-3 for E5M2) plus the FP32 rounding of x s, for values in
    the normal range."""
    x = synth.normal_outliers(5, (16, 64))
    q, s, d = orc.quantize(x, fmt, True)
    y = orc.decode(fmt, q) * d[:, None].astype(np.float64)
    rel = 2.0 ** (-4 if fmt == orc.E4M3 else -3)
    tiny = np.float64(2.0 ** (-6 if fmt == orc.E4M3 else -14)) * d[:, None]
    ok = np.abs(y - x) <= rel * np.abs(x) * (1 + 2.0 ** -20) + tiny
    assert ok.all()


def test_quantize_zero_row_gets_unit_scale():
    x = np.zeros((3, 16), np.float32)
    x[1] = synth.uniform(0, 1, (16,))
    q, s, d = orc.quantize(x, orc.E4M3, True)
    assert s[0] == 1.0 and d[0] == 1.0 and s[2] == 1.0 and np.all(q[0] == 0)


# ---------------------------------------------------------------- prune ----

def _golden_cases():
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if line:
            f = line.split()
            yield [float(v) for v in f[:4]], int(f[4]), int(f[5]), int(f[6])


def test_prune_worked_cases():
    for vals, i0, i1, nib in _golden_cases():
        row = orc.encode(orc.E4M3, np.array(vals + [0, 0, 0, 0], np.float32))[None, :]
        values, meta, mask, pruned = orc.prune24(row, orc.E4M3)
        assert list(values[0, :2]) == [row[0, i0], row[0, i1]], vals
        assert meta[0, 0] & 0xF == nib, vals
        assert mask[0, 0] & 0xF == (1 << i0) | (1 << i1), vals


def _second_prune(codes: np.ndarray, fmt: int):
    """Independent implementation: stable sort of the four positions by
    descending magnitude, first two kept (numpy, vectorised)."""
    t = np.abs(orc.decode_table(fmt))
    mag = t[codes.reshape(-1, 4)]
    order = np.argsort(-mag, axis=1, kind="stable")[:, :2]
    order.sort(axis=1)
    return order


@pytest.mark.parametrize("fmt", [orc.E4M3, orc.E5M2])
def test_prune_exhaustive_order_patterns(fmt):
    """All 4^4 weak orders of four magnitudes (ties included), each with all 16
    sign patterns, plus all 16^4 patterns over 16 magnitudes spread across the
    code range; compared with a sort-based second implementation."""
    top = 0x7E if fmt == orc.E4M3 else 0x7B
    pats = []
    lv = np.array([0, 9, 40, top], np.uint8)
    g = np.array(np.meshgrid(*[np.arange(4)] * 4, indexing="ij")).reshape(4, -1).T
    for sgn in range(16):
        sb = np.array([(sgn >> i) & 1 for i in range(4)], np.uint8) << 7
        pats.append(lv[g] | sb)
    mags = np.linspace(0, top, 16).astype(np.uint8)
    g16 = np.array(np.meshgrid(*[np.arange(16)] * 4, indexing="ij")).reshape(4, -1).T
    pats.append(mags[g16])
    codes = np.concatenate(pats).astype(np.uint8)
    K = 512
    n = codes.shape[0]
    pad = (-n) % (K // 4)
    codes = np.concatenate([codes, np.zeros((pad, 4), np.uint8)])
    x = codes.reshape(-1, K)
    values, meta, mask, pruned = orc.prune24(x, fmt)
    ref = _second_prune(x, fmt)
    nib = np.stack([meta & 0xF, meta >> 4], axis=-1).reshape(-1)
    assert np.array_equal(nib & 3, ref[:, 0])
    assert np.array_equal(nib >> 2, ref[:, 1])
    vals = values.reshape(-1, 2)
    grp = x.reshape(-1, 4)
    assert np.array_equal(vals[:, 0], grp[np.arange(grp.shape[0]), ref[:, 0]])
    assert np.array_equal(vals[:, 1], grp[np.arange(grp.shape[0]), ref[:, 1]])


@pytest.mark.parametrize("fmt", [orc.E4M3, orc.E5M2])
def test_prune_invariants_random(fmt):
    rng = np.random.default_rng(1)
    t = orc.decode_table(fmt)
    finite = np.flatnonzero(np.isfinite(t)).astype(np.uint8)
    x = rng.choice(finite, size=(64, 256))
    values, meta, mask, pruned = orc.prune24(x, fmt)
    # exactly two kept per group; mask agrees with the pruned matrix
    bits = np.unpackbits(mask, axis=1, bitorder="little").astype(bool)
    assert np.all(bits.reshape(64, -1, 4).sum(-1) == 2)
    assert np.array_equal(np.where(bits, x, 0).astype(np.uint8), pruned)
    # min kept >= max dropped (by magnitude)
    mag = np.abs(t[x]).reshape(64, -1, 4)
    b4 = bits.reshape(64, -1, 4)
    assert np.all(np.where(b4, mag, np.inf).min(-1) >= np.where(~b4, mag, -np.inf).max(-1))
    # compressed form decompresses to the pruned matrix
    assert np.array_equal(orc.decompress24(values, meta, 256), pruned)
    # idempotence: pruning the pruned matrix changes nothing
    v2, m2, k2, p2 = orc.prune24(pruned, fmt)
    assert np.array_equal(v2, values) and np.array_equal(m2, meta) and np.array_equal(p2, pruned)
    # library cross-check on a sample: the nibbles name the kept positions
    ref = _second_prune(x, fmt)
    nib = np.stack([meta & 0xF, meta >> 4], axis=-1).reshape(-1)
    assert np.array_equal(nib & 3, ref[:, 0]) and np.array_equal(nib >> 2, ref[:, 1])


def test_meta_nibble_order():
    """Low nibble of each metadata byte is the even group; the little-endian
    32-bit word w of a row holds groups 8w .. 8w+7."""
    v = np.zeros((1, 32), np.float32)
    for g in range(8):                      # group g keeps positions (g % 3, 3)
        v[0, 4 * g + g % 3] = 2.0
        v[0, 4 * g + 3] = 4.0
    x = orc.encode(orc.E4M3, v)
    _, meta, _, _ = orc.prune24(x, orc.E4M3)
    word = int(meta[0].view("<u4")[0])
    for g in range(8):
        assert (word >> (4 * g)) & 0xF == (g % 3) | (3 << 2)
