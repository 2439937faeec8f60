"""Pins for the oracle's FP8 decode and encode (OCP E4M3 / E5M2, the FP8
formats of the paper's Sec. 2 "FP8 Matrix Cores")."""
import math
import os

import numpy as np
import pytest
import torch

import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ocp_fp8_anchors.txt")
FMT = {"E4M3": orc.E4M3, "E5M2": orc.E5M2}
TORCH_DT = {orc.E4M3: torch.float8_e4m3fn, orc.E5M2: torch.float8_e5m2}


def _golden():
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if line:
            f, c, v = line.split()
            yield FMT[f], int(c, 16), v


def test_decode_matches_spec_anchors():
    n = 0
    for fmt, code, v in _golden():
        got = orc.decode(fmt, [code])[0]
        if v == "nan":
            assert math.isnan(got), (fmt, hex(code))
        elif v == "-0":
            assert got == 0.0 and math.copysign(1.0, got) < 0
        else:
            assert got == float(v), (fmt, hex(code), got, v)
        n += 1
    assert n >= 20


@pytest.mark.parametrize("fmt", [orc.E4M3, orc.E5M2])
def test_decode_matches_library_decoder(fmt):
    """torch's float8 dtypes decode the same OCP formats independently."""
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8)
    ref = codes.view(TORCH_DT[fmt]).to(torch.float64).numpy()
    got = orc.decode_table(fmt)
    nan = np.isnan(ref)
    assert np.array_equal(nan, np.isnan(got))
    assert np.array_equal(ref[~nan], got[~nan])
    assert np.array_equal(np.signbit(ref[~nan]), np.signbit(got[~nan]))


@pytest.mark.parametrize("fmt", [orc.E4M3, orc.E5M2])
def test_decode_structure(fmt):
    t = orc.decode_table(fmt)
    top = 0x7E if fmt == orc.E4M3 else 0x7B
    pos = t[: top + 1]
    assert np.all(np.diff(pos) > 0), "finite codes ascend with the code"
    assert np.array_equal(t[0x80:0x80 + top + 1], -pos)
    n_nan = int(np.isnan(t).sum())
    assert n_nan == (2 if fmt == orc.E4M3 else 6)
    assert int(np.isinf(t).sum()) == (0 if fmt == orc.E4M3 else 2)
    assert orc.FMAX[fmt] == t[top]


@pytest.mark.parametrize("fmt", [orc.E4M3, orc.E5M2])
def test_encode_roundtrip_all_codes(fmt):
    t = orc.decode_table(fmt)
    for c in range(256):
        v = t[c]
        if math.isnan(v):
            continue
        got = int(orc.encode(fmt, [np.float32(v)])[0])
        if math.isinf(v):   # saturation
            assert got == (0x7B | (c & 0x80)), hex(c)
        else:
            assert got == c, (hex(c), hex(got))


@pytest.mark.parametrize("fmt", [orc.E4M3, orc.E5M2])
def test_encode_midpoints_go_to_even(fmt):
    t = orc.decode_table(fmt)
    top = 0x7E if fmt == orc.E4M3 else 0x7B
    for c in range(top):
        lo, hi = t[c], t[c + 1]
        mid = np.float32(0.5 * (lo + hi))
        assert float(mid) == 0.5 * (lo + hi)        # representable in FP32
        even = c if c % 2 == 0 else c + 1
        assert orc.encode(fmt, [mid])[0] == even
        assert orc.encode(fmt, [-mid])[0] == even | 0x80
        below = np.nextafter(mid, np.float32(0))
        above = np.nextafter(mid, np.float32(np.inf))
        assert orc.encode(fmt, [below])[0] == c
        assert orc.encode(fmt, [above])[0] == c + 1


@pytest.mark.parametrize("fmt", [orc.E4M3, orc.E5M2])
def test_encode_specials(fmt):
    top = 0x7E if fmt == orc.E4M3 else 0x7B
    fmax = orc.FMAX[fmt]
    cases = [
        (0.0, 0x00), (-0.0, 0x80), (float("inf"), top), (float("-inf"), top | 0x80),
        (fmax * 1.001, top), (-fmax * 4, top | 0x80), (3.0e38, top), (1e-30, 0x00),
        (-1e-30, 0x80), (1.4e-45, 0x00),
    ]
    for x, want in cases:
        assert orc.encode(fmt, [np.float32(x)])[0] == want, (x, want)
    assert orc.encode(fmt, [np.float32("nan")])[0] == 0x7F
    assert orc.encode(fmt, [-np.float32("nan")])[0] == 0xFF


@pytest.mark.parametrize("fmt", [orc.E4M3, orc.E5M2])
def test_encode_matches_library_in_range(fmt):
    """torch's float32 -> float8 cast rounds to nearest-even; inside the finite
    range (where it does not overflow to NaN/Inf) it must agree bit for bit."""
    rng = np.random.default_rng(7)
    fmax = orc.FMAX[fmt]
    x = np.concatenate([
        rng.uniform(-fmax, fmax, 20000),
        rng.standard_normal(20000) * 2.0 ** rng.integers(-20, 8, 20000),
    ]).astype(np.float32)
    x = x[np.abs(x) <= fmax]
    ref = torch.from_numpy(x).to(TORCH_DT[fmt]).view(torch.uint8).numpy()
    got = orc.encode(fmt, x)
    assert np.array_equal(ref, got)


@pytest.mark.parametrize("fmt", [orc.E4M3, orc.E5M2])
def test_encode_exhaustive_against_second_encoder(fmt):
    """Every non-negative FP32 bit pattern: the definition encoder (nearest by
    search) equals an independent integer-rounding encoder."""
    bad, first = orc.encode_sweep(fmt, 0, 1 << 31, nthreads=os.cpu_count() or 8)
    assert bad == 0, hex(first)


@pytest.mark.parametrize("fmt", [orc.E4M3, orc.E5M2])
def test_encode_sign_symmetry(fmt):
    rng = np.random.default_rng(3)
    bits = rng.integers(0, 1 << 31, 50000, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    pos = orc.encode(fmt, x)
    neg = orc.encode(fmt, -x)
    assert np.array_equal(neg, pos | 0x80)
