"""Python face of the CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU-baseline
leg of the benchmark call this module; the library never does.  It imports
nothing from the GPU package and the GPU package imports nothing from it.

Each wrapper marshals numpy arrays into the C routine that states the
definition it follows (FP8 decode/encode per the OCP formats the paper names in
Sec. 2; amax-derived scales; the 2:4 pattern of Sec. 2 and Sec. 7; the FP64
GEMM), plus the acceptance bound the GPU results are checked against.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

E4M3, E5M2 = 0, 1
FMAX = {E4M3: 448.0, E5M2: 57344.0}
OUT_F32, OUT_BF16, OUT_F16 = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile oracle.c with plain gcc (no fast-math) into liboracle.so."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P, I64, I, F = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_float
    lib.orc_decode.argtypes = [I, ctypes.c_uint8]
    lib.orc_decode.restype = ctypes.c_double
    lib.orc_max_finite.argtypes = [I]
    lib.orc_max_finite.restype = ctypes.c_double
    lib.orc_encode.argtypes = [I, F]
    lib.orc_encode.restype = ctypes.c_uint8
    lib.orc_encode_bitwise.argtypes = [I, F]
    lib.orc_encode_bitwise.restype = ctypes.c_uint8
    lib.orc_encode_sweep.argtypes = [I, ctypes.c_uint64, ctypes.c_uint64, I, ctypes.POINTER(ctypes.c_uint32)]
    lib.orc_encode_sweep.restype = ctypes.c_uint64
    lib.orc_encode_range.argtypes = [I, ctypes.c_uint32, I64, P, I]
    lib.orc_scale.argtypes = [I, F, P, P]
    lib.orc_quantize.argtypes = [P, I64, I64, I64, I, I, P, I64, P, P]
    lib.orc_prune24.argtypes = [P, I, I64, I64, I64, P, P, P, P]
    lib.orc_decompress24.argtypes = [P, P, I64, I64, P]
    lib.orc_gemm.argtypes = [P, I, I64, P, I, I64, P, I, P, I, I64, I64, I64, I64, I64, P, P, I]
    lib.orc_gemm_at.argtypes = [P, I, I64, P, I, I64, P, I, P, I, I64, P, P, I64, P, P]
    lib.orc_gemm_real.argtypes = [P, I64, P, I64, P, I, P, I, I64, I64, I64, P, P, I]
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def decode(fmt: int, codes) -> np.ndarray:
    """Exact FP64 value of each FP8 code."""
    lib = _load()
    codes = np.asarray(codes, dtype=np.uint8)
    table = np.array([lib.orc_decode(fmt, c) for c in range(256)], dtype=np.float64)
    return table[codes]


def decode_table(fmt: int) -> np.ndarray:
    return decode(fmt, np.arange(256, dtype=np.uint8))


def encode(fmt: int, x) -> np.ndarray:
    """Definition encoder: nearest finite FP8 value, ties to even, saturating."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(x.shape, dtype=np.uint8)
    flat, of = x.reshape(-1), out.reshape(-1)
    for i in range(flat.size):
        of[i] = lib.orc_encode(fmt, float(flat[i]))
    return out


def encode_bitwise(fmt: int, x) -> np.ndarray:
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(x.shape, dtype=np.uint8)
    flat, of = x.reshape(-1), out.reshape(-1)
    for i in range(flat.size):
        of[i] = lib.orc_encode_bitwise(fmt, float(flat[i]))
    return out


def encode_sweep(fmt: int, lo: int, hi: int, nthreads: int = 8):
    """Compare both encoders on FP32 bit patterns [lo, hi): (mismatches, first)."""
    lib = _load()
    first = ctypes.c_uint32(0)
    bad = lib.orc_encode_sweep(fmt, lo, hi, nthreads, ctypes.byref(first))
    return int(bad), int(first.value)


def encode_range(fmt: int, lo: int, n: int, nthreads: int | None = None) -> np.ndarray:
    """Codes of the FP32 values whose bit patterns are lo, lo+1, ..., lo+n-1."""
    lib = _load()
    out = np.empty(n, np.uint8)
    lib.orc_encode_range(fmt, lo, n, _ptr(out), nthreads or os.cpu_count() or 1)
    return out


def scale(fmt: int, amax: float):
    lib = _load()
    s = np.zeros(1, np.float32)
    d = np.zeros(1, np.float32)
    lib.orc_scale(fmt, float(amax), _ptr(s), _ptr(d))
    return s[0], d[0]


def quantize(x: np.ndarray, fmt: int, per_row: bool):
    """(codes, s, d) for a row-major FP32 matrix; s, d hold 1 or rows floats."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32)
    rows, cols = x.shape
    q = np.empty((rows, cols), np.uint8)
    n = rows if per_row else 1
    s = np.empty(n, np.float32)
    d = np.empty(n, np.float32)
    lib.orc_quantize(_ptr(x), rows, cols, cols, fmt, int(per_row), _ptr(q), cols, _ptr(s), _ptr(d))
    return q, s, d


def prune24(x: np.ndarray, fmt: int):
    """(values, meta, mask, pruned) for a row-major rows x K code matrix."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.uint8)
    rows, K = x.shape
    assert K % 4 == 0
    values = np.zeros((rows, K // 2), np.uint8)
    if K % 8 != 0:
        raise ValueError("the compressed format packs two groups per metadata byte: K % 8 == 0")
    meta = np.zeros((rows, K // 8), np.uint8)
    mask = np.zeros_like(meta)
    pruned = np.zeros((rows, K), np.uint8)
    lib.orc_prune24(_ptr(x), fmt, rows, K, K, _ptr(values), _ptr(meta), _ptr(mask), _ptr(pruned))
    return values, meta, mask, pruned


def decompress24(values: np.ndarray, meta: np.ndarray, K: int) -> np.ndarray:
    lib = _load()
    values = np.ascontiguousarray(values, dtype=np.uint8)
    meta = np.ascontiguousarray(meta, dtype=np.uint8)
    rows = values.shape[0]
    out = np.empty((rows, K), np.uint8)
    lib.orc_decompress24(_ptr(values), _ptr(meta), rows, K, _ptr(out))
    return out


def gemm(a: np.ndarray, a_fmt: int, b_nk: np.ndarray, b_fmt: int, da, db,
         rows=None, nthreads: int | None = None):
    """FP64 (C_ref, S_abs) for C = diag(d_a) dec(A) dec(B) diag(d_b).

    a: M x K codes (row-major); b_nk: N x K codes (B column-major, one row per
    column of B); da: 1 or M floats; db: 1 or N floats.  rows = (lo, hi)
    restricts the computation to a block of rows (returned arrays are M x N
    with only those rows filled)."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b_nk = np.ascontiguousarray(b_nk, dtype=np.uint8)
    M, K = a.shape
    N, K2 = b_nk.shape
    assert K == K2
    da = np.ascontiguousarray(np.atleast_1d(np.asarray(da, dtype=np.float32)))
    db = np.ascontiguousarray(np.atleast_1d(np.asarray(db, dtype=np.float32)))
    a_per_row = int(da.size > 1)
    b_per_col = int(db.size > 1)
    assert da.size in (1, M) and db.size in (1, N)
    lo, hi = (0, M) if rows is None else rows
    cref = np.zeros((M, N), np.float64)
    sabs = np.zeros((M, N), np.float64)
    nt = nthreads or os.cpu_count() or 1
    lib.orc_gemm(_ptr(a), a_fmt, K, _ptr(b_nk), b_fmt, K, _ptr(da), a_per_row, _ptr(db), b_per_col,
                 M, N, K, lo, hi, _ptr(cref), _ptr(sabs), nt)
    return cref, sabs


def gemm_at(a: np.ndarray, a_fmt: int, b_nk: np.ndarray, b_fmt: int, da, db, ii, jj):
    """(C_ref, S_abs) at the listed output positions only."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b_nk = np.ascontiguousarray(b_nk, dtype=np.uint8)
    M, K = a.shape
    N, _ = b_nk.shape
    da = np.ascontiguousarray(np.atleast_1d(np.asarray(da, dtype=np.float32)))
    db = np.ascontiguousarray(np.atleast_1d(np.asarray(db, dtype=np.float32)))
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    cref = np.zeros(ii.size, np.float64)
    sabs = np.zeros(ii.size, np.float64)
    lib.orc_gemm_at(_ptr(a), a_fmt, K, _ptr(b_nk), b_fmt, K, _ptr(da), int(da.size > 1), _ptr(db),
                    int(db.size > 1), K, _ptr(ii), _ptr(jj), ii.size, _ptr(cref), _ptr(sabs))
    return cref, sabs


def gemm_real(a: np.ndarray, b_nk: np.ndarray, sa=1.0, sb=1.0, nthreads: int | None = None):
    """FP64 (C_ref, S_abs) for C = diag(s_a) A B diag(s_b) with real-valued
    operands (FP32, FP16 or BF16 arrays, or FP64 holding such values).

    a: M x K (row-major); b_nk: N x K (B column-major); sa: 1 or M floats;
    sb: 1 or N floats."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float64)
    b_nk = np.ascontiguousarray(b_nk, dtype=np.float64)
    M, K = a.shape
    N, K2 = b_nk.shape
    assert K == K2
    sa = np.ascontiguousarray(np.atleast_1d(np.asarray(sa, dtype=np.float32)))
    sb = np.ascontiguousarray(np.atleast_1d(np.asarray(sb, dtype=np.float32)))
    assert sa.size in (1, M) and sb.size in (1, N)
    cref = np.zeros((M, N), np.float64)
    sabs = np.zeros((M, N), np.float64)
    nt = nthreads or os.cpu_count() or 1
    lib.orc_gemm_real(_ptr(a), K, _ptr(b_nk), K, _ptr(sa), int(sa.size > 1), _ptr(sb), int(sb.size > 1),
                      M, N, K, _ptr(cref), _ptr(sabs), nt)
    return cref, sabs


# --------------------------------------------------------------------------
# Acceptance bound
# --------------------------------------------------------------------------

U32 = 2.0 ** -24     # unit roundoff of FP32
UBF16 = 2.0 ** -8    # unit roundoff of BF16 (8 significant bits)
UF16 = 2.0 ** -11    # unit roundoff of FP16 (11 significant bits)
F16_SUB_HALF = 2.0 ** -25   # half the spacing of FP16 subnormals


def bound(sabs: np.ndarray, cref: np.ndarray, K: int, out_type: int) -> np.ndarray:
    """Elementwise tolerance: 4 K u S_abs for FP32 output; for BF16 output the
    FP32 bound grown by one BF16 round-to-nearest step:
    (1 + 2^-8) 4 K u S_abs + 2^-8 |C_ref|; for FP16 output likewise with
    2^-11, plus 2^-25 for results in the FP16 subnormal range (in range: no
    result may exceed the FP16 maximum)."""
    base = 4.0 * K * U32 * sabs
    if out_type == OUT_F32:
        return base
    if out_type == OUT_F16:
        return (1.0 + UF16) * base + UF16 * np.abs(cref) + F16_SUB_HALF
    return (1.0 + UBF16) * base + UBF16 * np.abs(cref)


def bf16_to_f64(raw: np.ndarray) -> np.ndarray:
    """Exact value of BF16 bit patterns (uint16) as FP64."""
    raw = np.asarray(raw, dtype=np.uint16).astype(np.uint32) << 16
    return raw.view(np.float32).astype(np.float64)


def check(c: np.ndarray, cref: np.ndarray, sabs: np.ndarray, K: int, out_type: int) -> dict:
    """Max abs error, max error/bound ratio (must be <= 1), normwise error."""
    c = np.asarray(c, dtype=np.float64)
    err = np.abs(c - cref)
    b = bound(sabs, cref, K, out_type)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(b > 0, err / np.where(b > 0, b, 1.0), np.where(err > 0, np.inf, 0.0))
    nref = float(np.linalg.norm(cref.ravel()))
    return {
        "max_abs_err": float(err.max()) if err.size else 0.0,
        "max_ratio": float(ratio.max()) if ratio.size else 0.0,
        "normwise": float(np.linalg.norm((c - cref).ravel()) / nref) if nref > 0 else float(np.linalg.norm(err)),
        "ok": bool(np.all(err <= b)) and bool(np.all(np.isfinite(c) == np.isfinite(cref))),
        "n": int(c.size),
    }
