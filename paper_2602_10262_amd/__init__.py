"""MI355X-native FP8 GEMM (dense and 2:4 structured-sparse) for gfx950.

Thin Python binding of libfp8gemm.so (include/fp8gemm.h): every function has
the name of the C entry point it calls and only marshals arguments.  Device
memory and streams come from PyTorch (tensors' data_ptr, the current stream);
every step of the computation runs in the library's HIP kernels.  There is no
fallback: if the library is not built, load() raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfp8gemm.so")

FP8_E4M3, FP8_E5M2 = 0, 1
FP8_OUT_F32, FP8_OUT_BF16, FP8_OUT_F16 = 0, 1, 2
FP8_HP_F32, FP8_HP_F16, FP8_HP_BF16 = 0, 1, 2
FP8_STAGE_F32, FP8_STAGE_F16, FP8_STAGE_BF16, FP8_STAGE_FP8 = 0, 1, 2, 3
FP8_CHAIN_SERIAL, FP8_CHAIN_IN_PHASE, FP8_CHAIN_STAGGERED = 0, 1, 2
FP8_SCALE_TENSOR, FP8_SCALE_ROW = 0, 1
FP8_SPARSE_A, FP8_SPARSE_B = 0, 1
STATUS = ["FP8_OK", "FP8_ERR_ARG", "FP8_ERR_SHAPE", "FP8_ERR_ALIGN", "FP8_ERR_UNSUPPORTED", "FP8_ERR_HIP",
          "FP8_ERR_NOMEM", "FP8_ERR_BUDGET", "FP8_ERR_CLOSED", "FP8_ERR_PENDING", "FP8_ERR_TIMEOUT"]
FP8_OK, FP8_ERR_PENDING, FP8_ERR_TIMEOUT = 0, 9, 10

_P, _I64, _I, _SZ, _D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t, ctypes.c_double


class GemmArgs(ctypes.Structure):
    _fields_ = [("M", _I64), ("N", _I64), ("K", _I64),
                ("a", _P), ("a_fmt", _I), ("lda", _I64),
                ("b", _P), ("b_fmt", _I), ("ldb", _I64),
                ("a_descale", _P), ("a_kind", _I),
                ("b_descale", _P), ("b_kind", _I),
                ("c", _P), ("c_type", _I), ("ldc", _I64)]


class Plan(ctypes.Structure):
    _fields_ = [("tile", _I), ("split_k", _I)]


class Sparse24GemmArgs(ctypes.Structure):
    _fields_ = [("g", GemmArgs), ("side", _I), ("values", _P), ("meta", _P)]


class Sparse24BothGemmArgs(ctypes.Structure):
    _fields_ = [("g", GemmArgs), ("a_values", _P), ("a_meta", _P), ("b_values", _P), ("b_meta", _P)]


class HpGemmArgs(ctypes.Structure):
    _fields_ = [("M", _I64), ("N", _I64), ("K", _I64), ("a", _P), ("lda", _I64), ("b", _P), ("ldb", _I64),
                ("ab_type", _I), ("a_scale", _P), ("a_kind", _I), ("b_scale", _P), ("b_kind", _I),
                ("c", _P), ("c_type", _I), ("ldc", _I64), ("tile_rows", _I)]


class ChainStage(ctypes.Structure):
    _fields_ = [("precision", _I), ("N", _I64), ("w", _P), ("w_scale", _P)]


class ChainStats(ctypes.Structure):
    _fields_ = [("makespan_ms", _D), ("stage_ms_mean", _D * 4), ("stage_ms_cv", _D * 4), ("stage_count", _I * 4),
                ("tflops", _D)]


class GroupProblem(ctypes.Structure):
    _fields_ = [("is_sparse", _I), ("dense", GemmArgs), ("sparse", Sparse24GemmArgs)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", _SZ), ("num_streams", _I), ("max_inflight", _I)]


class Request(ctypes.Structure):
    _fields_ = [("M", _I64), ("weight_id", _I), ("x", _P), ("c", _P), ("c_type", _I), ("x_fmt", _I),
                ("arrival_time_s", _D)]


class ServerStats(ctypes.Structure):
    _fields_ = [("p50_ms", _D), ("p99_ms", _D), ("mean_ms", _D), ("max_ms", _D), ("tflops", _D),
                ("span_s", _D), ("stream_cv", _D), ("fairness_range", _D), ("fairness_minmax", _D),
                ("done", ctypes.c_uint64), ("failed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("peak_inflight", ctypes.c_uint64), ("peak_bytes", _SZ)]


# Every exported entry point with its argument types (restype is fp8_status
# unless listed in _RESTYPE).
_SIGS = {
    "fp8_last_error": [],
    "fp8_version": [],
    "fp8_quantize_workspace_size": [_I64, _I64, _I, _P],
    "fp8_quantize": [_P, _I64, _I64, _I64, _I, _I, _P, _I64, _P, _P, _P, _SZ, _P],
    "fp8_tile_info": [_I, _P, _P, _P, _P, _P, _P],
    "fp8_num_tiles": [],
    "fp8_gemm_plan_resolve": [_P, _P, _P],
    "fp8_gemm_workspace_size": [_P, _P, _P],
    "fp8_gemm": [_P, _P, _P, _SZ, _P],
    "fp8_gemm_noalloc": [_P, _P, _P],
    "fp8_noalloc_scratch_bytes": [],
    "fp8_sparse24_prune_compress": [_P, _I, _I64, _I64, _I64, _P, _P, _P, _P],
    "fp8_sparse24_decompress": [_P, _P, _I64, _I64, _P, _I64, _P],
    "fp8_quantize_prune24": [_P, _I64, _I64, _I64, _I, _I, _P, _P, _P, _P, _P, _P, _SZ, _P],
    "fp8_sparse24_gemm_workspace_size": [_P, _P, _P],
    "fp8_sparse24_gemm": [_P, _P, _P, _SZ, _P],
    "fp8_tune_gemm": [_P, _I, _P, _P, _P],
    "fp8_tune_sparse24_gemm": [_P, _I, _P, _P, _P],
    "fp8_tune_cache_save": [ctypes.c_char_p],
    "fp8_tune_cache_load": [ctypes.c_char_p],
    "fp8_tune_cache_clear": [],
    "fp8_tune_sparse_vs_dense": [_P, _P, _I, _P, _P],
    "fp8_tune_breakeven_lookup": [_I64, _I64, _I64, _I, _I, _I, _I, _P, _P],
    "fp8_tune_breakeven_count": [],
    "fp8_tune_breakeven_get": [_I, _P],
    "fp8_tune_device_key": [_P, _SZ, _P],
    "fp8_grouped_tune": [_P, _I, _I, _P, _P, _P],
    "fp8_ubench_mfma": [_I, _I, _I, _I, _P, _P],
    "fp8_ubench_lds": [_I, _I, _P, _P],
    "fp8_ubench_lds_pattern": [_I, _I, _I, _P, _P],
    "fp8_ubench_lds_offsets": [_P, _I, _I, _I, _P, _P],
    "fp8_ubench_clock": [_I, _P, _P],
    "fp8_hp_gemm": [_P, _P],
    "fp8_chain_create": [_P, _I, _I64, _I64, _I, _I, _P],
    "fp8_chain_buffer": [_P, _I, _I, _P, _P],
    "fp8_chain_run": [_P, _I, _I, _P],
    "fp8_chain_stage_ms": [_P, _I, _I, _P],
    "fp8_chain_destroy": [_P],
    "fp8_sparse24_both_gemm_plan_resolve": [_P, _P, _P],
    "fp8_sparse24_both_gemm_workspace_size": [_P, _P, _P],
    "fp8_sparse24_both_gemm": [_P, _P, _P, _SZ, _P],
    "fp8_grouped_plan_create": [_P, _I, _I, _I, _P],
    "fp8_grouped_gemm": [_P, _P],
    "fp8_grouped_plan_info": [_P, _P, _P, _P],
    "fp8_grouped_plan_destroy": [_P],
    "fp8_server_create": [_P, _P],
    "fp8_server_create_simulated": [_P, _D, _D, _P],
    "fp8_server_register_weight": [_P, _P, _P, _P, _I64, _I64, _I, _P],
    "fp8_server_submit": [_P, _P, _P],
    "fp8_server_poll": [_P, ctypes.c_uint64],
    "fp8_server_wait": [_P, ctypes.c_uint64, _I64],
    "fp8_server_latency": [_P, ctypes.c_uint64, _P],
    "fp8_server_drain": [_P],
    "fp8_server_stats_get": [_P, _P],
    "fp8_server_reset_stats": [_P],
    "fp8_server_now": [_P],
    "fp8_server_destroy": [_P],
    "fp8_validate": [_P, _I, _I64, _P, _P, _I64, _I64, _I64, _P, _P],
}
_RESTYPE = {"fp8_last_error": ctypes.c_char_p, "fp8_version": _I, "fp8_num_tiles": _I,
            "fp8_noalloc_scratch_bytes": _SZ, "fp8_tune_breakeven_count": _I,
            "fp8_tune_cache_clear": None, "fp8_server_now": _D}

_lib = None


class Fp8Error(RuntimeError):
    def __init__(self, fn: str, status: int, text: str):
        name = STATUS[status] if 0 <= status < len(STATUS) else str(status)
        super().__init__(f"{fn}: {name}: {text}")
        self.status = status


def load() -> ctypes.CDLL:
    """Loads libfp8gemm.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run paper_2602_10262_amd/build.py (or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        if not hasattr(lib, name):
            continue
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = _RESTYPE.get(name, _I)
    _lib = lib
    return lib


def _check(fn: str, status: int) -> int:
    if status != FP8_OK:
        raise Fp8Error(fn, status, load().fp8_last_error().decode())
    return status


def _call(fn: str, *args) -> int:
    return _check(fn, getattr(load(), fn)(*args))


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream if hasattr(s, "cuda_stream") else int(s)


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _u8(t):
    import torch
    return t.view(torch.uint8) if t.dtype != torch.uint8 else t


def _out_type(dtype) -> int:
    import torch
    return {torch.bfloat16: FP8_OUT_BF16, torch.float16: FP8_OUT_F16}.get(dtype, FP8_OUT_F32)


# ---------------------------------------------------------------- quantize --

def fp8_quantize(x, fmt: int = FP8_E4M3, kind: int = FP8_SCALE_TENSOR, q=None, scale=None, descale=None,
                 ws=None, stream=None):
    """FP32 rows x cols (CUDA tensor, row-major) -> (codes uint8, s, d)."""
    import torch
    rows, cols = x.shape
    n = rows if kind == FP8_SCALE_ROW else 1
    q = torch.empty((rows, (cols + 15) // 16 * 16), dtype=torch.uint8, device=x.device)[:, :cols] if q is None else q
    scale = torch.empty(n, dtype=torch.float32, device=x.device) if scale is None else scale
    descale = torch.empty(n, dtype=torch.float32, device=x.device) if descale is None else descale
    if ws is None and kind == FP8_SCALE_TENSOR:
        ws = torch.empty(16, dtype=torch.uint8, device=x.device)
    _call("fp8_quantize", x.data_ptr(), rows, cols, x.stride(0), fmt, kind, q.data_ptr(), q.stride(0),
          scale.data_ptr(), descale.data_ptr(), _ptr(ws), 0 if ws is None else ws.numel() * ws.element_size(),
          _stream(stream))
    return q, scale, descale


# -------------------------------------------------------------------- gemm --

def gemm_args(a, b_nk, a_descale, b_descale, c, a_fmt=FP8_E4M3, b_fmt=FP8_E4M3, c_type=None,
              M=None, N=None, K=None) -> GemmArgs:
    import torch
    c_type = _out_type(c.dtype) if c_type is None else c_type
    M = M if M is not None else (a.shape[0] if a is not None else c.shape[0])
    N = N if N is not None else (b_nk.shape[0] if b_nk is not None else c.shape[1])
    K = K if K is not None else (a.shape[1] if a is not None else b_nk.shape[1])
    return GemmArgs(M, N, K,
                    _ptr(a), a_fmt, a.stride(0) if a is not None else K,
                    _ptr(b_nk), b_fmt, b_nk.stride(0) if b_nk is not None else K,
                    a_descale.data_ptr(), FP8_SCALE_ROW if a_descale.numel() > 1 else FP8_SCALE_TENSOR,
                    b_descale.data_ptr(), FP8_SCALE_ROW if b_descale.numel() > 1 else FP8_SCALE_TENSOR,
                    c.data_ptr(), c_type, c.stride(0))


def _plan(plan):
    if plan is None:
        return None
    if isinstance(plan, Plan):
        return ctypes.byref(plan)
    tile, split = plan
    return ctypes.byref(Plan(tile, split))


def _workspace(size_fn, args_ref, plan_ref, device):
    import torch
    nbytes = ctypes.c_size_t(0)
    _call(size_fn, args_ref, plan_ref, ctypes.byref(nbytes))
    if nbytes.value == 0:
        return None, 0
    return torch.empty(nbytes.value, dtype=torch.uint8, device=device), nbytes.value


def fp8_gemm(a, b_nk, a_descale, b_descale, a_fmt=FP8_E4M3, b_fmt=FP8_E4M3, out_dtype=None, c=None,
             plan=None, ws=None, stream=None):
    """C (M x N) = diag(d_a) dec(A) dec(B) diag(d_b); A: M x K codes, B given as N x K codes."""
    import torch
    if c is None:
        c = torch.empty((a.shape[0], b_nk.shape[0]), dtype=out_dtype or torch.float32, device=a.device)
    args = gemm_args(_u8(a), _u8(b_nk), a_descale, b_descale, c, a_fmt, b_fmt)
    pref = _plan(plan)
    if ws is None:
        ws, nbytes = _workspace("fp8_gemm_workspace_size", ctypes.byref(args), pref, a.device)
    else:
        nbytes = ws.numel() * ws.element_size()
    _call("fp8_gemm", ctypes.byref(args), pref, _ptr(ws), nbytes, _stream(stream))
    return c


def fp8_gemm_noalloc(a, b_nk, a_descale, b_descale, a_fmt=FP8_E4M3, b_fmt=FP8_E4M3, out_dtype=None, c=None,
                     plan=None, stream=None):
    """fp8_gemm whose split-K partial sums use the library's fixed device
    scratch array: the call itself allocates nothing (c must be given for
    that; otherwise torch allocates it here)."""
    import torch
    if c is None:
        c = torch.empty((a.shape[0], b_nk.shape[0]), dtype=out_dtype or torch.float32, device=a.device)
    args = gemm_args(_u8(a), _u8(b_nk), a_descale, b_descale, c, a_fmt, b_fmt)
    _call("fp8_gemm_noalloc", ctypes.byref(args), _plan(plan), _stream(stream))
    return c


def fp8_noalloc_scratch_bytes() -> int:
    return int(load().fp8_noalloc_scratch_bytes())


def fp8_gemm_plan_resolve(args: GemmArgs, plan=None) -> tuple:
    out = Plan(0, 0)
    _call("fp8_gemm_plan_resolve", ctypes.byref(args), _plan(plan), ctypes.byref(out))
    return out.tile, out.split_k


def fp8_tile_info(tile: int) -> dict:
    v = [ctypes.c_int(0) for _ in range(6)]
    _call("fp8_tile_info", tile, *[ctypes.byref(x) for x in v])
    return {"block_m": v[0].value, "block_n": v[1].value, "waves": v[2].value, "sparse": v[3].value,
            "dense": v[4].value, "exact": v[5].value}


def fp8_num_tiles() -> int:
    return load().fp8_num_tiles()


# ------------------------------------------------------------------- 2:4 ----

def fp8_sparse24_prune_compress(x, fmt=FP8_E4M3, with_mask=True, stream=None):
    """Row-major rows x K codes -> (values rows x K/2, meta rows x K/8, mask rows x K/8 or None)."""
    import torch
    rows, K = x.shape
    values = torch.empty((rows, K // 2), dtype=torch.uint8, device=x.device)
    meta = torch.empty((rows, K // 8), dtype=torch.uint8, device=x.device)
    mask = torch.empty((rows, K // 8), dtype=torch.uint8, device=x.device) if with_mask else None
    _call("fp8_sparse24_prune_compress", _u8(x).data_ptr(), fmt, rows, K, x.stride(0), values.data_ptr(),
          meta.data_ptr(), _ptr(mask), _stream(stream))
    return values, meta, mask


def fp8_quantize_prune24(x, fmt=FP8_E4M3, kind=FP8_SCALE_ROW, with_mask=True, ws=None, stream=None):
    """FP32 rows x K (CUDA tensor, row-major) -> (values, meta, mask or None, s, d) in one pass."""
    import torch
    rows, K = x.shape
    n = rows if kind == FP8_SCALE_ROW else 1
    values = torch.empty((rows, K // 2), dtype=torch.uint8, device=x.device)
    meta = torch.empty((rows, K // 8), dtype=torch.uint8, device=x.device)
    mask = torch.empty((rows, K // 8), dtype=torch.uint8, device=x.device) if with_mask else None
    scale = torch.empty(n, dtype=torch.float32, device=x.device)
    descale = torch.empty(n, dtype=torch.float32, device=x.device)
    if ws is None and kind == FP8_SCALE_TENSOR:
        ws = torch.empty(16, dtype=torch.uint8, device=x.device)
    _call("fp8_quantize_prune24", x.data_ptr(), rows, K, x.stride(0), fmt, kind, values.data_ptr(), meta.data_ptr(),
          _ptr(mask), scale.data_ptr(), descale.data_ptr(), _ptr(ws),
          0 if ws is None else ws.numel() * ws.element_size(), _stream(stream))
    return values, meta, mask, scale, descale


def fp8_sparse24_decompress(values, meta, K, out=None, stream=None):
    import torch
    rows = values.shape[0]
    out = torch.empty((rows, K), dtype=torch.uint8, device=values.device) if out is None else out
    _call("fp8_sparse24_decompress", values.data_ptr(), meta.data_ptr(), rows, K, out.data_ptr(), out.stride(0),
          _stream(stream))
    return out


def sparse24_args(values, meta, dense, side, a_descale, b_descale, c, sparse_fmt=FP8_E4M3, dense_fmt=FP8_E4M3,
                  M=None, N=None, K=None):
    K = K if K is not None else values.shape[1] * 2
    if side == FP8_SPARSE_A:
        M = values.shape[0] if M is None else M
        N = dense.shape[0] if N is None else N
        g = gemm_args(None, _u8(dense), a_descale, b_descale, c, sparse_fmt, dense_fmt, M=M, N=N, K=K)
    else:
        M = dense.shape[0] if M is None else M
        N = values.shape[0] if N is None else N
        g = gemm_args(_u8(dense), None, a_descale, b_descale, c, dense_fmt, sparse_fmt, M=M, N=N, K=K)
    return Sparse24GemmArgs(g, side, values.data_ptr(), meta.data_ptr())


def fp8_sparse24_gemm(values, meta, dense, side, a_descale, b_descale, sparse_fmt=FP8_E4M3, dense_fmt=FP8_E4M3,
                      out_dtype=None, c=None, plan=None, ws=None, stream=None):
    """side A: C = A'(values, meta) x B, dense = B as N x K codes.
    side B: C = A x B', dense = A (M x K codes), (values, meta) = compressed N x K weight."""
    import torch
    K = values.shape[1] * 2
    M = values.shape[0] if side == FP8_SPARSE_A else dense.shape[0]
    N = dense.shape[0] if side == FP8_SPARSE_A else values.shape[0]
    if c is None:
        c = torch.empty((M, N), dtype=out_dtype or torch.float32, device=values.device)
    args = sparse24_args(values, meta, dense, side, a_descale, b_descale, c, sparse_fmt, dense_fmt, M, N, K)
    pref = _plan(plan)
    if ws is None:
        ws, nbytes = _workspace("fp8_sparse24_gemm_workspace_size", ctypes.byref(args), pref, values.device)
    else:
        nbytes = ws.numel() * ws.element_size()
    _call("fp8_sparse24_gemm", ctypes.byref(args), pref, _ptr(ws), nbytes, _stream(stream))
    return c


def sparse24_both_args(a_values, a_meta, b_values, b_meta, a_descale, b_descale, c, a_fmt=FP8_E4M3,
                       b_fmt=FP8_E4M3):
    M, N, K = a_values.shape[0], b_values.shape[0], a_values.shape[1] * 2
    g = gemm_args(None, None, a_descale, b_descale, c, a_fmt, b_fmt, M=M, N=N, K=K)
    return Sparse24BothGemmArgs(g, a_values.data_ptr(), a_meta.data_ptr(), b_values.data_ptr(), b_meta.data_ptr())


def fp8_sparse24_both_gemm(a_values, a_meta, b_values, b_meta, a_descale, b_descale, a_fmt=FP8_E4M3,
                           b_fmt=FP8_E4M3, out_dtype=None, c=None, plan=None, ws=None, stream=None):
    """C = A' x W'^T with both operands given compressed: (a_values, a_meta) the
    M x K activations, (b_values, b_meta) the N x K weight rows."""
    import torch
    M, N = a_values.shape[0], b_values.shape[0]
    if c is None:
        c = torch.empty((M, N), dtype=out_dtype or torch.float32, device=a_values.device)
    args = sparse24_both_args(a_values, a_meta, b_values, b_meta, a_descale, b_descale, c, a_fmt, b_fmt)
    pref = _plan(plan)
    if ws is None:
        ws, nbytes = _workspace("fp8_sparse24_both_gemm_workspace_size", ctypes.byref(args), pref, a_values.device)
    else:
        nbytes = ws.numel() * ws.element_size()
    _call("fp8_sparse24_both_gemm", ctypes.byref(args), pref, _ptr(ws), nbytes, _stream(stream))
    return c


def fp8_sparse24_both_gemm_plan_resolve(args, plan=None):
    res = Plan(0, 0)
    _call("fp8_sparse24_both_gemm_plan_resolve", ctypes.byref(args), _plan(plan), ctypes.byref(res))
    return res.tile, res.split_k


# ------------------------------------------------ higher-precision GEMM ----

def fp8_hp_gemm(a, b_nk, a_scale=None, b_scale=None, out_dtype=None, c=None, stream=None, tile_rows=0):
    """C = diag(s_a) A B diag(s_b) for FP32, FP16 or BF16 tensors A (M x K) and
    B given as N x K rows; scales: None (1), one float or M / N floats."""
    import torch
    types = {torch.float32: FP8_HP_F32, torch.float16: FP8_HP_F16, torch.bfloat16: FP8_HP_BF16}
    if a.dtype != b_nk.dtype or a.dtype not in types:
        raise ValueError("A and B must share one of float32, float16, bfloat16")
    M, K = a.shape
    N = b_nk.shape[0]
    one = None
    if a_scale is None or b_scale is None:
        one = torch.ones(1, dtype=torch.float32, device=a.device)
    a_scale = one if a_scale is None else a_scale
    b_scale = one if b_scale is None else b_scale
    if c is None:
        c = torch.empty((M, N), dtype=out_dtype or torch.float32, device=a.device)
    args = HpGemmArgs(M, N, K, a.data_ptr(), a.stride(0), b_nk.data_ptr(), b_nk.stride(0), types[a.dtype],
                      a_scale.data_ptr(), FP8_SCALE_ROW if a_scale.numel() > 1 else FP8_SCALE_TENSOR,
                      b_scale.data_ptr(), FP8_SCALE_ROW if b_scale.numel() > 1 else FP8_SCALE_TENSOR,
                      c.data_ptr(), _out_type(c.dtype), c.stride(0), tile_rows)
    _call("fp8_hp_gemm", ctypes.byref(args), _stream(stream))
    return c


class Chain:
    """Mixed-precision GEMM chains (fp8_chain_*): stages = [(precision, weight
    tensor N x K, w_scale tensor or None)], M rows, in_width columns of input."""

    def __init__(self, stages, M: int, in_width: int, n_chains: int, max_streams: int = 4):
        if any(not w.is_contiguous() for _, w, _ in stages):
            raise ValueError("chain weights must be contiguous N x K tensors")
        self._keep = [(w, sc) for _, w, sc in stages]
        arr = (ChainStage * len(stages))(*[ChainStage(p, w.shape[0], w.data_ptr(), _ptr(sc)) for p, w, sc in stages])
        self.stages = stages
        self.n_chains = n_chains
        self.M = M
        self._h = ctypes.c_void_p()
        _call("fp8_chain_create", arr, len(stages), M, in_width, n_chains, max_streams, ctypes.byref(self._h))

    def buffer(self, chain: int, stage: int):
        """(device pointer, leading dimension) of a stage's input (stage =
        len(stages): the FP32 output)."""
        ptr = ctypes.c_void_p()
        ld = ctypes.c_int64()
        _call("fp8_chain_buffer", self._h, chain, stage, ctypes.byref(ptr), ctypes.byref(ld))
        return ptr.value, ld.value

    def run(self, schedule: int, n_streams: int = 1) -> dict:
        st = ChainStats()
        _call("fp8_chain_run", self._h, schedule, n_streams, ctypes.byref(st))
        names = ("f32", "f16", "bf16", "fp8")
        return {"makespan_ms": st.makespan_ms, "tflops": st.tflops,
                "stage_ms_mean": {names[p]: st.stage_ms_mean[p] for p in range(4) if st.stage_count[p]},
                "stage_ms_cv": {names[p]: st.stage_ms_cv[p] for p in range(4) if st.stage_count[p]},
                "stage_count": {names[p]: st.stage_count[p] for p in range(4) if st.stage_count[p]}}

    def tensor(self, chain: int, stage: int):
        """A torch view (no copy) of a stage's input buffer (stage =
        len(stages): the FP32 output), through the CUDA array interface."""
        import torch
        ptr, ld = self.buffer(chain, stage)
        if stage == len(self.stages):
            typestr, dtype = "<f4", torch.float32
        else:
            prec = self.stages[stage][0]
            typestr, dtype = {FP8_STAGE_F32: ("<f4", torch.float32), FP8_STAGE_FP8: ("<f4", torch.float32),
                              FP8_STAGE_F16: ("<f2", torch.float16), FP8_STAGE_BF16: ("<i2", torch.bfloat16)}[prec]

        class _View:
            __cuda_array_interface__ = {"shape": (self.M, ld), "typestr": typestr, "data": (ptr, False),
                                        "version": 2, "strides": None}
        t = torch.as_tensor(_View(), device="cuda")
        return t.view(dtype) if dtype == torch.bfloat16 else t

    def stage_ms(self, chain: int, stage: int) -> float:
        ms = ctypes.c_double()
        _call("fp8_chain_stage_ms", self._h, chain, stage, ctypes.byref(ms))
        return ms.value

    def close(self):
        if self._h:
            _call("fp8_chain_destroy", self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- tuning ---

def fp8_tune_gemm(args: GemmArgs, iters: int = 10, stream=None):
    best = Plan(0, 0)
    us = ctypes.c_double(0)
    _call("fp8_tune_gemm", ctypes.byref(args), iters, _stream(stream), ctypes.byref(best), ctypes.byref(us))
    return (best.tile, best.split_k), us.value


def fp8_tune_sparse24_gemm(args: Sparse24GemmArgs, iters: int = 10, stream=None):
    best = Plan(0, 0)
    us = ctypes.c_double(0)
    _call("fp8_tune_sparse24_gemm", ctypes.byref(args), iters, _stream(stream), ctypes.byref(best),
          ctypes.byref(us))
    return (best.tile, best.split_k), us.value


class Breakeven(ctypes.Structure):
    _fields_ = [("M", _I64), ("N", _I64), ("K", _I64), ("side", _I), ("a_fmt", _I), ("b_fmt", _I), ("c_type", _I),
                ("dense_us", _D), ("sparse_us", _D), ("dense_plan", Plan), ("sparse_plan", Plan),
                ("use_sparse", _I)]

    def as_dict(self) -> dict:
        return {"M": self.M, "N": self.N, "K": self.K, "side": "A" if self.side == FP8_SPARSE_A else "B",
                "a_fmt": self.a_fmt, "b_fmt": self.b_fmt, "c_type": self.c_type,
                "dense_us": self.dense_us, "sparse_us": self.sparse_us,
                "dense_plan": [self.dense_plan.tile, self.dense_plan.split_k],
                "sparse_plan": [self.sparse_plan.tile, self.sparse_plan.split_k],
                "use_sparse": bool(self.use_sparse), "speedup_2to4": self.dense_us / self.sparse_us}


def fp8_tune_sparse_vs_dense(sparse_args: Sparse24GemmArgs, dense_args: GemmArgs, iters: int = 10,
                             stream=None) -> dict:
    r = Breakeven()
    _call("fp8_tune_sparse_vs_dense", ctypes.byref(sparse_args), ctypes.byref(dense_args), iters, _stream(stream),
          ctypes.byref(r))
    return r.as_dict()


def fp8_tune_breakeven_records() -> list:
    L = load()
    out = []
    for i in range(L.fp8_tune_breakeven_count()):
        r = Breakeven()
        _call("fp8_tune_breakeven_get", i, ctypes.byref(r))
        out.append(r.as_dict())
    return out


def fp8_tune_breakeven_lookup(M, N, K, side, a_fmt=FP8_E4M3, b_fmt=FP8_E4M3, c_type=FP8_OUT_BF16):
    r = Breakeven()
    found = ctypes.c_int(0)
    _call("fp8_tune_breakeven_lookup", M, N, K, side, a_fmt, b_fmt, c_type, ctypes.byref(r), ctypes.byref(found))
    return r.as_dict() if found.value else None


def fp8_tune_device_key() -> tuple:
    buf = ctypes.create_string_buffer(256)
    rt = ctypes.c_int(0)
    _call("fp8_tune_device_key", buf, 256, ctypes.byref(rt))
    return buf.value.decode(), rt.value


def fp8_tune_cache_save(path: str):
    _call("fp8_tune_cache_save", path.encode())


def fp8_tune_cache_load(path: str):
    _call("fp8_tune_cache_load", path.encode())


def fp8_tune_cache_clear():
    load().fp8_tune_cache_clear()


# ---------------------------------------------------------- microbenchmarks --

UBENCH_KINDS = {0: ("mfma_16x16x128_f8", 16 * 16 * 128), 1: ("mfma_32x32x64_f8", 32 * 32 * 64),
                2: ("smfmac_16x16x128_f8", 16 * 16 * 128), 3: ("smfmac_32x32x64_f8", 32 * 32 * 64)}


def fp8_ubench_mfma(kind: int, waves_per_cu: int, chains: int, iters: int, stream=None) -> float:
    """Device milliseconds of one microbenchmark launch (see the C header)."""
    ms = ctypes.c_double(0)
    _call("fp8_ubench_mfma", kind, waves_per_cu, chains, iters, _stream(stream), ctypes.byref(ms))
    return ms.value


def fp8_ubench_lds(waves_per_cu: int, iters: int, stream=None) -> float:
    ms = ctypes.c_double(0)
    _call("fp8_ubench_lds", waves_per_cu, iters, _stream(stream), ctypes.byref(ms))
    return ms.value


LDS_PATTERNS = {0: "linear", 1: "dense_fragment", 2: "compressed_fragment", 3: "2to4_b_operand",
                4: "metadata_b32", 5: "compressed_unswizzled", 6: "metadata_pair_read2st64",
                7: "2to4_b_chunks_on_dense_swizzle"}


def fp8_ubench_lds_pattern(pattern: int, waves_per_cu: int, iters: int, stream=None) -> float:
    ms = ctypes.c_double(0)
    _call("fp8_ubench_lds_pattern", pattern, waves_per_cu, iters, _stream(stream), ctypes.byref(ms))
    return ms.value


def fp8_ubench_clock(iters: int = 20000, stream=None) -> float:
    """Engine clock (GHz) under 16x16x128 FP8 MFMA load."""
    ghz = ctypes.c_double(0)
    _call("fp8_ubench_clock", iters, _stream(stream), ctypes.byref(ghz))
    return ghz.value


def fp8_ubench_lds_offsets(lane_offsets, waves_per_cu: int, iters: int, stream=None, write: bool = False) -> float:
    arr = (ctypes.c_int * 64)(*[int(o) for o in lane_offsets])
    ms = ctypes.c_double(0)
    _call("fp8_ubench_lds_offsets", arr, int(write), waves_per_cu, iters, _stream(stream), ctypes.byref(ms))
    return ms.value


# -------------------------------------------------------------- validate ----

def fp8_validate(c, cref, sabs, K, stream=None) -> dict:
    """FP64 error norms of c against FP64 references held on the device."""
    import torch
    M, N = c.shape
    out = torch.empty(5, dtype=torch.float64, device=c.device)
    c_type = _out_type(c.dtype)
    _call("fp8_validate", c.data_ptr(), c_type, c.stride(0), cref.data_ptr(), sabs.data_ptr(), M, N, K,
          out.data_ptr(), _stream(stream))
    o = out.cpu().tolist()
    return {"max_abs_err": o[0], "max_ratio": o[1], "normwise": (o[2] / o[3]) ** 0.5 if o[3] > 0 else o[2] ** 0.5,
            "over": int(o[4]), "ok": o[4] == 0}


# ----------------------------------------------------------------- grouped --

def fp8_grouped_tune(problems, iters: int = 5, stream=None) -> tuple:
    """(fastest grouped tile, its median microseconds) for these problems."""
    arr = (GroupProblem * len(problems))(*problems)
    t = ctypes.c_int(-1)
    us = ctypes.c_double(0)
    _call("fp8_grouped_tune", ctypes.cast(arr, _P), len(problems), iters, _stream(stream), ctypes.byref(t),
          ctypes.byref(us))
    return t.value, us.value


class GroupedPlan:
    """Owns an fp8_grouped_plan; problems' buffers must outlive it."""

    def __init__(self, problems, tile: int = -1, use_graph: bool = False):
        arr = (GroupProblem * len(problems))(*problems)
        self._h = ctypes.c_void_p(0)
        _call("fp8_grouped_plan_create", ctypes.cast(arr, _P), len(problems), tile, int(use_graph),
              ctypes.byref(self._h))
        self._keep = problems

    def run(self, stream=None):
        _call("fp8_grouped_gemm", self._h, _stream(stream))

    def info(self) -> dict:
        t, n, g = ctypes.c_int(0), ctypes.c_int64(0), ctypes.c_int(0)
        _call("fp8_grouped_plan_info", self._h, ctypes.byref(t), ctypes.byref(n), ctypes.byref(g))
        return {"tile": t.value, "tiles": n.value, "workgroups": g.value}

    def close(self):
        if self._h:
            load().fp8_grouped_plan_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dense_problem(a, w_nk, a_descale, w_descale, c, a_fmt=FP8_E4M3, w_fmt=FP8_E4M3) -> GroupProblem:
    g = gemm_args(_u8(a), _u8(w_nk), a_descale, w_descale, c, a_fmt, w_fmt)
    return GroupProblem(0, g, Sparse24GemmArgs())


def sparse_weight_problem(a, w_values, w_meta, a_descale, w_descale, c, a_fmt=FP8_E4M3, w_fmt=FP8_E4M3):
    sa = sparse24_args(w_values, w_meta, _u8(a), FP8_SPARSE_B, a_descale, w_descale, c, w_fmt, a_fmt)
    return GroupProblem(1, GemmArgs(), sa)


# ------------------------------------------------------------------ server --

class Server:
    """Owns an fp8_server (HIP streams + scheduler thread, or simulated)."""

    def __init__(self, hbm_budget_bytes: int, num_streams: int = 4, max_inflight: int = 0,
                 simulated: bool = False, gflop_per_ms: float = 1000.0, launch_us: float = 10.0):
        cfg = ServerConfig(hbm_budget_bytes, num_streams, max_inflight)
        self._h = ctypes.c_void_p(0)
        if simulated:
            _call("fp8_server_create_simulated", ctypes.byref(cfg), gflop_per_ms, launch_us, ctypes.byref(self._h))
        else:
            _call("fp8_server_create", ctypes.byref(cfg), ctypes.byref(self._h))

    def register_weight(self, w, meta, w_descale, N: int, K: int, fmt: int = FP8_E4M3) -> int:
        wid = ctypes.c_int(0)
        _call("fp8_server_register_weight", self._h, _ptr(w), _ptr(meta), _ptr(w_descale), N, K, fmt,
              ctypes.byref(wid))
        return wid.value

    def submit(self, M: int, weight_id: int, x=None, c=None, c_type: int = FP8_OUT_BF16,
               x_fmt: int = FP8_E4M3, arrival_time_s: float = -1.0, x_ptr: int | None = None,
               c_ptr: int | None = None) -> int:
        req = Request(M, weight_id, x_ptr if x_ptr is not None else _ptr(x),
                      c_ptr if c_ptr is not None else _ptr(c), c_type, x_fmt, arrival_time_s)
        t = ctypes.c_uint64(0)
        _call("fp8_server_submit", self._h, ctypes.byref(req), ctypes.byref(t))
        return t.value

    def poll(self, ticket: int) -> int:
        return load().fp8_server_poll(self._h, ticket)

    def wait(self, ticket: int, timeout_us: int = -1) -> int:
        st = load().fp8_server_wait(self._h, ticket, timeout_us)
        if st not in (FP8_OK, FP8_ERR_TIMEOUT):
            _check("fp8_server_wait", st)
        return st

    def latency_ms(self, ticket: int) -> float:
        v = ctypes.c_double(0)
        _call("fp8_server_latency", self._h, ticket, ctypes.byref(v))
        return v.value

    def drain(self):
        _call("fp8_server_drain", self._h)

    def stats(self) -> dict:
        st = ServerStats()
        _call("fp8_server_stats_get", self._h, ctypes.byref(st))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def reset_stats(self):
        _call("fp8_server_reset_stats", self._h)

    def now(self) -> float:
        return load().fp8_server_now(self._h)

    def close(self):
        if self._h:
            load().fp8_server_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
