"""The C ABI: the library loads without a GPU and exports every entry point
include/fp8gemm.h declares; argument errors come back as status codes."""
import ctypes
import os
import re

import pytest

import paper_2602_10262_amd as lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fp8gemm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(fp8_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ["fp8_gemm", "fp8_sparse24_prune_compress", "fp8_sparse24_gemm", "fp8_grouped_gemm",
                     "fp8_server_create", "fp8_server_submit", "fp8_quantize"]:
        assert required in names
    assert len(names) >= 30


def test_library_exports_every_declared_symbol():
    L = lib.load()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(declared_functions()) <= set(lib._SIGS), "binding lacks a declared entry point"


def test_argument_errors_are_status_codes_without_gpu():
    L = lib.load()
    args = lib.GemmArgs()
    assert L.fp8_gemm(ctypes.byref(args), None, None, 0, None) == 2  # FP8_ERR_SHAPE: M = 0
    args.M = args.N = args.K = 16
    args.a_descale = args.b_descale = args.c = 256
    args.ldc = 16
    assert L.fp8_gemm(ctypes.byref(args), None, None, 0, None) == 1  # FP8_ERR_ARG: null A
    assert b"null A" in L.fp8_last_error()
    args.a = args.b = 4096 + 8         # misaligned
    args.lda = args.ldb = 16
    assert L.fp8_gemm(ctypes.byref(args), None, None, 0, None) == 3  # FP8_ERR_ALIGN
    assert L.fp8_sparse24_prune_compress(4096, 0, 4, 12, 16, 4096, 4096, None, None) == 2  # K % 8
    n = ctypes.c_size_t(0)
    assert L.fp8_quantize_workspace_size(8, 8, 0, ctypes.byref(n)) == 0 and n.value == 4


def test_plan_resolution_and_workspace_on_host():
    L = lib.load()
    args = lib.GemmArgs(16, 8192, 8192, 4096, 0, 8192, 4096, 0, 8192, 256, 1, 256, 1, 256, 1, 8192)
    tile, split = lib.fp8_gemm_plan_resolve(args)
    assert 0 <= tile < lib.fp8_num_tiles() and split >= 1
    info = lib.fp8_tile_info(tile)
    assert info["block_m"] >= 16
    nbytes = ctypes.c_size_t(0)
    assert L.fp8_gemm_workspace_size(ctypes.byref(args), None, ctypes.byref(nbytes)) == 0
    assert nbytes.value == (split * 16 * 8192 * 4 if split > 1 else 0)
    # explicit plan is honoured
    assert lib.fp8_gemm_plan_resolve(args, (0, 3)) == (0, 3)
    with pytest.raises(lib.Fp8Error):
        lib.fp8_gemm_plan_resolve(args, (999, 1))


def test_gpu_tests_cover_every_tile():
    from tests.test_gpu_gemm import NUM_TILES
    assert lib.fp8_num_tiles() == NUM_TILES
    for t in range(NUM_TILES):
        info = lib.fp8_tile_info(t)
        assert info["block_m"] % 16 == 0 and info["block_n"] % 16 == 0


def test_tuning_cache_roundtrip(tmp_path):
    """Plans and dense-vs-2:4 records persist as JSON lines keyed by the
    device and runtime they were measured on; other devices' lines are
    skipped on load."""
    import json
    lib.fp8_tune_cache_clear()
    dev, rt = lib.fp8_tune_device_key()
    plan = {"kind": "plan", "device": dev, "runtime": rt, "mk": 8192, "nk": 8192, "kk": 8192, "fa": 0, "fb": 0,
            "out_type": 1, "si_per": 1, "sj_per": 1, "sparse": 0, "tile": 3, "split_k": 2, "us": 123.0}
    be = {"kind": "breakeven", "device": dev, "runtime": rt, "M": 16, "N": 8192, "K": 8192, "side": 1, "fa": 0,
          "fb": 0, "c_type": 1, "dense_us": 20.0, "sparse_us": 15.0, "dense_tile": 24, "dense_split": 1,
          "sparse_tile": 4, "sparse_split": 4, "use_sparse": 1}
    other = dict(plan, device="gfx000 elsewhere", tile=5)
    p = tmp_path / "cache.jsonl"
    p.write_text("\n".join(json.dumps(x) for x in (other, plan, be)) + "\n")
    lib.fp8_tune_cache_load(str(p))
    args = lib.GemmArgs(8192, 8192, 8192, 4096, 0, 8192, 4096, 0, 8192, 256, 1, 256, 1, 256, 1, 8192)
    assert lib.fp8_gemm_plan_resolve(args) == (3, 2)
    rec = lib.fp8_tune_breakeven_lookup(9, 8192, 8192, lib.FP8_SPARSE_B)   # M rounds up to 16
    assert rec and rec["use_sparse"] and rec["sparse_plan"] == [4, 4] and rec["speedup_2to4"] == 20.0 / 15.0
    assert lib.fp8_tune_breakeven_lookup(9, 8192, 8192, lib.FP8_SPARSE_A) is None
    out = tmp_path / "out.jsonl"
    lib.fp8_tune_cache_save(str(out))
    lines = [json.loads(x) for x in out.read_text().splitlines()]
    assert {x["kind"] for x in lines} == {"plan", "breakeven"}
    assert all(x["device"] == dev and x["runtime"] == rt for x in lines)
    assert not any(x.get("tile") == 5 for x in lines)
    lib.fp8_tune_cache_clear()
    assert lib.fp8_gemm_plan_resolve(args) != (3, 2)
    assert lib.fp8_tune_breakeven_records() == []
    lib.fp8_tune_cache_load(str(out))
    assert lib.fp8_gemm_plan_resolve(args) == (3, 2) and len(lib.fp8_tune_breakeven_records()) == 1
    lib.fp8_tune_cache_clear()


def test_noalloc_entry_point_without_gpu():
    L = lib.load()
    assert L.fp8_noalloc_scratch_bytes() == 32 << 20
    args = lib.GemmArgs()
    assert L.fp8_gemm_noalloc(ctypes.byref(args), None, None) == 2  # FP8_ERR_SHAPE: M = 0


def test_ctypes_structs_match_the_c_header(tmp_path):
    """Every ctypes mirror of a header struct has the C layout: size and the
    offset of each field, from a C program compiled against the header."""
    import ctypes
    import subprocess
    import paper_2602_10262_amd as lib
    pairs = {
        "fp8_gemm_args": lib.GemmArgs, "fp8_plan": lib.Plan, "fp8_sparse24_gemm_args": lib.Sparse24GemmArgs,
        "fp8_sparse24_both_gemm_args": lib.Sparse24BothGemmArgs, "fp8_hp_gemm_args": lib.HpGemmArgs,
        "fp8_chain_stage": lib.ChainStage, "fp8_chain_stats": lib.ChainStats,
        "fp8_group_problem": lib.GroupProblem, "fp8_server_config": lib.ServerConfig,
        "fp8_request": lib.Request, "fp8_server_stats": lib.ServerStats, "fp8_breakeven": lib.Breakeven,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{os.path.join(ROOT, "include", "fp8gemm.h")}"',
             "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(src)], check=True)
    got = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    c = {}
    for line in got:
        if line:
            name, field, val = line.split()
            c[(name, field)] = int(val)
    for cname, py in pairs.items():
        assert c[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert c[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
