"""Builds libfp8gemm.so for gfx950 in-tree with hipcc.

Every source under csrc/ is compiled to an object under _build/ (in
parallel), then linked into paper_2602_10262_amd/libfp8gemm.so.  All HIP
code is built with packed FP32 instructions disabled (-packed-fp32-ops).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfp8gemm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# The GEMM tile table is instantiated over several files so that it compiles in
# parallel; the slowest files come first.
SOURCES = ["gemm_tiles_b.hip", "gemm_tiles_c.hip", "gemm_tiles_d.hip", "gemm_tiles_e.hip", "gemm_tiles_f.hip",
           "gemm_tiles_g.hip", "gemm_tiles_h.hip", "gemm_tiles_i.hip", "gemm_tiles_j.hip", "gemm_tiles_k.hip", "gemm_tiles_a.hip", "gemm_both_a.hip", "gemm_both_b.hip", "grouped_tiles_a.hip", "grouped_tiles_b.hip",
           "grouped_tiles_c.hip", "grouped_tiles_d.hip", "grouped.hip", "gemm.hip", "quantize.hip", "quantize_prune.hip", "sparse24.hip", "validate.hip",
           "noalloc.hip", "ubench.hip", "gemm_hp.hip", "api.cpp", "tune.cpp", "server.cpp", "chain.cpp"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _stale(src: str, out: str) -> bool:
    if not os.path.exists(out):
        return True
    t = os.path.getmtime(out)
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".hpp")]
    deps.append(os.path.join(os.path.dirname(HERE), "include", "fp8gemm.h"))
    return any(os.path.getmtime(d) > t for d in deps if os.path.exists(d))


def _compile(src: str, force: bool = True) -> str:
    out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    if not force and not _stale(src, out):
        return out
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return out


def build(jobs: int | None = None, verbose: bool = True, force: bool = True) -> str:
    """Compiles every source (force) or only those older than their inputs."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(len(srcs), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda x: _compile(x, force), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(force="--incremental" not in sys.argv)
