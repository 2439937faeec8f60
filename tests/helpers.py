"""Shared helpers of the GPU tests: seeded inputs, device transfer, oracle
comparison of GEMM results."""
from __future__ import annotations

import sys

import numpy as np

import oracle as orc
from paper_2602_10262_amd import synth


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t) -> np.ndarray:
    import torch
    if t.dtype == torch.bfloat16:
        return orc.bf16_to_f64(t.view(torch.int16).cpu().numpy().view(np.uint16))
    return t.cpu().numpy()


def codes_with_pad(rows: int, K: int, data: np.ndarray):
    """A CUDA uint8 tensor with a 16-byte-multiple row stride holding data."""
    import torch
    ld = (K + 15) // 16 * 16
    t = torch.zeros((rows, ld), dtype=torch.uint8, device="cuda")
    t[:, :K] = torch.from_numpy(np.ascontiguousarray(data)).cuda()
    return t[:, :K]


def operands(M: int, N: int, K: int, seed: int, dist: str, fa: int, fb: int, per_row: bool):
    """Quantized operands drawn on the host through the oracle: (qa, da, qb, db)."""
    if dist == "uniform":
        xa = synth.uniform(seed, 1, (M, K))
        xb = synth.uniform(seed, 2, (N, K))
    else:
        xa = synth.normal_outliers(seed * 2 + 1, (M, K))
        xb = synth.normal_outliers(seed * 2 + 2, (N, K))
    qa, _, da = orc.quantize(xa, fa, per_row)
    qb, _, db = orc.quantize(xb, fb, per_row)
    return qa, da, qb, db


def check_gemm(c_dev, qa, fa, qb, fb, da, db, out_bf16: bool, what: str = "") -> dict:
    cref, sabs = orc.gemm(qa, fa, qb, fb, da, db)
    res = orc.check(host(c_dev), cref, sabs, qa.shape[1], orc.OUT_BF16 if out_bf16 else orc.OUT_F32)
    log(f"  {what} max_err={res['max_abs_err']:.3e} max_ratio={res['max_ratio']:.3e} normwise={res['normwise']:.3e}")
    assert res["ok"], (what, res)
    return res


def check_gemm_sampled(c_dev, qa, fa, qb, fb, da, db, out_bf16: bool, n: int = 4096, seed: int = 0,
                       what: str = "") -> dict:
    """Full-size results checked on sampled outputs (plus the four corners and
    a full first/last row and column) that the oracle computes one by one."""
    M, N = c_dev.shape
    rng = np.random.default_rng(seed)
    ii = [rng.integers(0, M, n), np.zeros(N, np.int64), np.full(N, M - 1), np.arange(M), np.arange(M)]
    jj = [rng.integers(0, N, n), np.arange(N), np.arange(N), np.zeros(M, np.int64), np.full(M, N - 1)]
    ii = np.concatenate(ii)
    jj = np.concatenate(jj)
    cref, sabs = orc.gemm_at(qa, fa, qb, fb, da, db, ii, jj)
    import torch
    flat = c_dev.reshape(-1)
    got = flat[torch.from_numpy(ii * N + jj).cuda()]
    res = orc.check(host(got), cref, sabs, qa.shape[1], orc.OUT_BF16 if out_bf16 else orc.OUT_F32)
    log(f"  {what} sampled n={ii.size} max_ratio={res['max_ratio']:.3e} normwise={res['normwise']:.3e}")
    assert res["ok"], (what, res)
    return res
