"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke
check.

This module holds no FP8 arithmetic (no encoding, scaling, pruning or GEMM):
it only draws FP32 matrices, shapes and arrival times, so that the GPU path and
the CPU oracle can be fed identical inputs.

Generators:
  uniform(seed, tensor_id, shape)  values on the grid 2^-23 in [-1, 1): a
      SplitMix64 hash of (seed, tensor_id, element index); the top 24 bits u
      give x = 2 u / 2^24 - 1.  Bit-exact and order-free.
  normal_outliers(seed, shape)     N(0, 1) from numpy's PCG64 generator,
      rounded to FP32; each element independently, with probability 1/100, is
      replaced by +-20 (20 sigma), the sign drawn from the same generator.
  log_uniform_int(rng, lo, hi, n)  integers whose logarithm is uniform:
      floor(exp(U ln(hi + 1))) clamped to [lo, hi].
  poisson_arrivals(rng, rate, n)   cumulative exponential gaps.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014), vectorised, wrapping."""
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def uniform(seed: int, tensor_id: int, shape) -> np.ndarray:
    """FP32 values in [-1, 1) on a 2^-23 grid from a counter hash."""
    n = int(np.prod(shape))
    key = _mix64(np.array([(seed & 0xFFFFFFFF) << 32 | (tensor_id & 0xFFFFFFFF)], dtype=np.uint64))[0]
    out = np.empty(n, dtype=np.float32)
    chunk = 1 << 24
    for lo in range(0, n, chunk):
        idx = np.arange(lo, min(n, lo + chunk), dtype=np.uint64)
        with np.errstate(over="ignore"):
            h = _mix64(idx * _GOLDEN + key)
        u = (h >> np.uint64(40)).astype(np.int64)               # top 24 bits
        out[lo:lo + idx.size] = (u.astype(np.float64) * 2.0 ** -23 - 1.0).astype(np.float32)
    return out.reshape(shape)


def normal_outliers(seed: int, shape, p_outlier: float = 0.01, outlier: float = 20.0) -> np.ndarray:
    """N(0,1) FP32 values; a fraction p_outlier replaced by +-outlier."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape, dtype=np.float32)
    hit = rng.random(shape, dtype=np.float32) < p_outlier
    sign = np.where(rng.random(shape, dtype=np.float32) < 0.5, -1.0, 1.0).astype(np.float32)
    x[hit] = outlier * sign[hit]
    return x


def log_uniform_int(rng: np.random.Generator, lo: int, hi: int, n: int) -> np.ndarray:
    u = rng.random(n)
    v = np.floor(np.exp(u * np.log(hi + 1.0))).astype(np.int64)
    return np.clip(v, lo, hi)


def poisson_arrivals(rng: np.random.Generator, rate_per_s: float, n: int) -> np.ndarray:
    gaps = rng.exponential(1.0 / rate_per_s, n)
    return np.cumsum(gaps) - gaps[0]
