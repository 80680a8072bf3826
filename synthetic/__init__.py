"""Seeded synthetic inputs for the dot / asum / gemv workloads.

This module only draws numbers; it holds none of the reduction arithmetic.
Both sides of every parity check (the HIP library and the CPU oracle) take
their inputs from here, so they see the same bytes.

Generator: numpy ``default_rng(seed)`` (PCG64).  Distributions:

* ``uniform_pm1``: 2*U[0,1) - 1 in binary32.  ``rng.random(dtype=float32)``
  returns multiples of 2^-24, so 2u is exact and 2u - 1 is exact as well
  (every value k*2^-23 - 1 in (-1, 1) is a binary32 number).
* ``normal``: standard normal in binary32 (``rng.standard_normal``).
* ``log_uniform_signed``: 10^U(lo, hi) with a random sign, rounded to
  binary32; it spans many binades so different summation orders give
  different roundings.
* bf16 / fp8-e4m3 matrices are quantised once here, on the host, from a
  binary32 matrix: bf16 by round-to-nearest-even (torch ``to(bfloat16)``);
  fp8 with a per-row scale s_r = amax_r / 448 (s_r = 1 for an all-zero row)
  and codes RNE(A / s_r) clamped to [-448, 448] (torch
  ``to(float8_e4m3fn)``).  The codes and scales are what both sides read.
"""

from __future__ import annotations

import numpy as np

SEEDS = {"small": 1711, "scale": 1712, "sweep": 1713, "precision": 1714, "batch": 1715}


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def uniform_pm1(g: np.random.Generator, shape) -> np.ndarray:
    u = g.random(shape, dtype=np.float32)
    return np.float32(2.0) * u - np.float32(1.0)


def normal(g: np.random.Generator, shape) -> np.ndarray:
    return g.standard_normal(shape, dtype=np.float32)


def log_uniform_signed(g: np.random.Generator, shape, lo: float = -4.0, hi: float = 4.0) -> np.ndarray:
    mag = 10.0 ** g.uniform(lo, hi, size=shape)
    sign = np.where(g.random(shape) < 0.5, -1.0, 1.0)
    return (sign * mag).astype(np.float32)


def integers_u32(g: np.random.Generator, shape, lo: int = -(1 << 31), hi: int = 1 << 31) -> np.ndarray:
    """Signed 32-bit integers stored as their two's-complement uint32 bits."""
    return g.integers(lo, hi, size=shape, dtype=np.int64).astype(np.int32).view(np.uint32)


def quantise_bf16(a: np.ndarray) -> np.ndarray:
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16)


def quantise_fp8_rows(a: np.ndarray):
    """(codes uint8 [m, k], scale float32 [m])."""
    import torch
    a = np.ascontiguousarray(a, dtype=np.float32)
    amax = np.abs(a).max(axis=1)
    scale = np.where(amax > 0, amax / np.float32(448.0), np.float32(1.0)).astype(np.float32)
    q = np.clip(a / scale[:, None], -448.0, 448.0).astype(np.float32)
    codes = torch.from_numpy(q).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    return codes, scale


# ------------------------------------------------------------- workloads

def dot_inputs(n: int, seed: int):
    g = rng(seed)
    return uniform_pm1(g, n), uniform_pm1(g, n)


def asum_inputs(n: int, seed: int):
    return uniform_pm1(rng(seed), n)


def gemv_inputs(m: int, k: int, seed: int):
    g = rng(seed)
    A = normal(g, (m, k))
    x = uniform_pm1(g, k)
    return A, x


def kahan_dot_inputs(n: int, seed: int):
    g = rng(seed)
    return log_uniform_signed(g, n), log_uniform_signed(g, n)
