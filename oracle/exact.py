"""Correctly rounded reference values and error bounds (test infrastructure).

``math.fsum`` returns the correctly rounded sum of its binary64 arguments
(Shewchuk's exact partials; CPython documents it as exact up to the final
rounding).  The product of two binary32 numbers is exact in binary64
(24 + 24 significant bits < 53), so ``fsum`` of the binary64 products is the
correctly rounded value of the exact dot product.

The error bound is the standard one for summation in any fixed order
(N. J. Higham, Accuracy and Stability of Numerical Algorithms, 2nd ed.,
Sec. 4.2): if every term passes through at most h rounded additions, and
the terms were themselves rounded once, the computed sum s' satisfies
|s' - s| <= gamma_{h+1} * sum |t_i| with gamma_k = k u / (1 - k u) and
u = 2^-24 for binary32.
"""

from __future__ import annotations

import math

import numpy as np

U32 = 2.0 ** -24


def gamma(k: int, u: float = U32) -> float:
    if k * u >= 1:
        return math.inf
    return k * u / (1 - k * u)


def dot_exact(x: np.ndarray, y: np.ndarray) -> float:
    return math.fsum((np.asarray(x, np.float64) * np.asarray(y, np.float64)).tolist())


def dot_abs_terms(x: np.ndarray, y: np.ndarray) -> float:
    return math.fsum(np.abs(np.asarray(x, np.float64) * np.asarray(y, np.float64)).tolist())


def asum_exact(x: np.ndarray) -> float:
    return math.fsum(np.abs(np.asarray(x, np.float64)).tolist())


def gemv_exact(A: np.ndarray, x: np.ndarray) -> np.ndarray:
    A64 = np.asarray(A, np.float64)
    x64 = np.asarray(x, np.float64)
    return np.array([math.fsum((A64[r] * x64).tolist()) for r in range(A64.shape[0])])


def strategy_depth(n: int, seq: int, lanes: int, combine: str, row_parts: int = 1) -> int:
    """Most rounded additions any term passes through in the plain strategy
    (lane fold of ``seq`` additions from +0, then the chunk combine, then the
    sequential fold of the chunk results from +0)."""
    chunks = n // (seq * lanes)
    within = lanes if combine == "seq" else 2 * max(1, int(math.log2(lanes)))
    return seq + within + chunks + row_parts + 1
