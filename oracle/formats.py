"""Decoding of the low-precision storage formats, from their definitions.

Both decoders are exact: every bf16 and every finite fp8-e4m3 value is a
binary32 value.  They are written from the format definitions, not from any
library, and are pinned in the tests against torch's own conversions over
every code.

bf16: the upper 16 bits of an IEEE-754 binary32 (1 sign, 8 exponent,
7 fraction bits), so decoding places the code in the high half of a 32-bit
word.

fp8-e4m3 (OCP 8-bit floating point specification, "E4M3"): 1 sign bit,
4 exponent bits with bias 7, 3 fraction bits.  Exponent field 0 encodes
subnormals, value (-1)^s * 2^(1-7) * (m/8).  All other exponent fields are
normal, value (-1)^s * 2^(e-7) * (1 + m/8), except S.1111.111, the only NaN
encodings.  There are no infinities; the largest finite value is 448.
"""

from __future__ import annotations

import math

import numpy as np


def bf16_decode(codes: np.ndarray) -> np.ndarray:
    c = np.asarray(codes)
    if c.dtype != np.uint16:
        raise TypeError("bf16 codes must be uint16")
    return (c.astype(np.uint32) << np.uint32(16)).view(np.float32)


def fp8_e4m3_value(code: int) -> float:
    """Value of one fp8-e4m3 code as a Python float (NaN for S.1111.111)."""
    if not 0 <= code <= 0xFF:
        raise ValueError("fp8 code out of range")
    sign = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 0x7
    if e == 0xF and m == 0x7:
        return math.nan
    if e == 0:
        return sign * math.ldexp(m / 8.0, 1 - 7)
    return sign * math.ldexp(1.0 + m / 8.0, e - 7)


# All 256 decoded values, in binary32 (exact: at most 4 significant bits).
FP8_E4M3_TABLE = np.array([fp8_e4m3_value(c) for c in range(256)], dtype=np.float32)


def fp8_decode(codes: np.ndarray) -> np.ndarray:
    c = np.asarray(codes)
    if c.dtype != np.uint8:
        raise TypeError("fp8 codes must be uint8")
    return FP8_E4M3_TABLE[c]
