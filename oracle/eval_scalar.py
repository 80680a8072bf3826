"""Element-by-element evaluator of functional DPIA expressions (tiny inputs).

An independent second reading of the same semantics as ``eval_numpy``, kept
as simple as possible so it can be checked by eye against the paper:

* arrays are Python lists, pairs are Python tuples (Sec. 5.1 data sets);
* ``map f e`` builds the list of ``f`` applied to every element
  (Stage II: mapI = parfor over indices, Sec. 4.2); all hierarchy variants
  and the address-space wrappers mean the same (Sec. 6.1);
* ``reduce f init e`` keeps one accumulator, starts it at ``init`` and
  replaces it by ``f element accumulator`` for each element in increasing
  index order (Stage II: reduceI = new + sequential for, Sec. 4.2);
* ``split n`` cuts a list into consecutive rows of n, ``join`` concatenates
  rows, ``zip`` pairs elements, ``transpose`` swaps rows and columns
  (Fig. 7 index paths);
* numbers are tagged with their format.  binary32 arithmetic is done on
  Python floats (binary64) and rounded to binary32 after every single
  operation with ``struct``.  For + - * / this double rounding returns the
  correctly rounded binary32 result, since 53 >= 2*24 + 2 (S. A. Figueroa,
  "When is double rounding innocuous?", SIGNUM Newsletter 30(3), 1995);
  integers are reduced modulo 2^32.

It shares no code with ``eval_numpy`` beyond the parser and the format
decoders of single codes.
"""

from __future__ import annotations

import math
import struct
from typing import Dict

import numpy as np

from . import formats
from .dpia_lang import (ADDRESS_SPACE, MAP_LIKE, REDUCE_LIKE, App, Lam, Lit, Prim,
                        Var, parse)


def round_f32(x: float) -> float:
    """Nearest binary32 value (ties to even) of a Python float."""
    if math.isnan(x) or math.isinf(x):
        return x
    try:
        return struct.unpack("<f", struct.pack("<f", x))[0]
    except OverflowError:
        # beyond the largest binary32: IEEE rounding to nearest gives inf
        return math.copysign(math.inf, x)


class N:
    """A number with its format: 'f32', 'f64', 'u32', 'u16' or 'u8'."""
    __slots__ = ("fmt", "v")

    def __init__(self, fmt: str, v):
        self.fmt = fmt
        self.v = v

    def __repr__(self):
        return f"N({self.fmt},{self.v!r})"


def _arith(name: str, a: N, b: N) -> N:
    if a.fmt != b.fmt:
        raise ValueError(f"{name} on {a.fmt} and {b.fmt}")
    if a.fmt == "u32":
        if name == "/":
            raise ValueError("integer division is not defined")
        r = {"+": a.v + b.v, "-": a.v - b.v, "*": a.v * b.v}[name]
        return N("u32", r % (1 << 32))
    if a.fmt not in ("f32", "f64"):
        raise ValueError(f"no arithmetic on storage codes ({a.fmt})")
    x, y = a.v, b.v
    if name == "+":
        r = x + y
    elif name == "-":
        r = x - y
    elif name == "*":
        r = x * y
    else:
        if y == 0.0:
            if x == 0.0 or math.isnan(x):
                r = math.nan
            else:
                r = math.copysign(math.inf, x) * math.copysign(1.0, y)
        else:
            r = x / y
    return N(a.fmt, round_f32(r) if a.fmt == "f32" else r)


def _to_value(a: np.ndarray):
    if a.ndim == 0:
        dt = a.dtype
        if dt == np.float32:
            return N("f32", float(a))
        if dt == np.float64:
            return N("f64", float(a))
        if dt == np.uint32:
            return N("u32", int(a))
        if dt == np.uint16:
            return N("u16", int(a))
        if dt == np.uint8:
            return N("u8", int(a))
        raise ValueError(f"unsupported dtype {dt}")
    return [_to_value(a[i]) for i in range(a.shape[0])]


def _from_value(v):
    if isinstance(v, Vc):
        return np.array([_from_value(x) for x in v])
    if isinstance(v, tuple):
        return tuple(_from_value(x) for x in v)
    if isinstance(v, list):
        return np.array([_from_value(x) for x in v])
    dt = {"f32": np.float32, "f64": np.float64, "u32": np.uint32,
          "u16": np.uint16, "u8": np.uint8}[v.fmt]
    return np.array(v.v, dtype=dt)


class Vc(tuple):
    """A vector value num<n>: a tuple of n numbers of one format."""


def _vec_arith(name, a, b):
    if isinstance(a, Vc) and isinstance(b, Vc):
        if len(a) != len(b):
            raise ValueError("vectors of different lengths")
        return Vc(_arith(name, a[i], b[i]) for i in range(len(a)))
    if isinstance(a, Vc) or isinstance(b, Vc):
        raise ValueError(f"{name} of a vector and a number")
    return _arith(name, a, b)


class _Fn:
    def __init__(self, lam: Lam, env):
        self.lam = lam
        self.env = env


def _eval(e, env, num: str):
    if isinstance(e, Lit):
        if num == "u32":
            return N("u32", int(e.text) % (1 << 32))
        v = float(e.text)
        return N(num, round_f32(v) if num == "f32" else v)
    if isinstance(e, Var):
        return env[e.name]
    if isinstance(e, Lam):
        return _Fn(e, env)
    if isinstance(e, App):
        return _call(_eval(e.fn, env, num), [_eval(a, env, num) for a in e.args], num)
    assert isinstance(e, Prim)
    name, args = e.name, e.args
    if name in ADDRESS_SPACE:
        return _eval(args[0], env, num)
    if name in MAP_LIKE:
        f = _eval(args[0], env, num)
        xs = _eval(args[1], env, num)
        out = [None] * len(xs)
        for i in range(len(xs)):          # parfor: independent iterations
            out[i] = _call(f, [xs[i]], num)
        return out
    if name in REDUCE_LIKE:
        f = _eval(args[0], env, num)
        acc = _eval(args[1], env, num)
        xs = _eval(args[2], env, num)
        for i in range(len(xs)):          # for: sequential, increasing i
            acc = _call(f, [xs[i], acc], num)
        return acc
    if name == "zip":
        a = _eval(args[0], env, num)
        b = _eval(args[1], env, num)
        if len(a) != len(b):
            raise ValueError("zip of arrays of different lengths")
        return [(a[i], b[i]) for i in range(len(a))]
    if name == "split":
        n = int(args[0].text)
        v = _eval(args[1], env, num)
        if n <= 0 or len(v) % n:
            raise ValueError("split does not divide")
        return [v[r * n:(r + 1) * n] for r in range(len(v) // n)]
    if name == "join":
        v = _eval(args[0], env, num)
        out = []
        for row in v:
            out.extend(row)
        return out
    if name == "transpose":
        v = _eval(args[0], env, num)
        if not v:
            raise ValueError("transpose of an empty array")
        return [[v[r][c] for r in range(len(v))] for c in range(len(v[0]))]
    if name == "pair":
        return (_eval(args[0], env, num), _eval(args[1], env, num))
    if name == "fst":
        return _eval(args[0], env, num)[0]
    if name == "snd":
        return _eval(args[0], env, num)[1]
    if name == "asVector":
        n = int(args[0].text)
        v = _eval(args[1], env, num)
        if n <= 0 or len(v) % n:
            raise ValueError("asVector does not divide")
        return [Vc(v[r * n:(r + 1) * n]) for r in range(len(v) // n)]
    if name == "asScalar":
        n = int(args[0].text)
        out = []
        for vec in _eval(args[1], env, num):
            if not isinstance(vec, Vc) or len(vec) != n:
                raise ValueError("asScalar of a non-vector")
            out.extend(vec)
        return out
    if name == "broadcast":
        n = int(args[0].text)
        a = _eval(args[1], env, num)
        return Vc([a] * n)
    if name in ("+", "-", "*", "/"):
        return _vec_arith(name, _eval(args[0], env, num), _eval(args[1], env, num))
    a = _eval(args[0], env, num)
    if isinstance(a, Vc) and name in ("negate", "abs"):
        return Vc(N(c.fmt, -c.v if name == "negate" else abs(c.v)) for c in a)
    if name == "negate":
        return N(a.fmt, -a.v)
    if name == "abs":
        return N(a.fmt, abs(a.v))
    if name == "f64":
        return N("f64", a.v)
    if name == "f32":
        return N("f32", round_f32(a.v))
    if name == "bf16":
        if a.fmt != "u16":
            raise ValueError("bf16 decodes 16-bit codes")
        return N("f32", struct.unpack("<f", struct.pack("<I", a.v << 16))[0])
    if name == "fp8":
        if a.fmt != "u8":
            raise ValueError("fp8 decodes 8-bit codes")
        return N("f32", formats.fp8_e4m3_value(a.v))
    raise ValueError(f"unknown primitive {name!r}")


def _call(f, args, num):
    if not isinstance(f, _Fn) or len(args) != len(f.lam.params):
        raise ValueError("bad application")
    env = dict(f.env)
    env.update(zip(f.lam.params, args))
    return _eval(f.lam.body, env, num)


def evaluate(expr, inputs: Dict[str, np.ndarray], num: str = "f32"):
    """Same contract as ``eval_numpy.evaluate``; meant for inputs of at most a
    few thousand elements."""
    e = parse(expr) if isinstance(expr, str) else expr
    env = {k: _to_value(np.asarray(a)) for k, a in inputs.items()}
    return _from_value(_eval(e, env, num))
