"""Evaluator of functional DPIA expressions that runs at full problem sizes.

Semantics followed (the paper's, restated):

* Data types denote sets: ``num`` a set of numbers, ``d1 x d2`` pairs and
  ``n.d`` functions from {0..n-1} to d (Sec. 5.1).  An array is therefore
  nothing but its element at every index.
* ``map f e`` is the array whose element i is ``f`` applied to element i of
  ``e`` (Stage II: mapI is a parfor over the indices whose iterations are
  independent, Sec. 4.2).  Its hierarchy variants mapGlobal, mapWorkgroup,
  mapLocal, mapSeq denote the same function (Sec. 6.1), and toGlobal,
  toLocal, toPrivate are the identity on functions (Sec. 6.1).
* ``reduce f init e``: a fresh accumulator holds ``init``; then for
  i = 0, 1, ..., n-1 in that order the accumulator becomes
  ``f (element i of e) accumulator`` (Stage II definition of reduceI,
  Sec. 4.2; element first, accumulator second as in the dot-product
  examples of Sec. 2.1).  reduceSeq is the same.
* Layout primitives move indices, never values (Fig. 7): element (i, j) of
  ``split n e`` is element i*n + j of e, element i of ``join e`` is element
  (i div n, i mod n) of e where n is the inner length, element i of
  ``zip a b`` is the pair (a[i], b[i]).  ``transpose`` swaps the two outer
  indices.
* Arithmetic: each of + - * / negate abs is one IEEE-754 operation with
  round-to-nearest-even in the value's own format (binary32 unless the
  expression converts to binary64); integer values are 32-bit and wrap
  modulo 2^32.  No operation is fused or reassociated.

How it runs: because the iterations of a map are independent, evaluating the
body once on a whole array of arguments gives, element for element, exactly
the values of evaluating it per index.  Every value therefore carries
leading "batch" axes, one per enclosing map, and the arithmetic of all map
iterations happens in single numpy ufunc calls (which round each element
separately and never fuse a multiply into an add).  A reduce never becomes a
vector operation: it is a Python loop over its index, in increasing order,
applying the operator to all batch elements at once.  No numpy reduction
(``sum``, ``add.reduce``, ``dot``), whose summation order is unspecified, is
used anywhere.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, Tuple, Union

import numpy as np

from . import formats
from .dpia_lang import (ADDRESS_SPACE, MAP_LIKE, REDUCE_LIKE, App, Expr, Lam, Lit,
                        Prim, Var, parse)

NUM_DTYPES = {
    "f32": np.dtype(np.float32),
    "f64": np.dtype(np.float64),
    "u32": np.dtype(np.uint32),   # 32-bit integers, arithmetic modulo 2^32
    "u16": np.dtype(np.uint16),   # bf16 storage codes (decoded by "bf16")
    "u8": np.dtype(np.uint8),     # fp8-e4m3 storage codes (decoded by "fp8")
}


# ----------------------------------------------------------------- data types

@dataclass(frozen=True)
class Num:
    dt: np.dtype


@dataclass(frozen=True)
class Vec:
    """num<n>: n numbers of one format (Sec. 6.1 vector type)."""
    n: int
    dt: np.dtype


@dataclass(frozen=True)
class Arr:
    n: int
    elem: "Ty"


@dataclass(frozen=True)
class Tup:
    a: "Ty"
    b: "Ty"


Ty = Union[Num, Vec, Arr, Tup]


def type_of_array(a: np.ndarray) -> Ty:
    t: Ty = Num(a.dtype)
    for n in reversed(a.shape):
        t = Arr(int(n), t)
    return t


class EvalError(ValueError):
    pass


# ----------------------------------------------------------------- values
# A data value at batch rank ``nb`` holds, for every leaf number of its type,
# an ndarray whose first ``nb`` axes are the batch axes (size 1 where the
# value does not vary along that enclosing map) followed by one axis per
# array level of the type, outermost first, and, for a vector, one last axis
# of its n components.  Pairs hold a tuple of the two component
# representations; an array of pairs is therefore a pair of arrays.

@dataclass
class Data:
    ty: Ty
    rep: object   # ndarray or nested tuple of ndarrays


@dataclass
class Closure:
    lam: Lam
    env: Dict[str, Tuple[object, int]]


def _leaves(rep, f):
    if isinstance(rep, tuple):
        return tuple(_leaves(r, f) for r in rep)
    return f(rep)


def _raise_rank(v, frm: int, to: int):
    """A value bound at batch rank ``frm`` seen from inside deeper maps."""
    if frm == to or isinstance(v, Closure):
        return v
    axes = tuple(range(frm, to))
    return Data(v.ty, _leaves(v.rep, lambda a: np.expand_dims(a, axes)))


# ----------------------------------------------------------------- evaluation

class _Evaluator:
    def __init__(self, num: str):
        if num not in ("f32", "f64", "u32"):
            raise EvalError(f"unsupported num type {num!r}")
        self.num = NUM_DTYPES[num]

    def eval(self, e: Expr, env, nb: int):
        if isinstance(e, Lit):
            if self.num.kind == "f":
                val = float(e.text)
            else:
                val = int(e.text)
            return Data(Num(self.num), np.full((1,) * nb, val, dtype=self.num))
        if isinstance(e, Var):
            if e.name not in env:
                raise EvalError(f"unbound variable {e.name!r}")
            v, bound = env[e.name]
            return _raise_rank(v, bound, nb)
        if isinstance(e, Lam):
            return Closure(e, env)
        if isinstance(e, App):
            fn = self.eval(e.fn, env, nb)
            args = [self.eval(a, env, nb) for a in e.args]
            return self.apply(fn, args, nb)
        if isinstance(e, Prim):
            return self.prim(e, env, nb)
        raise EvalError(f"not an expression: {e!r}")

    def apply(self, fn, args, nb: int):
        if not isinstance(fn, Closure):
            raise EvalError("application of a non-function")
        if len(args) != len(fn.lam.params):
            raise EvalError("wrong number of arguments")
        env = dict(fn.env)
        for p, a in zip(fn.lam.params, args):
            env[p] = (a, nb)
        return self.eval(fn.lam.body, env, nb)

    def data(self, e, env, nb) -> Data:
        v = self.eval(e, env, nb)
        if not isinstance(v, Data):
            raise EvalError("expected data, got a function")
        return v

    def fun(self, e, env, nb) -> Closure:
        v = self.eval(e, env, nb)
        if not isinstance(v, Closure):
            raise EvalError("expected a function")
        return v

    def prim(self, e: Prim, env, nb: int):
        name, args = e.name, e.args

        if name in ADDRESS_SPACE:           # identity on functions
            return self.fun(args[0], env, nb)

        if name in MAP_LIKE:
            f = self.fun(args[0], env, nb)
            xs = self.data(args[1], env, nb)
            if not isinstance(xs.ty, Arr):
                raise EvalError(f"{name} over a non-array")
            n = xs.ty.n
            # element i of xs, for every i at once: the array axis becomes
            # the innermost batch axis
            elem = Data(xs.ty.elem, xs.rep)
            r = self.apply(f, [elem], nb + 1)
            if not isinstance(r, Data):
                raise EvalError("map body returned a function")

            def widen(a):
                if a.shape[nb] != n:
                    shape = a.shape[:nb] + (n,) + a.shape[nb + 1:]
                    a = np.broadcast_to(a, shape)
                return a
            return Data(Arr(n, r.ty), _leaves(r.rep, widen))

        if name in REDUCE_LIKE:
            f = self.fun(args[0], env, nb)
            acc = self.data(args[1], env, nb)
            xs = self.data(args[2], env, nb)
            if not isinstance(xs.ty, Arr):
                raise EvalError(f"{name} over a non-array")
            idx_prefix = (slice(None),) * nb
            for i in range(xs.ty.n):       # sequential, increasing index
                elem = Data(xs.ty.elem, _leaves(xs.rep, lambda a: a[idx_prefix + (i,)]))
                acc2 = self.apply(f, [elem, acc], nb)
                if not isinstance(acc2, Data) or acc2.ty != acc.ty:
                    raise EvalError(f"{name}: operator changes the accumulator type "
                                    f"({acc.ty} -> {getattr(acc2, 'ty', None)})")
                acc = acc2
            return acc

        if name == "zip":
            a = self.data(args[0], env, nb)
            b = self.data(args[1], env, nb)
            if not (isinstance(a.ty, Arr) and isinstance(b.ty, Arr)) or a.ty.n != b.ty.n:
                raise EvalError("zip of arrays of different lengths")
            return Data(Arr(a.ty.n, Tup(a.ty.elem, b.ty.elem)), (a.rep, b.rep))

        if name == "split":
            n = int(args[0].text)
            v = self.data(args[1], env, nb)
            if not isinstance(v.ty, Arr) or n <= 0 or v.ty.n % n:
                raise EvalError(f"split {n} of an array of length {getattr(v.ty, 'n', None)}")
            m = v.ty.n // n

            def cut(a):
                return a.reshape(a.shape[:nb] + (m, n) + a.shape[nb + 1:])
            return Data(Arr(m, Arr(n, v.ty.elem)), _leaves(v.rep, cut))

        if name == "join":
            v = self.data(args[0], env, nb)
            if not (isinstance(v.ty, Arr) and isinstance(v.ty.elem, Arr)):
                raise EvalError("join of a non-nested array")
            m, n = v.ty.n, v.ty.elem.n

            def glue(a):
                return a.reshape(a.shape[:nb] + (m * n,) + a.shape[nb + 2:])
            return Data(Arr(m * n, v.ty.elem.elem), _leaves(v.rep, glue))

        if name == "transpose":
            v = self.data(args[0], env, nb)
            if not (isinstance(v.ty, Arr) and isinstance(v.ty.elem, Arr)):
                raise EvalError("transpose of a non-nested array")
            return Data(Arr(v.ty.elem.n, Arr(v.ty.n, v.ty.elem.elem)),
                        _leaves(v.rep, lambda a: np.swapaxes(a, nb, nb + 1)))

        if name == "pair":
            a = self.data(args[0], env, nb)
            b = self.data(args[1], env, nb)
            return Data(Tup(a.ty, b.ty), (a.rep, b.rep))

        if name in ("fst", "snd"):
            p = self.data(args[0], env, nb)
            if not isinstance(p.ty, Tup):
                raise EvalError(f"{name} of a non-pair")
            k = 0 if name == "fst" else 1
            return Data(p.ty.a if k == 0 else p.ty.b, p.rep[k])

        if name == "asVector":
            n = int(args[0].text)
            v = self.data(args[1], env, nb)
            if not (isinstance(v.ty, Arr) and isinstance(v.ty.elem, Num)) or n <= 0 \
                    or v.ty.n % n:
                raise EvalError(f"asVector {n} of {v.ty}")
            m = v.ty.n // n
            return Data(Arr(m, Vec(n, v.ty.elem.dt)),
                        v.rep.reshape(v.rep.shape[:nb] + (m, n)))

        if name == "asScalar":
            n = int(args[0].text)
            v = self.data(args[1], env, nb)
            if not (isinstance(v.ty, Arr) and isinstance(v.ty.elem, Vec)) or v.ty.elem.n != n:
                raise EvalError(f"asScalar {n} of {v.ty}")
            m = v.ty.n
            return Data(Arr(m * n, Num(v.ty.elem.dt)),
                        v.rep.reshape(v.rep.shape[:nb] + (m * n,)))

        if name == "broadcast":
            n = int(args[0].text)
            a = self.data(args[1], env, nb)
            if not isinstance(a.ty, Num) or n <= 0:
                raise EvalError(f"broadcast {n} of {a.ty}")
            return Data(Vec(n, a.ty.dt),
                        np.array(np.broadcast_to(a.rep[..., None], a.rep.shape + (n,))))

        if name in ("+", "-", "*", "/"):
            a = self.data(args[0], env, nb)
            b = self.data(args[1], env, nb)
            # numbers of one format, or vectors of one type (per component)
            if not (isinstance(a.ty, (Num, Vec)) and a.ty == b.ty):
                raise EvalError(f"{name} on {a.ty} and {b.ty}")
            if a.ty.dt.kind not in "fu" or a.ty.dt.itemsize < 4:
                raise EvalError(f"no arithmetic on storage codes ({a.ty.dt})")
            op = {"+": np.add, "-": np.subtract, "*": np.multiply}.get(name)
            if op is None:
                if a.ty.dt.kind != "f":
                    raise EvalError("integer division is not defined")
                op = np.divide
            return Data(a.ty, np.asarray(op(a.rep, b.rep), dtype=a.ty.dt))

        if name in ("negate", "abs", "f32", "f64", "bf16", "fp8"):
            a = self.data(args[0], env, nb)
            if isinstance(a.ty, Vec) and name in ("negate", "abs"):
                if a.ty.dt.kind != "f":
                    raise EvalError(f"{name} is defined on floating point only")
                op = np.negative if name == "negate" else np.abs
                return Data(a.ty, np.asarray(op(a.rep)))
            if not isinstance(a.ty, Num):
                raise EvalError(f"{name} of a non-number")
            dt = a.ty.dt
            if name == "negate":
                if dt.kind != "f":
                    raise EvalError("negate is defined on floating point only")
                return Data(a.ty, np.asarray(np.negative(a.rep)))
            if name == "abs":
                if dt.kind != "f":
                    raise EvalError("abs is defined on floating point only")
                return Data(a.ty, np.asarray(np.abs(a.rep)))
            if name in ("f32", "f64"):
                if dt.kind != "f":
                    raise EvalError(f"{name} converts floating point only")
                to = NUM_DTYPES[name]
                return Data(Num(to), np.asarray(a.rep, dtype=dt).astype(to))
            if name == "bf16":
                return Data(Num(NUM_DTYPES["f32"]), formats.bf16_decode(a.rep))
            return Data(Num(NUM_DTYPES["f32"]), formats.fp8_decode(a.rep))

        raise EvalError(f"unknown primitive {name!r}")


def evaluate(expr, inputs: Dict[str, np.ndarray], num: str = "f32"):
    """Value of ``expr`` (text or AST) with the named input arrays bound.

    Returns an ndarray (a 0-d array for a number) or a tuple of them for a
    pair.  ``num`` is the type of numeric literals ("f32", "f64", "u32").
    """
    e = parse(expr) if isinstance(expr, str) else expr
    env = {}
    for k, a in inputs.items():
        a = np.asarray(a)
        if a.dtype not in NUM_DTYPES.values():
            raise EvalError(f"input {k!r} has unsupported dtype {a.dtype}")
        env[k] = (Data(type_of_array(a), a), 0)
    with np.errstate(over="ignore", under="ignore", invalid="ignore", divide="ignore"):
        v = _Evaluator(num).data(e, env, 0)
    return _leaves(v.rep, np.asarray)
