"""Functional DPIA expression -> imperative program -> HIP source.

Stage I and II (Sec. 4).  Two mutually recursive translations, written here
with Python closures standing for the paper's meta-level functions:

* ``acc(e, out)`` (the acceptor-passing translation A) appends commands that
  write the value of ``e`` through the acceptor ``out``;
* ``val(e)`` (the continuation-passing translation C, with the continuation
  being "the rest of this function") returns the value of ``e`` as an
  expression or view, first appending the commands that compute any
  temporary it needs.

The Stage II meanings are used directly: a map becomes a parallel (or
sequential) loop over its index whose iteration i writes element i of the
acceptor (mapI = parfor), and a reduce becomes a fresh accumulator set to the
initial value, then a sequential loop in increasing index order replacing it
by ``f element accumulator``, then a copy to the acceptor (reduceI = new +
for).  Layout primitives never copy: ``split``, ``join``, ``zip``,
``transpose``, ``fst`` / ``snd``, ``asVector`` / ``asScalar`` are views whose
element i is an index computation on their argument (Fig. 7's access paths),
and their acceptor forms rewrite indices the same way.

Temporaries (Sec. 6.3): a map or reduce whose value is needed as an
expression is written to a fresh variable first.  Where it lives follows
OpenCL's memory levels: outside every parallel loop it is global memory
(hoisted to a workspace buffer that is a kernel argument), inside a
mapWorkgroup body and outside any mapLocal an array is local memory (hoisted
to the top of the kernel: one copy per work-group) and a number is private,
and inside a work-item it is private.  A toGlobal annotation puts the value
of the function it wraps in global memory wherever it is: inside parallel
loops the temporary is hoisted out of them as the paper's rule for hoisting
`new` out of a parallel loop has it, to one workspace buffer whose size is
the temporary's times the extents of the enclosing parallel loops, each
iteration using its own copy.  The annotations never change a value (Sec.
6.1); a choice that would break sharing (a private array written by several
work-items) is never made.

Stage III: every top-level parallel loop becomes one kernel; host-level
sequential code between them becomes a kernel run by a single work-item.
In a work-group body, code outside mapLocal is run alike by every work-item;
its writes to local or global memory are made by work-item 0 only and are
followed by a barrier, and every mapLocal loop ends with a barrier, so each
read of local memory sees the writes before it.

Arithmetic is emitted as C expressions on float / double / unsigned with one
operation per node, compiled without contraction, so every operation is one
IEEE-754 operation in the expression's order.
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass
from typing import Callable, Dict, List, Optional, Tuple, Union

from . import ir, passes
from .ir import Assign, Decl, For, IX, ParFor, iadd, idiv, imod, imul
from .lang import (MAPS, REDUCES, SPACES, Arr, Call, Lam, Lit, Name, Node, Num, Pair, Type,
                   Vec, check, parse)

CTYPES = {"f32": "float", "f64": "double", "u32": "unsigned", "u16": "unsigned short",
          "u8": "unsigned char"}
CODES = {"bf16": "unsigned short", "fp8": "unsigned char"}


class TranslateError(ValueError):
    pass


# ------------------------------------------------------------------ values

@dataclass
class SV:                      # a number: an expression
    ty: Num
    e: ir.Ex


@dataclass
class VV:                      # a vector: one expression per component
    ty: Vec
    comps: List[ir.Ex]


@dataclass
class AV:                      # an array: element i for an index expression i
    ty: Arr
    get: Callable[[IX], "Value"]


@dataclass
class PV:
    ty: Pair
    a: "Value"
    b: "Value"


@dataclass
class FV:                      # a function: a lambda with its environment
    lam: Lam
    env: Dict[str, object]
    space: Optional[str] = None


Value = Union[SV, VV, AV, PV]


# acceptors
@dataclass
class SA:
    ty: Num
    name: str
    idx: Optional[IX]
    space: str                 # "private", "local" or "global"


@dataclass
class VA:
    ty: Vec
    comps: List[SA]


@dataclass
class AA:
    ty: Arr
    at: Callable[[IX], "Acc"]


@dataclass
class PA:
    ty: Pair
    a: "Acc"
    b: "Acc"


Acc = Union[SA, VA, AA, PA]


# ------------------------------------------------------------------ storage

def _leaves(ty: Type, shape: Tuple[int, ...], name: str, out: list):
    """Storage of a value of type ty: one C array per number leaf (pairs are
    stored component-wise), with the array dimensions as a flat shape."""
    if isinstance(ty, Arr):
        _leaves(ty.elem, shape + (ty.n,), name, out)
    elif isinstance(ty, Pair):
        _leaves(ty.a, shape, name + "_a", out)
        _leaves(ty.b, shape, name + "_b", out)
    elif isinstance(ty, Vec):
        out.append((name, ty.c, shape + (ty.n,)))
    else:
        out.append((name, ty.c, shape))
    return out


def _flat(idx: List[IX], dims: Tuple[int, ...]) -> IX:
    code = idx[0]
    for i, d in zip(idx[1:], dims[1:]):
        code = iadd(imul(code, d), i)
    return code


def _ref(name: str, idx: List[IX], dims_of, scalar: set) -> Tuple[str, Optional[IX]]:
    if name in scalar:
        return name, None
    d = dims_of[name]
    return name, (_flat(idx, d) if d else ir.IConst(0))


def _view(ty: Type, name: str, idx: List[IX], dims_of: Dict[str, tuple], scalar: set) -> Value:
    if isinstance(ty, Arr):
        return AV(ty, lambda i, ty=ty: _view(ty.elem, name, idx + [i], dims_of, scalar))
    if isinstance(ty, Pair):
        return PV(ty, _view(ty.a, name + "_a", idx, dims_of, scalar),
                  _view(ty.b, name + "_b", idx, dims_of, scalar))
    if isinstance(ty, Vec):
        return VV(ty, [ir.Ref(*_ref(name, idx + [ir.IConst(c)], dims_of, scalar))
                       for c in range(ty.n)])
    return SV(ty, ir.Ref(*_ref(name, idx, dims_of, scalar)))


def _acceptor(ty: Type, name: str, idx: List[IX], dims_of, scalar: set, space: str) -> Acc:
    if isinstance(ty, Arr):
        return AA(ty, lambda i, ty=ty: _acceptor(ty.elem, name, idx + [i], dims_of, scalar,
                                                 space))
    if isinstance(ty, Pair):
        return PA(ty, _acceptor(ty.a, name + "_a", idx, dims_of, scalar, space),
                  _acceptor(ty.b, name + "_b", idx, dims_of, scalar, space))
    if isinstance(ty, Vec):
        return VA(ty, [SA(Num(ty.c), *_ref(name, idx + [ir.IConst(c)], dims_of, scalar), space)
                       for c in range(ty.n)])
    return SA(ty, *_ref(name, idx, dims_of, scalar), space)


# ------------------------------------------------------------------ translator

@dataclass
class Buffer:
    """A kernel argument: an input, an output or a workspace array."""
    name: str
    ctype: str
    elems: int
    kind: str                  # "in", "out" or "ws"


class Translator:
    def __init__(self, inputs: Dict[str, Tuple[str, Tuple[int, ...]]], num: str = "f32"):
        """inputs: name -> (element type "f32" / "f64" / "u32", shape)."""
        self.num = CTYPES[num]
        self.ids = itertools.count()
        self.buffers: List[Buffer] = []
        self.dims: Dict[str, tuple] = {}
        self.scalars: set = set()       # private numbers declared as C scalars
        self.env: Dict[str, object] = {}
        # the parallel loops around the code being translated: (index, extent)
        self.par: List[Tuple[str, int]] = []
        self.input_types: Dict[str, Type] = {}
        for name, (et, shape) in inputs.items():
            ty: Type = Num(CTYPES[et])
            for n in reversed(shape):
                ty = Arr(int(n), ty)
            self.input_types[name] = ty
            self.dims[name] = tuple(int(s) for s in shape)
            self.buffers.append(Buffer(name, CTYPES[et], max(1, _prod(shape)), "in"))
            self.env[name] = _view(ty, name, [], self.dims, self.scalars)

    def fresh(self, base: str) -> str:
        return f"{base}{next(self.ids)}"

    # -------------------------------------------------------------- types
    def tyof(self, n: Node, tenv: Dict[str, object]) -> Type:
        if isinstance(n, Lit):
            return Num(self.num)
        if isinstance(n, Name):
            t = tenv.get(n.id)
            if t is None:
                raise TranslateError(f"unbound name {n.id!r}")
            if isinstance(t, FV):
                raise TranslateError(f"{n.id!r} is a function, not data")
            return t
        if isinstance(n, Lam):
            raise TranslateError("a lambda is not data")
        h, a = n.head, n.args
        if not isinstance(h, str):
            fn, space = self.tyfun(h, tenv)
            return self.tyapp(fn, [self.tyof(x, tenv) for x in a], tenv)
        if h in MAPS:
            xs = self.tyof(a[1], tenv)
            if not isinstance(xs, Arr):
                raise TranslateError(f"{h} over {xs}")
            fn, _ = self.tyfun(a[0], tenv)
            return Arr(xs.n, self.tyapp(fn, [xs.elem], tenv))
        if h in REDUCES:
            return self.tyof(a[1], tenv)
        if h == "zip":
            x, y = self.tyof(a[0], tenv), self.tyof(a[1], tenv)
            if not (isinstance(x, Arr) and isinstance(y, Arr) and x.n == y.n):
                raise TranslateError(f"zip of {x} and {y}")
            return Arr(x.n, Pair(x.elem, y.elem))
        if h == "split":
            k = int(a[0].text)
            x = self.tyof(a[1], tenv)
            if not isinstance(x, Arr) or k <= 0 or x.n % k:
                raise TranslateError(f"split {k} of {x}")
            return Arr(x.n // k, Arr(k, x.elem))
        if h == "join":
            x = self.tyof(a[0], tenv)
            if not (isinstance(x, Arr) and isinstance(x.elem, Arr)):
                raise TranslateError(f"join of {x}")
            return Arr(x.n * x.elem.n, x.elem.elem)
        if h == "transpose":
            x = self.tyof(a[0], tenv)
            if not (isinstance(x, Arr) and isinstance(x.elem, Arr)):
                raise TranslateError(f"transpose of {x}")
            return Arr(x.elem.n, Arr(x.n, x.elem.elem))
        if h == "asVector":
            k = int(a[0].text)
            x = self.tyof(a[1], tenv)
            if not (isinstance(x, Arr) and isinstance(x.elem, Num)) or x.n % k:
                raise TranslateError(f"asVector {k} of {x}")
            return Arr(x.n // k, Vec(k, x.elem.c))
        if h == "asScalar":
            k = int(a[0].text)
            x = self.tyof(a[1], tenv)
            if not (isinstance(x, Arr) and isinstance(x.elem, Vec) and x.elem.n == k):
                raise TranslateError(f"asScalar {k} of {x}")
            return Arr(x.n * k, Num(x.elem.c))
        if h == "broadcast":
            x = self.tyof(a[1], tenv)
            if not isinstance(x, Num):
                raise TranslateError(f"broadcast of {x}")
            return Vec(int(a[0].text), x.c)
        if h == "pair":
            return Pair(self.tyof(a[0], tenv), self.tyof(a[1], tenv))
        if h in ("fst", "snd"):
            x = self.tyof(a[0], tenv)
            if not isinstance(x, Pair):
                raise TranslateError(f"{h} of {x}")
            return x.a if h == "fst" else x.b
        if h in ("+", "-", "*", "/"):
            x, y = self.tyof(a[0], tenv), self.tyof(a[1], tenv)
            if x != y or not isinstance(x, (Num, Vec)) or x.c in CODES.values():
                raise TranslateError(f"{h} on {x} and {y}")
            return x
        if h in CODES:
            x = self.tyof(a[0], tenv)
            if x != Num(CODES[h]):
                raise TranslateError(f"{h} decodes {CODES[h]} codes, not {x}")
            return Num("float")
        if h in ("negate", "abs"):
            x = self.tyof(a[0], tenv)
            if not isinstance(x, (Num, Vec)):
                raise TranslateError(f"{h} of {x}")
            return x
        if h in ("f32", "f64"):
            x = self.tyof(a[0], tenv)
            if not isinstance(x, Num):
                raise TranslateError(f"{h} of {x}")
            return Num(CTYPES[h])
        if h in SPACES:
            raise TranslateError(f"{h} wraps a function, not data")
        raise TranslateError(f"unknown primitive {h!r}")

    def tyfun(self, n: Node, tenv):
        """(lambda, type environment of its free names), space annotation."""
        if isinstance(n, Lam):
            return (n, tenv), None
        if isinstance(n, Name) and isinstance(tenv.get(n.id), FV):
            f = tenv[n.id]
            return (f.lam, self.tenv_of(f.env)), f.space
        if isinstance(n, Call) and isinstance(n.head, str) and n.head in SPACES:
            fn, _ = self.tyfun(n.args[0], tenv)
            return fn, n.head
        raise TranslateError("expected a function")

    def tyapp(self, fn, arg_types, tenv):
        lam, lam_tenv = fn
        if len(lam.params) != len(arg_types):
            raise TranslateError("wrong number of arguments")
        e2 = dict(lam_tenv)
        e2.update(zip(lam.params, arg_types))
        return self.tyof(lam.body, e2)

    # -------------------------------------------------------------- helpers
    def tenv_of(self, env) -> Dict[str, object]:
        return {k: (v if isinstance(v, FV) else v.ty) for k, v in env.items()}

    def new_var(self, ty: Type, space: str, out: list, base: str = "t"):
        name = self.fresh(base)
        leaves = _leaves(ty, (), name, [])
        # A global temporary inside parallel loops is hoisted out of them
        # (Sec. 6.3): one buffer with a copy per iteration of every
        # enclosing parallel loop -- its size scaled by their extents -- and
        # each iteration uses its own copy, indexed by the loops' indices.
        scale = tuple(n for _, n in self.par) if space == "global" else ()
        prefix = [ir.IVar(i) for i, _ in self.par] if space == "global" else []
        for leaf, ctype, dims in leaves:
            self.dims[leaf] = scale + dims
            size = _prod(dims) if dims else 0
            if space == "global":
                self.buffers.append(Buffer(leaf, ctype, max(1, _prod(scale) * max(1, size)), "ws"))
            else:
                if size == 0 and space == "private":
                    self.scalars.add(leaf)
                out.append(Decl(leaf, ctype, size, space))
        return (_view(ty, name, list(prefix), self.dims, self.scalars),
                _acceptor(ty, name, list(prefix), self.dims, self.scalars, space))

    def copy(self, v: Value, a: Acc, out: list, ctx: str):
        """a := v, element by element (a sequential loop over arrays)."""
        if isinstance(a, SA):
            out.append(Assign(a.name, a.idx, v.e, a.space, ctx))
        elif isinstance(a, VA):
            for sa, c in zip(a.comps, v.comps):
                out.append(Assign(sa.name, sa.idx, c, sa.space, ctx))
        elif isinstance(a, PA):
            self.copy(v.a, a.a, out, ctx)
            self.copy(v.b, a.b, out, ctx)
        else:
            i = self.fresh("i")
            body: list = []
            self.copy(v.get(ir.IVar(i)), a.at(ir.IVar(i)), body, ctx)
            out.append(For(i, a.ty.n, body))

    def space_for(self, ty: Type, ctx: str, hint: Optional[str]) -> str:
        if ctx == "host" or hint == "toGlobal":
            return "global"
        if ctx == "group" and (isinstance(ty, Arr) or hint == "toLocal"):
            return "local"
        return "private"

    # -------------------------------------------------------------- A
    def acc(self, n: Node, env, a: Acc, out: list, ctx: str):
        if isinstance(n, Call) and isinstance(n.head, str):
            h, args = n.head, n.args
            if h in MAPS:
                xs = self.val(args[1], env, out, ctx)
                f = self.fun(args[0], env)
                level = {"mapWorkgroup": "workgroup", "mapLocal": "local",
                         "mapGlobal": "global"}.get(h)
                i = self.fresh("g" if level == "workgroup" else ("l" if level else "k"))
                body: list = []
                inner = {"workgroup": "group", "local": "item", "global": "item"}.get(level, ctx)
                if level:
                    self.par.append((i, xs.ty.n))
                self.acc_app(f, [xs.get(ir.IVar(i))], a.at(ir.IVar(i)), body, inner)
                if level:
                    self.par.pop()
                out.append(ParFor(level, i, xs.ty.n, body) if level else For(i, xs.ty.n, body))
                return
            if h in REDUCES:
                xs = self.val(args[2], env, out, ctx)
                init = self.val(args[1], env, out, ctx)
                f = self.fun(args[0], env)
                accv, acca = self.new_var(init.ty, "private", out, "acc")
                self.copy(init, acca, out, ctx)
                i = self.fresh("k")
                body = []
                xi = xs.get(ir.IVar(i))
                if isinstance(init.ty, Num):
                    self.acc_app(f, [xi, accv], acca, body, ctx)
                else:
                    # compound accumulators: compute the new value aside, then
                    # replace, so no part is read after it was overwritten
                    tv, ta = self.new_var(init.ty, "private", body, "nxt")
                    self.acc_app(f, [xi, accv], ta, body, ctx)
                    self.copy(tv, acca, body, ctx)
                out.append(For(i, xs.ty.n, body))
                self.copy(accv, a, out, ctx)
                return
            if h == "join" and isinstance(a, AA):
                inner_n = self.tyof(args[0], self.tenv_of(env)).elem.n
                self.acc(args[0], env, AA(Arr(a.ty.n // inner_n, Arr(inner_n, a.ty.elem)),
                                          lambda i: AA(Arr(inner_n, a.ty.elem),
                                                       lambda j: a.at(iadd(imul(i, inner_n), j)))),
                         out, ctx)
                return
            if h == "split" and isinstance(a, AA):
                k = int(args[0].text)
                self.acc(args[1], env, AA(Arr(a.ty.n * k, a.ty.elem.elem),
                                          lambda i: a.at(idiv(i, k)).at(imod(i, k))),
                         out, ctx)
                return
            if h == "asScalar" and isinstance(a, AA):
                k = int(args[0].text)
                self.acc(args[1], env, AA(Arr(a.ty.n // k, Vec(k, a.ty.elem.c)),
                                          lambda i: VA(Vec(k, a.ty.elem.c),
                                                       [a.at(iadd(imul(i, k), c))
                                                        for c in range(k)])),
                         out, ctx)
                return
            if h == "pair" and isinstance(a, PA):
                self.acc(args[0], env, a.a, out, ctx)
                self.acc(args[1], env, a.b, out, ctx)
                return
            if h in SPACES:
                raise TranslateError(f"{h} wraps a function, not data")
        if isinstance(n, Call) and not isinstance(n.head, str):
            f = self.fun(n.head, env)
            argv = [self.val(x, env, out, ctx) for x in n.args]
            self.acc_app(f, argv, a, out, ctx, bind=True)
            return
        self.copy(self.val(n, env, out, ctx), a, out, ctx)

    def acc_app(self, f: FV, args: List[Value], a: Acc, out: list, ctx: str, bind=False):
        env = dict(f.env)
        for p, v in zip(f.lam.params, self._bound(args, out, ctx) if bind else args):
            env[p] = v
        if len(f.lam.params) != len(args):
            raise TranslateError("wrong number of arguments")
        self.acc(f.lam.body, env, a, out, ctx)

    def _bound(self, args: List[Value], out: list, ctx: str) -> List[Value]:
        """Numbers passed to a lambda are computed once into private
        constants (a let binding), so a parameter used twice is not
        evaluated twice."""
        res = []
        for v in args:
            if isinstance(v, SV):
                # outside every parallel loop the value may be read by a later
                # kernel: global memory there, a private constant elsewhere
                bv, ba = self.new_var(v.ty, "global" if ctx == "host" else "private", out, "v")
                self.copy(v, ba, out, ctx)
                res.append(bv)
            else:
                res.append(v)
        return res

    def fun(self, n: Node, env) -> FV:
        if isinstance(n, Lam):
            return FV(n, env)
        if isinstance(n, Name) and isinstance(env.get(n.id), FV):
            return env[n.id]
        if isinstance(n, Call) and isinstance(n.head, str) and n.head in SPACES:
            f = self.fun(n.args[0], env)
            return FV(f.lam, f.env, n.head)
        raise TranslateError("expected a function")

    # -------------------------------------------------------------- C
    def val(self, n: Node, env, out: list, ctx: str) -> Value:
        if isinstance(n, Lit):
            v = float(n.text)
            return SV(Num(self.num), ir.Lit(int(v) if self.num == "unsigned" else v, self.num))
        if isinstance(n, Name):
            if n.id not in env:
                raise TranslateError(f"unbound name {n.id!r}")
            v = env[n.id]
            if isinstance(v, FV):
                raise TranslateError(f"{n.id!r} is a function, not data")
            return v
        if isinstance(n, Lam):
            raise TranslateError("a lambda is not data")
        h, args = n.head, n.args
        if not isinstance(h, str) or h in MAPS or h in REDUCES:
            # a computation whose value is needed: into a fresh variable
            hint = None
            if not isinstance(h, str):
                hint = self.fun(h, env).space
            ty = self.tyof(n, self.tenv_of(env))
            if not isinstance(h, str) and isinstance(ty, Num) and ctx != "host":
                v, a = self.new_var(ty, "private", out)
                self.acc(n, env, a, out, ctx)
                return v
            v, a = self.new_var(ty, self.space_for(ty, ctx, hint), out)
            self.acc(n, env, a, out, ctx)
            return v
        if h == "zip":
            x, y = self.val(args[0], env, out, ctx), self.val(args[1], env, out, ctx)
            return AV(Arr(x.ty.n, Pair(x.ty.elem, y.ty.elem)),
                      lambda i: PV(Pair(x.ty.elem, y.ty.elem), x.get(i), y.get(i)))
        if h == "split":
            k = int(args[0].text)
            x = self.val(args[1], env, out, ctx)
            row = Arr(k, x.ty.elem)
            return AV(Arr(x.ty.n // k, row),
                      lambda i: AV(row, lambda j: x.get(iadd(imul(i, k), j))))
        if h == "join":
            x = self.val(args[0], env, out, ctx)
            m = x.ty.elem.n
            return AV(Arr(x.ty.n * m, x.ty.elem.elem),
                      lambda i: x.get(idiv(i, m)).get(imod(i, m)))
        if h == "transpose":
            x = self.val(args[0], env, out, ctx)
            row = Arr(x.ty.n, x.ty.elem.elem)
            return AV(Arr(x.ty.elem.n, row), lambda i: AV(row, lambda j: x.get(j).get(i)))
        if h == "asVector":
            k = int(args[0].text)
            x = self.val(args[1], env, out, ctx)
            vt = Vec(k, x.ty.elem.c)
            return AV(Arr(x.ty.n // k, vt),
                      lambda i: VV(vt, [x.get(iadd(imul(i, k), c)).e for c in range(k)]))
        if h == "asScalar":
            k = int(args[0].text)
            x = self.val(args[1], env, out, ctx)
            nt = Num(x.ty.elem.c)

            def elem(i):
                comps = x.get(idiv(i, k)).comps
                sel = imod(i, k)
                if isinstance(sel, ir.IConst):
                    return SV(nt, comps[sel.v])
                return SV(nt, ir.Select(sel, tuple(comps)))
            return AV(Arr(x.ty.n * k, nt), elem)
        if h == "broadcast":
            k = int(args[0].text)
            x = self.val(args[1], env, out, ctx)
            return VV(Vec(k, x.ty.c), [x.e] * k)
        if h == "pair":
            x, y = self.val(args[0], env, out, ctx), self.val(args[1], env, out, ctx)
            return PV(Pair(x.ty, y.ty), x, y)
        if h in ("fst", "snd"):
            p = self.val(args[0], env, out, ctx)
            return p.a if h == "fst" else p.b
        if h in ("+", "-", "*", "/"):
            x, y = self.val(args[0], env, out, ctx), self.val(args[1], env, out, ctx)
            if x.ty != y.ty or x.ty.c in CODES.values():
                raise TranslateError(f"{h} on {x.ty} and {y.ty}")
            if x.ty.c == "unsigned" and h == "/":
                raise TranslateError("integer division is not defined")
            if isinstance(x, VV):
                return VV(x.ty, [ir.Bin(h, p, q) for p, q in zip(x.comps, y.comps)])
            return SV(x.ty, ir.Bin(h, x.e, y.e))
        if h in ("negate", "abs"):
            x = self.val(args[0], env, out, ctx)
            if x.ty.c == "unsigned":
                raise TranslateError(f"{h} is defined on floating point only")
            op = "abs" if h == "abs" else "neg"
            if isinstance(x, VV):
                return VV(x.ty, [ir.Un(op, c) for c in x.comps])
            return SV(x.ty, ir.Un(op, x.e))
        if h in ("f32", "f64"):
            x = self.val(args[0], env, out, ctx)
            return SV(Num(CTYPES[h]), ir.Cast(CTYPES[h], x.e))
        if h in CODES:
            x = self.val(args[0], env, out, ctx)
            if x.ty != Num(CODES[h]):
                raise TranslateError(f"{h} decodes {CODES[h]} codes, not {x.ty}")
            return SV(Num("float"), ir.Decode(h, x.e))
        raise TranslateError(f"{h} cannot be used as data here")


def _prod(shape) -> int:
    p = 1
    for s in shape:
        p *= int(s)
    return p


# ------------------------------------------------------------------ Stage III

@dataclass
class Kernel:
    name: str
    kind: str                  # "workgroup", "global" or "single"
    body: List[object]
    iterations: int            # parallel loop length (1 for "single")
    local_width: int           # widest mapLocal in the kernel (work-items)


@dataclass
class Program:
    """A translated expression: HIP source, kernels in launch order, the
    buffers every kernel takes (inputs, outputs, workspace) and the C type
    of every array and variable."""
    source: str
    kernels: List[Kernel]
    buffers: List[Buffer]
    out_type: Type
    types: Dict[str, str]
    dims: Dict[str, tuple]


def translate(text: str, inputs: Dict[str, Tuple[str, Tuple[int, ...]]], num: str = "f32",
              name: str = "dpia", optimise: bool = True) -> Program:
    """Expression text -> Program.  ``inputs`` maps each free name to its
    element type and shape; the result is written to ``out`` (stored
    component-wise for pairs: out_a, out_b)."""
    node = parse(text)
    check(node)
    t = Translator(inputs, num)
    out_ty = t.tyof(node, t.tenv_of(t.env))
    leaves = _leaves(out_ty, (), "out", [])
    for leaf, ctype, dims in leaves:
        t.dims[leaf] = dims
        t.buffers.append(Buffer(leaf, ctype, max(1, _prod(dims)), "out"))
    out_acc = _acceptor(out_ty, "out", [], t.dims, t.scalars, "global")
    top: list = []
    t.acc(node, t.env, out_acc, top, "host")
    big = [b.name for b in t.buffers if b.elems >= (1 << 31)]
    if big or _max_extent(top) >= (1 << 31):
        # every index is computed in 32-bit int arithmetic
        raise TranslateError(f"arrays or loops of 2^31 elements or more ({big or 'a loop'})")
    types = {b.name: b.ctype for b in t.buffers}
    _collect_types(top, types)
    if optimise:
        top = passes.optimise(top, {b.name for b in t.buffers if b.kind == "in"},
                              _streamed(t.buffers, t.dims), types, t.fresh)
        _collect_types(top, types)
    kernels = _split(top, name)
    src = _emit(kernels, t.buffers, types)
    return Program(src, kernels, t.buffers, out_ty, types, dict(t.dims))


def _max_extent(cmds) -> int:
    m = 0
    for c in cmds:
        if isinstance(c, Decl):
            m = max(m, c.size)
        elif isinstance(c, (For, ParFor)):
            m = max(m, c.n, _max_extent(c.body))
    return m


def _collect_types(cmds, types):
    for c in cmds:
        if isinstance(c, (Decl, ir.Load, ir.VLoad)):
            types[c.name] = c.ctype
        elif isinstance(c, (For, ParFor, ir.Lanes)):
            _collect_types(c.body, types)
        elif isinstance(c, ir.Blocked):
            _collect_types(c.main + c.tail, types)


def _split(top: list, name: str) -> List[Kernel]:
    kernels: List[Kernel] = []
    seq: list = []

    def flush():
        if seq:
            kernels.append(Kernel(f"{name}_k{len(kernels)}", "single", list(seq), 1, 1))
            seq.clear()
    for c in top:
        if isinstance(c, ParFor) and c.level in ("workgroup", "global"):
            flush()
            kernels.append(Kernel(f"{name}_k{len(kernels)}", c.level, [c], c.n,
                                  _local_width(c.body)))
        elif isinstance(c, Decl) and c.space == "global":
            continue
        else:
            seq.append(c)
    flush()
    return kernels


def _local_width(body) -> int:
    """Work-items per work-group: enough for the widest coarsened mapLocal
    (Lanes), else for the widest mapLocal.  Other mapLocal loops are
    block-stride loops and run with any width."""
    plain, coarse = [1], [0]

    def walk(cmds):
        for c in cmds:
            if isinstance(c, ir.Lanes):
                coarse[0] = max(coarse[0], c.n // c.lanes)
                walk(c.body)
            elif isinstance(c, ParFor):
                if c.level == "local":
                    plain[0] = max(plain[0], c.n)
                walk(c.body)
            elif isinstance(c, For):
                walk(c.body)
            elif isinstance(c, ir.Blocked):
                walk(c.main + c.tail)
    walk(body)
    return coarse[0] if coarse[0] else plain[0]


def block_size(k: Kernel) -> int:
    if k.kind == "single":
        return 1
    if k.kind == "global":
        return 256
    w = min(1024, k.local_width)
    return max(64, -(-w // 64) * 64)


def grid_size(k: Kernel, cus: int = 256) -> int:
    if k.kind == "single":
        return 1
    if k.kind == "global":
        return max(1, min(-(-k.iterations // 256), cus * 8))
    per_cu = max(1, 2048 // block_size(k))
    return max(1, min(k.iterations, cus * per_cu))


def _has_local_loop(body) -> bool:
    for c in body:
        if isinstance(c, ir.Lanes) or (isinstance(c, ParFor) and c.level == "local"):
            return True
        if isinstance(c, (For, ParFor)) and _has_local_loop(c.body):
            return True
    return False


# Large one-dimensional inputs (vectors of at least STREAM_BYTES) are read
# with non-temporal loads; matrices and small vectors with cached loads.  This
# is the policy measured best for the hand-written kernels (streamed dot
# operands non-temporal, the rows of a binary32 gemv cached).
STREAM_BYTES = 64 << 20
_SIZE = {"float": 4, "unsigned": 4, "double": 8, "unsigned short": 2, "unsigned char": 1}


def _streamed(buffers: List[Buffer], dims: Dict[str, tuple]) -> set:
    return {b.name for b in buffers
            if b.kind == "in" and len(dims.get(b.name, ())) == 1
            and b.elems * _SIZE.get(b.ctype, 4) >= STREAM_BYTES}


def _emit(kernels: List[Kernel], buffers: List[Buffer], types: Dict[str, str]) -> str:
    lines = ["#include <hip/hip_runtime.h>",
             "// generated from a DPIA expression: one operation per node, no contraction",
             "#pragma clang fp contract(off)", "", ir.DECODERS]
    params = ", ".join((f"const {b.ctype}* __restrict__ {b.name}" if b.kind == "in"
                        else f"{b.ctype}* {b.name}") for b in buffers)
    for k in kernels:
        body: List[str] = []
        shared: List[str] = []
        _emit_block(k.body, body, shared, 1, types)
        lines.append(f'extern "C" __global__ void __launch_bounds__({block_size(k)}) '
                     f"{k.name}({params}) {{")
        lines.extend("  " + s for s in shared)
        lines.extend(body)
        lines.append("}")
        lines.append("")
    return "\n".join(lines)


_VEC = {("float", 4): "dpia_f4", ("unsigned", 4): "dpia_u4", ("unsigned short", 4): "dpia_h4",
        ("unsigned short", 8): "dpia_h8", ("unsigned char", 4): "dpia_b4",
        ("unsigned char", 8): "dpia_b8", ("unsigned char", 16): "dpia_b16"}


def _emit_block(cmds, out: List[str], shared: List[str], depth: int, types: Dict[str, str]):
    pad = "  " * depth
    for c in cmds:
        if isinstance(c, Decl):
            if c.space == "local":
                shared.append(f"__shared__ {c.ctype} {c.name}[{max(1, c.size)}];")
            elif c.size:
                out.append(f"{pad}{c.ctype} {c.name}[{c.size}];")
            else:
                out.append(f"{pad}{c.ctype} {c.name};")
        elif isinstance(c, Assign):
            lv = c.name if c.idx is None else f"{c.name}[{ir.ix_c(c.idx)}]"
            rhs = ir.ex_c(c.rhs, types)
            if c.ctx == "group" and c.space in ("local", "global"):
                # work-group-level code runs in every work-item; one writes
                out.append(f"{pad}if (threadIdx.x == 0) {lv} = {rhs};")
                out.append(f"{pad}__syncthreads();")
            else:
                out.append(f"{pad}{lv} = {rhs};")
        elif isinstance(c, ir.Load):
            elem = f"{c.buf}[{ir.ix_c(c.idx)}]"
            if c.nt:
                elem = f"__builtin_nontemporal_load(&{elem})"
            out.append(f"{pad}const {c.ctype} {c.name} = {elem};")
        elif isinstance(c, ir.VLoad):
            vt = _VEC[(c.ctype, c.width)]
            ptr = f"reinterpret_cast<const {vt}*>({c.buf} + {ir.ix_c(c.idx)})"
            val = f"__builtin_nontemporal_load({ptr})" if c.nt else f"*{ptr}"
            out.append(f"{pad}const {vt} {c.name} = {val};")
        elif isinstance(c, ir.SchedBarrier):
            out.append(f"{pad}__builtin_amdgcn_sched_barrier(0);   // the loads above first")
        elif isinstance(c, ir.Blocked):
            out.append(f"{pad}int {c.var} = 0;")
            out.append(f"{pad}for (; {c.var} + {c.step} <= {c.n}; {c.var} += {c.step}) {{")
            _emit_block(c.main, out, shared, depth + 1, types)
            out.append(f"{pad}}}")
            out.append(f"{pad}for (; {c.var} < {c.n}; ++{c.var}) {{")
            _emit_block(c.tail, out, shared, depth + 1, types)
            out.append(f"{pad}}}")
        elif isinstance(c, For):
            out.append(f"{pad}for (int {c.var} = 0; {c.var} < {c.n}; ++{c.var}) {{")
            _emit_block(c.body, out, shared, depth + 1, types)
            if _has_local_loop(c.body):
                # a work-group-level loop around mapLocal: the next iteration
                # may overwrite local memory this one still reads
                out.append(f"{pad}  __syncthreads();")
            out.append(f"{pad}}}")
        elif isinstance(c, ir.Lanes):
            out.append(f"{pad}for (int {c.var} = threadIdx.x * {c.lanes}; {c.var} < {c.n};"
                       f" {c.var} += blockDim.x * {c.lanes}) {{")
            _emit_block(c.body, out, shared, depth + 1, types)
            out.append(f"{pad}}}")
            out.append(f"{pad}__syncthreads();")
        elif isinstance(c, ParFor):
            v, n = c.var, c.n
            if c.level == "workgroup":
                out.append(f"{pad}for (int {v} = blockIdx.x; {v} < {n}; {v} += gridDim.x) {{")
                _emit_block(c.body, out, shared, depth + 1, types)
                out.append(f"{pad}  __syncthreads();")
                out.append(f"{pad}}}")
            elif c.level == "local":
                out.append(f"{pad}for (int {v} = threadIdx.x; {v} < {n}; {v} += blockDim.x) {{")
                _emit_block(c.body, out, shared, depth + 1, types)
                out.append(f"{pad}}}")
                out.append(f"{pad}__syncthreads();")
            else:
                out.append(f"{pad}for (int {v} = blockIdx.x * blockDim.x + threadIdx.x; {v} < {n};"
                           f" {v} += gridDim.x * blockDim.x) {{")
                _emit_block(c.body, out, shared, depth + 1, types)
                out.append(f"{pad}}}")
        else:
            raise TranslateError(f"unknown command {c!r}")
