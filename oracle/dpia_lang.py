"""Abstract syntax, parser and printer for the functional DPIA sub-language.

The language is the purely functional fragment of DPIA (Sec. 3, "DPIA's
functional sub-language"): a typed lambda calculus over ``num``, arrays and
pairs, with the primitives of Fig. 5a and the OpenCL strategy primitives of
Sec. 6.1.  Size and type arguments are left implicit, as the paper notes they
usually can be (Sec. 3.3, dot-product example); the only size that is written
is the row length of ``split``.

Concrete syntax (S-expressions)::

    expr ::= NUMBER                   numeric literal (Fig. 5a, "n")
           | IDENT                    variable
           | (lam (x1 ... xk) expr)   lambda abstraction
           | (PRIM expr ...)          primitive application
           | (expr expr ...)          application of a function expression

Primitives and arities (``F`` marks a function argument):

    Fig. 5a:  map F e | reduce F init e | zip a b | split n e | join e
              pair a b | fst e | snd e | + a b | - a b | * a b | / a b
              negate a
    Sec. 6.1: mapGlobal, mapWorkgroup, mapLocal, mapSeq (same type as map)
              reduceSeq (same type as reduce; sequential by definition)
              toGlobal F, toLocal F, toPrivate F (wrap a function)
    Sec. 6.1 vector types:
              asVector n e   m*n.num -> m.num<n> (a split whose rows are
                             vectors: element i is elements i*n .. i*n+n-1)
              asScalar n e   m.num<n> -> m*n.num (element i is component
                             i mod n of vector i div n)
              Arithmetic and abs on two vectors of one type act on each
              component.  ``broadcast n a`` is the vector of n copies of the
              number a: the vector zero that a vector accumulator starts
              from, which the paper writes as 0 (OpenCL's (float4)(0)).
    Extensions that the paper's dot/asum/gemv benchmarks need but Fig. 5a
    does not define (each one is a plain total function):
              abs a          absolute value (asum, Sec. 7.1 benchmark list)
              transpose e    m.n.d -> n.m.d; the strided per-lane order
              f32 a / f64 a  conversion between binary32 and binary64
              bf16 a / fp8 a decode a bf16 / OCP fp8-e4m3 storage code
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Tuple, Union

# name -> number of arguments
PRIMS = {
    "map": 2, "mapGlobal": 2, "mapWorkgroup": 2, "mapLocal": 2, "mapSeq": 2,
    "reduce": 3, "reduceSeq": 3,
    "zip": 2, "split": 2, "join": 1, "transpose": 1,
    "pair": 2, "fst": 1, "snd": 1,
    "+": 2, "-": 2, "*": 2, "/": 2, "negate": 1, "abs": 1,
    "toGlobal": 1, "toLocal": 1, "toPrivate": 1,
    "f32": 1, "f64": 1, "bf16": 1, "fp8": 1,
    "asVector": 2, "asScalar": 2, "broadcast": 2,
}

# primitives whose first argument is a literal size
SIZED = ("split", "asVector", "asScalar", "broadcast")

MAP_LIKE = ("map", "mapGlobal", "mapWorkgroup", "mapLocal", "mapSeq")
REDUCE_LIKE = ("reduce", "reduceSeq")
ADDRESS_SPACE = ("toGlobal", "toLocal", "toPrivate")


@dataclass(frozen=True)
class Lit:
    text: str


@dataclass(frozen=True)
class Var:
    name: str


@dataclass(frozen=True)
class Lam:
    params: Tuple[str, ...]
    body: "Expr"


@dataclass(frozen=True)
class Prim:
    name: str
    args: Tuple["Expr", ...]


@dataclass(frozen=True)
class App:
    fn: "Expr"
    args: Tuple["Expr", ...]


Expr = Union[Lit, Var, Lam, Prim, App]


class ParseError(ValueError):
    pass


def _tokenize(text: str):
    out = []
    i = 0
    while i < len(text):
        ch = text[i]
        if ch.isspace():
            i += 1
        elif ch == ";":  # comment to end of line
            while i < len(text) and text[i] != "\n":
                i += 1
        elif ch in "()":
            out.append(ch)
            i += 1
        else:
            j = i
            while j < len(text) and not text[j].isspace() and text[j] not in "();":
                j += 1
            out.append(text[i:j])
            i = j
    return out


def _is_number(tok: str) -> bool:
    try:
        float(tok)
        return True
    except ValueError:
        return False


def parse(text: str) -> Expr:
    toks = _tokenize(text)
    pos = 0

    def expr():
        nonlocal pos
        if pos >= len(toks):
            raise ParseError("unexpected end of input")
        tok = toks[pos]
        pos += 1
        if tok == ")":
            raise ParseError("unexpected ')'")
        if tok != "(":
            if _is_number(tok):
                return Lit(tok)
            if tok in PRIMS or tok == "lam":
                raise ParseError(f"keyword {tok!r} used as a value")
            return Var(tok)
        if pos >= len(toks):
            raise ParseError("unexpected end of input")
        head = toks[pos]
        if head == "lam":
            pos += 1
            if toks[pos] != "(":
                raise ParseError("lam needs a parameter list")
            pos += 1
            params = []
            while toks[pos] != ")":
                params.append(toks[pos])
                pos += 1
            pos += 1
            body = expr()
            _close()
            if not params:
                raise ParseError("lam with no parameters")
            return Lam(tuple(params), body)
        if head in PRIMS:
            pos += 1
            args = []
            while toks[pos] != ")":
                args.append(expr())
            pos += 1
            if len(args) != PRIMS[head]:
                raise ParseError(f"{head} takes {PRIMS[head]} arguments, got {len(args)}")
            if head in SIZED and not isinstance(args[0], Lit):
                raise ParseError(f"{head} needs a literal size")
            return Prim(head, tuple(args))
        fn = expr()
        args = []
        while toks[pos] != ")":
            args.append(expr())
        pos += 1
        if not args:
            raise ParseError("application with no arguments")
        return App(fn, tuple(args))

    def _close():
        nonlocal pos
        if pos >= len(toks) or toks[pos] != ")":
            raise ParseError("expected ')'")
        pos += 1

    e = expr()
    if pos != len(toks):
        raise ParseError("trailing tokens after expression")
    return e


def to_text(e: Expr) -> str:
    if isinstance(e, Lit):
        return e.text
    if isinstance(e, Var):
        return e.name
    if isinstance(e, Lam):
        return f"(lam ({' '.join(e.params)}) {to_text(e.body)})"
    if isinstance(e, Prim):
        return "(" + " ".join([e.name] + [to_text(a) for a in e.args]) + ")"
    if isinstance(e, App):
        return "(" + " ".join([to_text(e.fn)] + [to_text(a) for a in e.args]) + ")"
    raise TypeError(f"not an expression: {e!r}")
