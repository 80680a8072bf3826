"""Front end: expression text -> typed AST, and the nesting rules.

Concrete syntax (S-expressions, the same text format the library's tests
use): a number literal, a name, ``(lam (x ...) body)``, ``(prim arg ...)``
or ``(f arg ...)``.  Size arguments are literals: ``(split n e)``,
``(asVector n e)``, ``(asScalar n e)``, ``(broadcast n e)``.

Types: ``Num(c)`` a scalar of C type c ("float", "double", "unsigned", or the
storage codes "unsigned short" of bf16 and "unsigned char" of OCP fp8-e4m3,
which ``bf16`` / ``fp8`` decode exactly to float and nothing else accepts),
``Vec(n, c)`` an OpenCL-style vector (Sec. 6.1), ``Arr(n, t)`` and
``Pair(a, b)`` (Sec. 5.1).  Functions are not first-class data: every lambda
is applied where it appears (as the argument of map / reduce / toX, or in a
direct application), which is all the strategies need.

Nesting (Sec. 6.1: the hierarchy primitives must follow OpenCL's levels):
mapGlobal and mapWorkgroup only outside every parallel map, mapLocal only
directly inside a mapWorkgroup (never inside another mapLocal, a mapGlobal
or a sequential loop that is itself inside a work-item), and nothing
parallel inside mapSeq / reduceSeq / map / reduce bodies that run per
work-item.  ``check`` rejects every other nesting with ``CheckError``.
"""

from __future__ import annotations

import re
from dataclasses import dataclass
from typing import Dict, List, Tuple, Union


class ParseError(ValueError):
    pass


class CheckError(ValueError):
    pass


# ------------------------------------------------------------------ AST

@dataclass(frozen=True)
class Num:
    c: str                       # "float", "double" or "unsigned"


@dataclass(frozen=True)
class Vec:
    n: int
    c: str


@dataclass(frozen=True)
class Arr:
    n: int
    elem: "Type"


@dataclass(frozen=True)
class Pair:
    a: "Type"
    b: "Type"


Type = Union[Num, Vec, Arr, Pair]


@dataclass(frozen=True)
class Lit:
    text: str


@dataclass(frozen=True)
class Name:
    id: str


@dataclass(frozen=True)
class Lam:
    params: Tuple[str, ...]
    body: "Node"


@dataclass(frozen=True)
class Call:
    """A primitive (head is a str) or the application of a lambda / name."""
    head: Union[str, "Node"]
    args: Tuple["Node", ...]


Node = Union[Lit, Name, Lam, Call]

ARITY = {
    "map": 2, "mapSeq": 2, "mapGlobal": 2, "mapWorkgroup": 2, "mapLocal": 2,
    "reduce": 3, "reduceSeq": 3,
    "zip": 2, "split": 2, "join": 1, "transpose": 1, "pair": 2, "fst": 1, "snd": 1,
    "asVector": 2, "asScalar": 2, "broadcast": 2,
    "+": 2, "-": 2, "*": 2, "/": 2, "negate": 1, "abs": 1, "f32": 1, "f64": 1,
    "bf16": 1, "fp8": 1,
    "toGlobal": 1, "toLocal": 1, "toPrivate": 1,
}
MAPS = ("map", "mapSeq", "mapGlobal", "mapWorkgroup", "mapLocal")
REDUCES = ("reduce", "reduceSeq")
SPACES = ("toGlobal", "toLocal", "toPrivate")
SIZED = ("split", "asVector", "asScalar", "broadcast")

_TOKEN = re.compile(r"\s*(?:;[^\n]*\n?\s*)*([()]|[^\s();]+)")


def parse(text: str) -> Node:
    toks: List[str] = []
    pos = 0
    while True:
        m = _TOKEN.match(text, pos)
        if not m:
            break
        toks.append(m.group(1))
        pos = m.end()
    if text[pos:].strip() and not text[pos:].lstrip().startswith(";"):
        raise ParseError(f"cannot read {text[pos:pos + 20]!r}")
    stack: List[list] = [[]]
    for t in toks:
        if t == "(":
            stack.append([])
        elif t == ")":
            if len(stack) == 1:
                raise ParseError("unbalanced ')'")
            items = stack.pop()
            stack[-1].append(items)
        else:
            stack[-1].append(t)
    if len(stack) != 1 or len(stack[0]) != 1:
        raise ParseError("expected exactly one expression")
    return _build(stack[0][0])


def _is_num(t: str) -> bool:
    try:
        float(t)
        return True
    except ValueError:
        return False


def _build(s) -> Node:
    if isinstance(s, str):
        if _is_num(s):
            return Lit(s)
        if s in ARITY or s == "lam":
            raise ParseError(f"{s!r} is not a value")
        return Name(s)
    if not s:
        raise ParseError("empty application")
    head = s[0]
    if head == "lam":
        if len(s) != 3 or not isinstance(s[1], list) or not s[1]:
            raise ParseError("lam takes a parameter list and a body")
        return Lam(tuple(s[1]), _build(s[2]))
    args = tuple(_build(a) for a in s[1:])
    if isinstance(head, str) and head in ARITY:
        if len(args) != ARITY[head]:
            raise ParseError(f"{head} takes {ARITY[head]} arguments, got {len(args)}")
        if head in SIZED and not (isinstance(args[0], Lit) and args[0].text.isdigit()):
            raise ParseError(f"{head} needs a literal size")
        return Call(head, args)
    return Call(_build(head), args)


# ------------------------------------------------------------------ nesting

# Contexts: "host" (outside every parallel map), "hostseq" (inside a
# sequential loop of host-level code, which runs as one work-item), "group"
# (inside a mapWorkgroup body, outside any mapLocal: code that every
# work-item of the work-group runs alike, sequential loops included) and
# "item" (inside a mapLocal or mapGlobal body).
def check(node: Node) -> None:
    """Raises CheckError where a parallel map is nested illegally."""
    _check(node, "host")


def _check(n: Node, ctx: str) -> None:
    if isinstance(n, (Lit, Name)):
        return
    if isinstance(n, Lam):
        _check(n.body, ctx)
        return
    if not isinstance(n.head, str):
        _check(n.head, ctx)
        for a in n.args:
            _check(a, ctx)
        return
    h = n.head
    if h in ("mapWorkgroup", "mapGlobal"):
        if ctx != "host":
            raise CheckError(f"{h} must not be nested inside another map or a sequential "
                             f"loop (found in {ctx} code)")
        _check(n.args[1], ctx)
        _check(n.args[0], "group" if h == "mapWorkgroup" else "item")
        return
    if h == "mapLocal":
        if ctx != "group":
            raise CheckError(f"mapLocal must be inside a mapWorkgroup and outside every "
                             f"mapLocal and mapGlobal (found in {ctx} code)")
        _check(n.args[1], ctx)
        _check(n.args[0], "item")
        return
    if h in ("map", "mapSeq") or h in REDUCES:
        for a in n.args[1:]:
            _check(a, ctx)
        _check(n.args[0], "hostseq" if ctx == "host" else ctx)
        return
    for a in n.args:
        _check(a, ctx)
