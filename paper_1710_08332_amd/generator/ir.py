"""The imperative program the translation produces.

Index expressions (``IX``) are integer arithmetic over loop variables;
scalar expressions (``Ex``) are the numeric operations of the expression,
one node per operation; commands are declarations, assignments, sequential
loops and parallel loops.  ``emit_c`` renders an expression as C.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Tuple, Union


# ------------------------------------------------------------------ indices

@dataclass(frozen=True)
class IConst:
    v: int


@dataclass(frozen=True)
class IVar:
    name: str


@dataclass(frozen=True)
class IBin:
    op: str                    # "+", "*", "/", "%" (operands are never negative)
    a: "IX"
    b: "IX"


IX = Union[IConst, IVar, IBin]


def ix(v) -> IX:
    if isinstance(v, int):
        return IConst(v)
    if isinstance(v, str):
        return IVar(v)
    return v


def iadd(a, b) -> IX:
    a, b = ix(a), ix(b)
    if isinstance(a, IConst) and a.v == 0:
        return b
    if isinstance(b, IConst) and b.v == 0:
        return a
    if isinstance(a, IConst) and isinstance(b, IConst):
        return IConst(a.v + b.v)
    return IBin("+", a, b)


def imul(a, b) -> IX:
    a, b = ix(a), ix(b)
    if isinstance(b, IConst) and b.v == 1:
        return a
    if isinstance(a, IConst) and a.v == 1:
        return b
    if (isinstance(a, IConst) and a.v == 0) or (isinstance(b, IConst) and b.v == 0):
        return IConst(0)
    if isinstance(a, IConst) and isinstance(b, IConst):
        return IConst(a.v * b.v)
    return IBin("*", a, b)


def idiv(a, k: int) -> IX:
    a = ix(a)
    if k == 1:
        return a
    if isinstance(a, IConst):
        return IConst(a.v // k)
    return IBin("/", a, IConst(k))


def imod(a, k: int) -> IX:
    a = ix(a)
    if k == 1:
        return IConst(0)
    if isinstance(a, IConst):
        return IConst(a.v % k)
    return IBin("%", a, IConst(k))


def ix_c(e: IX) -> str:
    if isinstance(e, IConst):
        return str(e.v)
    if isinstance(e, IVar):
        return e.name
    return f"({ix_c(e.a)} {e.op} {ix_c(e.b)})"


# ------------------------------------------------------------------ numbers

@dataclass(frozen=True)
class Lit:
    value: Union[int, float]
    ctype: str                 # "float", "double", "unsigned"


@dataclass(frozen=True)
class Ref:
    """Element ``idx`` of array ``name``, or the private number ``name``."""
    name: str
    idx: Optional[IX]


@dataclass(frozen=True)
class Bin:
    op: str                    # "+", "-", "*", "/"
    a: "Ex"
    b: "Ex"


@dataclass(frozen=True)
class Un:
    op: str                    # "neg", "abs"
    a: "Ex"


@dataclass(frozen=True)
class Cast:
    ctype: str
    a: "Ex"


@dataclass(frozen=True)
class Select:
    """options[sel] for an index expression sel in [0, len(options))."""
    sel: IX
    options: Tuple["Ex", ...]


@dataclass(frozen=True)
class Decode:
    """The binary32 value of a storage code: "bf16" or "fp8" (OCP E4M3)."""
    fmt: str
    a: "Ex"


Ex = Union[Lit, Ref, Bin, Un, Cast, Select, Decode]

# Device functions the emitted code may call.  bfloat16 is the upper half of
# a binary32.  OCP fp8 E4M3 (sign bit, 4 exponent bits with bias 7, 3
# mantissa bits, subnormals m * 2^-9 at exponent 0, S.1111.111 NaN, no
# infinities) is decoded by gfx950's converter, one instruction; the tests
# check it against the format definition for every code.
DECODERS = """typedef float dpia_f4 __attribute__((ext_vector_type(4)));
typedef unsigned dpia_u4 __attribute__((ext_vector_type(4)));
typedef unsigned short dpia_h4 __attribute__((ext_vector_type(4)));
typedef unsigned short dpia_h8 __attribute__((ext_vector_type(8)));
typedef unsigned char dpia_b4 __attribute__((ext_vector_type(4)));
typedef unsigned char dpia_b8 __attribute__((ext_vector_type(8)));
typedef unsigned char dpia_b16 __attribute__((ext_vector_type(16)));
__device__ __forceinline__ float dpia_bf16(unsigned short c) {
  return __uint_as_float(static_cast<unsigned>(c) << 16);
}
__device__ __forceinline__ float dpia_fp8(unsigned char c) {
  return __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(c), 0);
}
"""


def ex_c(e: Ex, types: dict) -> str:
    """C text of e.  ``types`` maps array and variable names to C types
    (needed to pick fabsf or fabs)."""
    if isinstance(e, Lit):
        if e.ctype == "unsigned":
            return f"{int(e.value) % (1 << 32)}u"
        t = repr(float(e.value))
        if t in ("inf", "-inf", "nan"):
            raise ValueError("non-finite literal")
        return t + ("f" if e.ctype == "float" else "")
    if isinstance(e, Ref):
        return e.name if e.idx is None else f"{e.name}[{ix_c(e.idx)}]"
    if isinstance(e, Bin):
        return f"({ex_c(e.a, types)} {e.op} {ex_c(e.b, types)})"
    if isinstance(e, Un):
        if e.op == "neg":
            return f"(-{ex_c(e.a, types)})"
        fn = "__builtin_fabsf" if ex_type(e.a, types) == "float" else "__builtin_fabs"
        return f"{fn}({ex_c(e.a, types)})"
    if isinstance(e, Cast):
        return f"(({e.ctype}){ex_c(e.a, types)})"
    if isinstance(e, Decode):
        return f"dpia_{e.fmt}({ex_c(e.a, types)})"
    code = ex_c(e.options[-1], types)
    for k in range(len(e.options) - 2, -1, -1):
        code = f"({ix_c(e.sel)} == {k} ? {ex_c(e.options[k], types)} : {code})"
    return code


def ex_type(e: Ex, types: dict) -> str:
    if isinstance(e, Lit):
        return e.ctype
    if isinstance(e, Ref):
        return types[e.name]
    if isinstance(e, (Bin,)):
        return ex_type(e.a, types)
    if isinstance(e, Un):
        return ex_type(e.a, types)
    if isinstance(e, Cast):
        return e.ctype
    if isinstance(e, Decode):
        return "float"
    return ex_type(e.options[0], types)


# ------------------------------------------------------------------ commands

@dataclass
class Decl:
    name: str
    ctype: str
    size: int                  # 0: one number
    space: str                 # "private", "local" or "global"


@dataclass
class Assign:
    name: str                  # target array or private number
    idx: Optional[IX]
    rhs: Ex
    space: str                 # where the target lives
    ctx: str                   # "host", "group" or "item": where this runs


@dataclass
class For:
    var: str
    n: int
    body: List[object]


@dataclass
class ParFor:
    level: str                 # "workgroup", "local" or "global"
    var: str
    n: int
    body: List[object]


@dataclass
class Load:
    """A private constant ``name`` = buf[idx] (non-temporal if ``nt``)."""
    name: str
    ctype: str
    buf: str
    idx: IX
    nt: bool = False


@dataclass
class VLoad:
    """A private vector ``name`` = buf[idx .. idx + width - 1], read at once
    (at most 16 bytes); idx is a multiple of width.  Its components are
    Ref(name, IConst(j))."""
    name: str
    ctype: str
    buf: str
    idx: IX
    nt: bool = False
    width: int = 4


@dataclass
class SchedBarrier:
    """Keeps the loads before it ahead of the code after it (scheduling only)."""


@dataclass
class Blocked:
    """``for var in 0, step, ...`` while var + step <= n, running ``main``
    (which covers iterations var .. var + step - 1), then ``tail`` for each
    remaining var < n."""
    var: str
    n: int
    step: int
    main: List[object]
    tail: List[object]


@dataclass
class Lanes:
    """A mapLocal loop run ``lanes`` adjacent iterations per work-item: for
    base = lanes * work-item, base < n, base += lanes * work-items, ``body``
    (which covers iterations base .. base + lanes - 1)."""
    var: str
    n: int
    lanes: int
    body: List[object]


Cmd = Union[Decl, Assign, For, ParFor, Load, VLoad, SchedBarrier, Blocked, Lanes]
