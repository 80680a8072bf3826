"""DPIA expressions for the dot / asum / gemv strategy families.

Each builder returns the text of one functional DPIA expression; its value
under the semantics of Secs. 4.2 and 5.1 (evaluated by ``eval_numpy`` or
``eval_scalar``) is what a kernel running that strategy must produce bit for
bit.

The shape follows the blocked dot product of Sec. 2.1, eq. (2): the input is
split into chunks of W elements, one chunk per work-group (mapWorkgroup);
each chunk is split into L rows of C elements, one row per local work-item
(mapLocal), and every work-item folds its row sequentially (reduceSeq) with
the fused operator ``lam x a. (fst x * snd x) + a``.  Two readings of the
printed equation are needed and are taken here:

* eq. (2) applies ``split 2048`` to a single element and sizes the chunk as
  2048*128; the reading used is that ``split n`` makes rows of length n
  (its type in Fig. 5a, nm.d -> m.n.d), so a chunk is ``split C`` into L
  rows of C: W = L*C.
* the per-work-group results must be combined.  Eq. (2) leaves them to the
  outer ``reduce``; here each chunk first combines its L lane results inside
  the work-group, either with a sequential ``reduceSeq`` ("seq") or with a
  binary tree in local memory ("tree": log2 L levels of
  ``mapLocal (reduceSeq add 0) (split 2 v)``, leaves in lane order, built
  from Fig. 5a primitives only), and the G chunk results are then folded by
  a sequential ``reduceSeq`` from +0 in chunk order (the final loop of the
  blocked listing in Sec. 2.2).

Strided lane order: the contiguous strategy gives work-item l the elements
l*C .. l*C + C-1 of its chunk.  The strided strategy gives it elements
l, l+L, l+2L, ..., expressed as ``transpose (split L ch)`` (an extension: a
layout primitive that swaps the two outer indices).  The test suite checks
it against the same order written with Fig. 5a primitives alone (a reduce
whose accumulator is an array of L lanes, as in the vector accumulators of
the dot kernel of Sec. 6.2).

asum uses ``lam x a. abs x + a``; the paper benchmarks asum (Sec. 7.1) but
Fig. 5a has no absolute value, so ``abs`` is an added scalar primitive.

gemv (y = A x, the BLAS operation with alpha = 1, beta = 0): rows are grouped
R per work-group and every row is reduced with the same lane / combine
strategy as a dot product of that row with x.  With two row parts, each half
row is reduced on its own and the two halves are folded by
``reduceSeq add 0``.

Vector strategies (Sec. 6.1 vectorisation; the dot expression of Sec. 6.2 is
one): with vector width V > 1 the inputs are read through ``asVector V``, so
the strategy works on vectors of V consecutive elements.  Each work-item
keeps a vector accumulator (from ``broadcast V 0``) and every operation acts
on each component, so component j of a lane folds elements j, j+V, ... of
the lane's vectors.  The combine acts per component too; ``asScalar V``
turns the chunks' vector values back into V numbers each, in component
order, before the outer fold.  The Sec. 6.2 expression has no work-group
combine at all: every work-item's value is written out.  Combine "none" is
that form: the chunk's value is its L lane values (join of the mapLocal), so
the outer fold runs over G*L (times V) numbers in chunk, lane, component
order.

A second compensated variant ("sum2") follows Ogita, Rump and Oishi's Sum2:
TwoSum at every step, the exact errors summed into c, value s + c; unlike
Kahan's step it keeps the error when a term outweighs the running sum.

The compensated ("kahan") variant keeps a pair (s, c) per accumulator:
Kahan's summation step (N. J. Higham, Accuracy and Stability of Numerical
Algorithms, 2nd ed., Alg. 4.2) inside the lanes, Knuth's TwoSum to merge two
pairs in the combines, and optionally a binary64 final fold of s - c.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .eval_numpy import evaluate

ADD = "(lam (e a) (+ e a))"
MUL_ADD = "(lam (z a) (+ (* (fst z) (snd z)) a))"
ABS_ADD = "(lam (e a) (+ (abs e) a))"

# Kahan step on acc = (s, c) with element z = (x, y):
#   y' = x*y - c ; t = s + y' ; new acc = (t, (t - s) - y')
KAHAN_MUL_STEP = ("(lam (z acc) ((lam (yk) ((lam (t) (pair t (- (- t (fst acc)) yk)))"
                  " (+ (fst acc) yk))) (- (* (fst z) (snd z)) (snd acc))))")

# Merge of an earlier pair l = (s1, c1) with a later pair r = (s2, c2), by
# TwoSum: s = s1 + s2 ; bp = s - s1 ; e = (s1 - (s - bp)) + (s2 - bp) ;
# new pair (s, (c1 + c2) - e).  Element first, accumulator second.
KAHAN_MERGE = ("(lam (r l) ((lam (s) ((lam (bp) (pair s (- (+ (snd l) (snd r))"
               " (+ (- (fst l) (- s bp)) (- (fst r) bp))))) (- s (fst l))))"
               " (+ (fst l) (fst r))))")

ZERO_PAIR = "(pair 0 0)"

# Sum2 (T. Ogita, S. M. Rump, S. Oishi, "Accurate sum and dot product", SIAM
# J. Sci. Comput. 26(6), 2005, Alg. 4.4) over the rounded products: the pair
# (s, c) has value s + c; each step adds the product p to s with TwoSum and
# adds the exact error to c:
#   p = x*y ; t = s + p ; bp = t - s ; new pair (t, c + ((s - (t - bp)) + (p - bp)))
SUM2_MUL_STEP = ("(lam (z acc) ((lam (p) ((lam (t) ((lam (bp) (pair t (+ (snd acc)"
                 " (+ (- (fst acc) (- t bp)) (- p bp))))) (- t (fst acc)))) (+ (fst acc) p)))"
                 " (* (fst z) (snd z))))")

# Merge of a later pair r into the earlier l: TwoSum of the s parts, the
# error joining the c parts: s = s_l + s_r ; bp = s - s_l ;
# new pair (s, (c_l + c_r) + ((s_l - (s - bp)) + (s_r - bp))).
SUM2_MERGE = ("(lam (r l) ((lam (s) ((lam (bp) (pair s (+ (+ (snd l) (snd r))"
              " (+ (- (fst l) (- s bp)) (- (fst r) bp))))) (- s (fst l))))"
              " (+ (fst l) (fst r))))")


@dataclass(frozen=True)
class Plan:
    """The oracle's reading of one strategy.

    seq (C)        elements folded sequentially by one work-item
    lanes (L)      work-items per chunk (mapLocal width)
    order          "contiguous" (rows of C) or "strided" (stride-L rows)
    combine        "tree" (pairwise in local memory) or "seq" (reduceSeq)
    accum          "plain", "kahan" or "sum2"
    final_f64      kahan / sum2 only: fold the chunk values in binary64
    rows (R)       gemv: rows per work-group
    row_parts      gemv: 1, or 2 halves reduced separately
    vec (V)        dot / asum: vector width of the asVector view (1: none)

    With vec = V the chunk holds L*C vectors, i.e. V*L*C numbers.
    """
    seq: int
    lanes: int
    order: str = "contiguous"
    combine: str = "tree"
    accum: str = "plain"
    final_f64: bool = False
    rows: int = 1
    row_parts: int = 1
    vec: int = 1

    @property
    def chunk(self) -> int:
        """Numbers per chunk."""
        return self.seq * self.lanes * self.vec

    def check(self):
        if self.seq < 1 or self.lanes < 1:
            raise ValueError("seq and lanes must be positive")
        if self.order not in ("contiguous", "strided"):
            raise ValueError(f"bad order {self.order!r}")
        if self.combine not in ("tree", "seq", "none"):
            raise ValueError(f"bad combine {self.combine!r}")
        if self.combine == "tree" and self.lanes & (self.lanes - 1):
            raise ValueError("a tree combine needs a power-of-two lane count")
        if self.accum not in ("plain", "kahan", "sum2"):
            raise ValueError(f"bad accum {self.accum!r}")
        if self.row_parts not in (1, 2):
            raise ValueError("row_parts must be 1 or 2")
        if self.vec < 1:
            raise ValueError("vec must be positive")
        if (self.vec > 1 or self.combine == "none") and self.accum != "plain":
            raise ValueError("vector and uncombined strategies are defined for plain accumulation")


def _rows_of(view: str, plan: Plan) -> str:
    if plan.order == "contiguous":
        return f"(split {plan.seq} {view})"
    return f"(transpose (split {plan.lanes} {view}))"


def _lanes(view: str, plan: Plan, step: str, init: str) -> str:
    """Arr(L): each work-item's sequential fold of its row of the chunk."""
    return (f"(mapLocal (toPrivate (lam (s) (reduceSeq {step} {init} s)))"
            f" {_rows_of(view, plan)})")


def _combine(lanes: str, plan: Plan, merge: str, init: str) -> str:
    """Fold the L lane results of one chunk into one value."""
    if plan.combine == "seq" or plan.lanes == 1:
        return f"(reduceSeq {merge} {init} {lanes})"
    v = lanes
    n = plan.lanes
    while n > 2:
        v = (f"((toLocal (lam (v) (mapLocal (lam (q) (reduceSeq {merge} {init} q))"
             f" (split 2 v)))) {v})")
        n //= 2
    return f"(reduceSeq {merge} {init} {v})"


def _chunk_value(view: str, plan: Plan, step: str) -> str:
    if plan.combine == "none":
        raise ValueError("an uncombined chunk has L values, not one")
    if plan.accum in ("kahan", "sum2"):
        merge = KAHAN_MERGE if plan.accum == "kahan" else SUM2_MERGE
        return _combine(_lanes(view, plan, step, ZERO_PAIR), plan, merge, ZERO_PAIR)
    return _combine(_lanes(view, plan, step, "0"), plan, ADD, "0")


def _final(partials: str, plan: Plan) -> str:
    if plan.accum == "sum2":
        if plan.final_f64:
            return (f"(reduceSeq (lam (p a) (+ (+ (f64 (fst p)) (f64 (snd p))) a))"
                    f" (f64 0) {partials})")
        return f"((lam (r) (+ (fst r) (snd r))) (reduceSeq {SUM2_MERGE} {ZERO_PAIR} {partials}))"
    if plan.accum == "kahan":
        if plan.final_f64:
            return (f"(reduceSeq (lam (p a) (+ (- (f64 (fst p)) (f64 (snd p))) a))"
                    f" (f64 0) {partials})")
        return f"((lam (r) (- (fst r) (snd r))) (reduceSeq {KAHAN_MERGE} {ZERO_PAIR} {partials}))"
    return f"(reduceSeq {ADD} 0 {partials})"


def _partials(n: int, view: str, plan: Plan, step: str) -> str:
    """The chunk values: what the mapWorkgroup level writes out."""
    plan.check()
    if n % plan.chunk:
        raise ValueError(f"n={n} is not a multiple of the chunk {plan.chunk}")
    V = plan.vec
    w = plan.seq * plan.lanes                    # elements (vectors if V > 1) per chunk
    zero = "0" if V == 1 else f"(broadcast {V} 0)"
    if plan.combine == "none":
        body = _lanes("ch", plan, step, zero)
        partials = f"(join (mapWorkgroup (lam (ch) {body}) (split {w} {view})))"
    elif V == 1:
        body = _chunk_value("ch", plan, step)
        partials = f"(mapWorkgroup (lam (ch) {body}) (split {w} {view}))"
    else:
        body = _combine(_lanes("ch", plan, step, zero), plan, ADD, zero)
        partials = f"(mapWorkgroup (lam (ch) {body}) (split {w} {view}))"
    if V > 1:
        partials = f"(asScalar {V} {partials})"
    return partials


def _reduction(n: int, view: str, plan: Plan, step: str) -> str:
    return _final(_partials(n, view, plan, step), plan)


def _vectors(name: str, plan: Plan) -> str:
    return name if plan.vec == 1 else f"(asVector {plan.vec} {name})"


def dot_expr(n: int, plan: Plan) -> str:
    """dot xs ys under ``plan``; inputs ``xs``, ``ys`` of length n."""
    step = {"kahan": KAHAN_MUL_STEP, "sum2": SUM2_MUL_STEP}.get(plan.accum, MUL_ADD)
    return _reduction(n, f"(zip {_vectors('xs', plan)} {_vectors('ys', plan)})", plan, step)


def dot_chunks_expr(n: int, plan: Plan) -> str:
    """The chunk values of dot xs ys under ``plan`` (the array the outer fold
    reads: one value per chunk, V per chunk for vector strategies, L*V for
    uncombined ones)."""
    if plan.accum != "plain":
        raise ValueError("chunk values are given for plain accumulation")
    return _partials(n, f"(zip {_vectors('xs', plan)} {_vectors('ys', plan)})", plan, MUL_ADD)


def asum_expr(n: int, plan: Plan) -> str:
    """sum of |xs[i]| under ``plan``; input ``xs`` of length n."""
    if plan.accum != "plain":
        raise ValueError("asum is defined for plain accumulation only")
    return _reduction(n, _vectors("xs", plan), plan, ABS_ADD)


def scal_expr() -> str:
    """scal (Sec. 7.1 benchmark): every element times the scalar input
    ``alpha``.  A map has no association to fix: whichever strategy places the
    elements on work-groups and work-items, element i is ``alpha * xs[i]``
    rounded once (the map law of Sec. 5.3), so the oracle is that map."""
    return "(map (lam (e) (* alpha e)) xs)"


def gemv_expr(m: int, k: int, plan: Plan, a_format: str = "f32") -> str:
    """y = A x under ``plan``; inputs ``A`` (m rows of k), ``x`` (k) and, for
    fp8, ``scale`` (m): row r is ``scale[r] * (row r of decoded A) . x``."""
    plan.check()
    if plan.accum != "plain":
        raise ValueError("gemv is defined for plain accumulation only")
    if plan.vec != 1 or plan.combine == "none":
        raise ValueError("gemv rows use scalar, combined strategies")
    if m % plan.rows:
        raise ValueError(f"m={m} is not a multiple of rows={plan.rows}")
    part = k // plan.row_parts
    if k % plan.row_parts or part != plan.chunk:
        raise ValueError(f"k={k} must equal row_parts*lanes*seq")

    def row_value(row: str) -> str:
        view = f"(zip {row} x)"
        if plan.row_parts == 1:
            return _chunk_value(view, plan, MUL_ADD)
        halves = f"(map (lam (h) {_chunk_value('h', plan, MUL_ADD)}) (split {part} {view}))"
        return f"(reduceSeq {ADD} 0 {halves})"

    if a_format == "f32":
        body = f"(map (lam (row) {row_value('row')}) rows)"
        src = "A"
    elif a_format in ("bf16", "fp8"):
        dec = f"(map (lam (c) ({a_format} c)) {{}})"
        if a_format == "bf16":
            body = f"(map (lam (row) {row_value(dec.format('row'))}) rows)"
            src = "A"
        else:
            body = (f"(map (lam (rw) (* (snd rw) {row_value(dec.format('(fst rw)'))}))"
                    f" rows)")
            src = "(zip A scale)"
    else:
        raise ValueError(f"bad a_format {a_format!r}")
    return f"(join (mapWorkgroup (lam (rows) {body}) (split {plan.rows} {src})))"


def gemv_blas_expr(m: int, k: int, plan: Plan, a_format: str = "f32",
                   beta_zero: bool = False) -> str:
    """The BLAS form y := alpha * (A x) + beta * y of the gemv benchmark
    (Sec. 7.1): a map over the rows' values zipped with the old ``y``, so
    every element is ``(alpha * v) + (beta * y)`` with each operation rounded
    once, where v is the row value of ``gemv_expr``.  When beta is zero the
    old y is not an input at all (the BLAS convention: y need not hold
    numbers then) and the element is ``alpha * v``."""
    rows = gemv_expr(m, k, plan, a_format)
    if beta_zero:
        return f"(map (lam (v) (* alpha v)) {rows})"
    return (f"(map (lam (p) (+ (* alpha (fst p)) (* beta (snd p)))) "
            f"(zip {rows} yin))")


# ------------------------------------------------------------------ running
#
# Lengths that the strategy's split does not divide.  Fig. 5a types split so
# that its argument's length is a multiple of the row length.  For a vector
# (or row) whose length is not a multiple of the chunk, the reading taken is
# that the strategy applies to the input extended with zeros up to the next
# multiple of the chunk (for gemv: of W * row parts).  For the plain
# operators this cannot change a result: a zero element contributes
# (0 * 0) + a or |0| + a, which equals a for every accumulator a a fold from
# +0 can hold (never -0).  Compensated (Kahan) accumulation is changed by
# extra zeros, so it is only defined for lengths the chunk divides.

def _zero_extend(v: np.ndarray, length: int, axis: int = -1) -> np.ndarray:
    v = np.asarray(v)
    pad = length - v.shape[axis]
    if pad == 0:
        return v
    if pad < 0:
        raise ValueError("cannot extend to a shorter length")
    width = [(0, 0)] * v.ndim
    width[axis] = (0, pad)
    return np.pad(v, width)


def extended_length(n: int, chunk: int) -> int:
    return -(-n // chunk) * chunk


def dot(xs: np.ndarray, ys: np.ndarray, plan: Plan, num: str = "f32"):
    n = extended_length(len(xs), plan.chunk)
    if n != len(xs) and plan.accum != "plain":
        raise ValueError("compensated accumulation needs n to be a multiple of the chunk")
    return evaluate(dot_expr(n, plan), {"xs": _zero_extend(xs, n), "ys": _zero_extend(ys, n)}, num)


def dot_chunks(xs: np.ndarray, ys: np.ndarray, plan: Plan, num: str = "f32"):
    n = extended_length(len(xs), plan.chunk)
    return evaluate(dot_chunks_expr(n, plan), {"xs": _zero_extend(xs, n),
                                               "ys": _zero_extend(ys, n)}, num)


def asum(xs: np.ndarray, plan: Plan, num: str = "f32"):
    n = extended_length(len(xs), plan.chunk)
    return evaluate(asum_expr(n, plan), {"xs": _zero_extend(xs, n)}, num)


def scal(alpha, xs: np.ndarray, num: str = "f32"):
    return evaluate(scal_expr(), {"alpha": np.asarray(alpha, np.float32 if num == "f32" else None),
                                  "xs": xs}, num)


def gemv(A: np.ndarray, x: np.ndarray, plan: Plan, a_format: str = "f32",
         scale: np.ndarray = None, num: str = "f32"):
    k = plan.chunk * plan.row_parts
    if A.shape[1] > k:
        raise ValueError(f"rows of {A.shape[1]} exceed W * row_parts = {k}")
    inputs = {"A": _zero_extend(A, k, axis=1), "x": _zero_extend(x, k)}
    if a_format == "fp8":
        inputs["scale"] = scale
    return evaluate(gemv_expr(A.shape[0], k, plan, a_format), inputs, num)


def gemv_blas(alpha, A: np.ndarray, x: np.ndarray, beta, y: np.ndarray, plan: Plan,
              a_format: str = "f32", scale: np.ndarray = None, num: str = "f32"):
    k = plan.chunk * plan.row_parts
    if A.shape[1] > k:
        raise ValueError(f"rows of {A.shape[1]} exceed W * row_parts = {k}")
    ft = np.float32 if num == "f32" else None
    beta_zero = float(beta) == 0.0
    inputs = {"A": _zero_extend(A, k, axis=1), "x": _zero_extend(x, k),
              "alpha": np.asarray(alpha, ft)}
    if not beta_zero:
        inputs["beta"] = np.asarray(beta, ft)
        inputs["yin"] = y
    if a_format == "fp8":
        inputs["scale"] = scale
    return evaluate(gemv_blas_expr(A.shape[0], k, plan, a_format, beta_zero), inputs, num)
