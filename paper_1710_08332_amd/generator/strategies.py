"""The DPIA expression a strategy descriptor stands for.

``dot_text`` / ``asum_text`` / ``gemv_text`` print, for a ``Strategy`` and a
problem size, the functional expression the library's hand-written kernels
evaluate (the blocked dot product of Sec. 2.1, eq. (2), with the lane order,
combine, vector width and accumulation the descriptor names), so that the
generator can compile a descriptor too.  Sizes must divide exactly: the
generator compiles the expression as written (the kernels' reading of
lengths that the chunk does not divide is extension with zeros).
"""

from __future__ import annotations

PLUS = "(lam (e acc) (+ e acc))"
DOT_STEP = "(lam (z acc) (+ (* (fst z) (snd z)) acc))"
ASUM_STEP = "(lam (e acc) (+ (abs e) acc))"
# Kahan's step with element z = (x, y) and accumulator (s, c):
# yk = x*y - c ; t = s + yk ; new accumulator (t, (t - s) - yk)
KAHAN_STEP = ("(lam (z acc) ((lam (yk) ((lam (t) (pair t (- (- t (fst acc)) yk)))"
              " (+ (fst acc) yk))) (- (* (fst z) (snd z)) (snd acc))))")
# Sum2 (Ogita, Rump, Oishi 2005) with element z = (x, y) and accumulator
# (s, c), value s + c: p = x*y ; t = s + p ; bp = t - s ;
# new accumulator (t, c + ((s - (t - bp)) + (p - bp)))
SUM2_STEP = ("(lam (z acc) ((lam (p) ((lam (t) ((lam (bp) (pair t (+ (snd acc)"
             " (+ (- (fst acc) (- t bp)) (- p bp))))) (- t (fst acc)))) (+ (fst acc) p)))"
             " (* (fst z) (snd z))))")
# Sum2 merge of a later pair r into l: TwoSum of the s parts, error into c:
# s = s_l + s_r ; bp = s - s_l ; new (s, (c_l + c_r) + ((s_l - (s - bp)) + (s_r - bp)))
SUM2_MERGE = ("(lam (r l) ((lam (s) ((lam (bp) (pair s (+ (+ (snd l) (snd r))"
              " (+ (- (fst l) (- s bp)) (- (fst r) bp))))) (- s (fst l))))"
              " (+ (fst l) (fst r))))")
# TwoSum merge of a later pair r into the earlier accumulator l:
# s = s_l + s_r ; bp = s - s_l ; e = (s_l - (s - bp)) + (s_r - bp) ;
# new accumulator (s, (c_l + c_r) - e)
KAHAN_MERGE = ("(lam (r l) ((lam (s) ((lam (bp) (pair s (- (+ (snd l) (snd r))"
               " (+ (- (fst l) (- s bp)) (- (fst r) bp))))) (- s (fst l))))"
               " (+ (fst l) (fst r))))")


def _parts(s):
    C, L = int(s.seq_len), int(s.local_size)
    V = max(1, int(getattr(s, "vec_width", 1) or 1))
    return C, L, V


def _zero(V: int, kahan: bool) -> str:
    if kahan:
        return "(pair 0 0)"
    return "0" if V == 1 else f"(broadcast {V} 0)"


def _rows(ch: str, s) -> str:
    C, L, _ = _parts(s)
    if s.order == 1:                                  # strided: lane l takes l, l+L, ...
        return f"(transpose (split {L} {ch}))"
    return f"(split {C} {ch})"


def _lanes(ch: str, s, step: str, zero: str) -> str:
    return f"(mapLocal (lam (row) (reduceSeq {step} {zero} row)) {_rows(ch, s)})"


def _combine(lanes: str, s, merge: str, zero: str) -> str:
    _, L, _ = _parts(s)
    if s.wg_combine == 1 or L == 1:                   # sequential
        return f"(reduceSeq {merge} {zero} {lanes})"
    level, width = lanes, L
    while width > 2:                                  # pairs in local memory
        level = (f"((toLocal (lam (v) (mapLocal (lam (q) (reduceSeq {merge} {zero} q))"
                 f" (split 2 v)))) {level})")
        width //= 2
    return f"(reduceSeq {merge} {zero} {level})"


def _reduction(s, view: str, n: int, step: str) -> str:
    C, L, V = _parts(s)
    kahan = s.accum != 0                              # a compensated pair
    if n % (C * L * V):
        raise ValueError(f"n = {n} is not a multiple of the chunk {C * L * V}")
    zero = _zero(V, kahan)
    pair_merge = KAHAN_MERGE if s.accum == 1 else SUM2_MERGE
    merge = pair_merge if kahan else PLUS
    if s.wg_combine == 2:                             # uncombined: every lane's value
        chunks = f"(join (mapWorkgroup (lam (ch) {_lanes('ch', s, step, zero)}) (split {C * L} {view})))"
    else:
        body = _combine(_lanes("ch", s, step, zero), s, merge, zero)
        chunks = f"(mapWorkgroup (lam (ch) {body}) (split {C * L} {view}))"
    if V > 1:
        chunks = f"(asScalar {V} {chunks})"
    if not kahan:
        return f"(reduceSeq {PLUS} 0 {chunks})"
    sign = "-" if s.accum == 1 else "+"               # Kahan s - c, Sum2 s + c
    if s.final_f64:
        return (f"(reduceSeq (lam (p acc) (+ ({sign} (f64 (fst p)) (f64 (snd p))) acc)) (f64 0)"
                f" {chunks})")
    return f"((lam (r) ({sign} (fst r) (snd r))) (reduceSeq {pair_merge} (pair 0 0) {chunks}))"


def _vec(name: str, V: int) -> str:
    return name if V == 1 else f"(asVector {V} {name})"


def dot_text(s, n: int) -> str:
    _, _, V = _parts(s)
    step = {1: KAHAN_STEP, 2: SUM2_STEP}.get(int(s.accum), DOT_STEP)
    return _reduction(s, f"(zip {_vec('xs', V)} {_vec('ys', V)})", n, step)


def asum_text(s, n: int) -> str:
    _, _, V = _parts(s)
    if s.accum != 0:
        raise ValueError("asum uses plain accumulation")
    return _reduction(s, _vec("xs", V), n, ASUM_STEP)


def dot_chunks_text(s, n: int) -> str:
    """Only the mapWorkgroup level: the chunk values dpia_chunks writes."""
    full = dot_text(s, n)
    prefix = f"(reduceSeq {PLUS} 0 "
    if s.accum != 0 or not full.startswith(prefix):
        raise ValueError("chunk values are printed for plain accumulation")
    return full[len(prefix):-1]


def gemv_text(s, m: int, k: int, a_format: str = "f32") -> str:
    """y = A x, A m x k row-major: binary32, or bf16 / fp8-e4m3 codes
    decoded exactly in the lane step (the decode fused into the fold, which
    gives the values of decoding first: the map fusion law, Sec. 5.3).  For
    fp8 every row value is multiplied by its ``scale`` afterwards."""
    C, L, V = _parts(s)
    R, parts = int(s.rows_per_wg), int(s.row_parts)
    if V != 1 or s.wg_combine == 2 or s.accum != 0:
        raise ValueError("gemv rows use scalar, combined, plain strategies")
    if m % R or k != C * L * parts:
        raise ValueError("m must be a multiple of R and k = C * L * row_parts")
    if a_format == "f32":
        step = DOT_STEP
    elif a_format in ("bf16", "fp8"):
        step = f"(lam (z acc) (+ (* ({a_format} (fst z)) (snd z)) acc))"
    else:
        raise ValueError(f"unknown matrix format {a_format!r}")

    def chunk(view: str) -> str:
        return _combine(_lanes(view, s, step, "0"), s, PLUS, "0")

    def rowred(row: str) -> str:
        if parts == 1:
            return chunk(f"(zip {row} x)")
        return (f"(reduceSeq {PLUS} 0 (map (lam (h) {chunk('h')})"
                f" (split {C * L} (zip {row} x))))")
    if a_format == "fp8":
        body = f"(map (lam (rw) (* (snd rw) {rowred('(fst rw)')})) rows)"
        src = "(zip A scale)"
    else:
        body = f"(map (lam (row) {rowred('row')}) rows)"
        src = "A"
    return f"(join (mapWorkgroup (lam (rows) {body}) (split {R} {src})))"
