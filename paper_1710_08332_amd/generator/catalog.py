"""Programs compiled ahead of time (by ``build``), for the tests and the
benchmark: each is an expression text, its inputs and its numeric type.
Code objects go to ``paper_1710_08332_amd/generated/``."""

from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, List, Tuple

from .. import CONTIGUOUS, KAHAN, SEQ, STRIDED, SUM2, TREE, Strategy
from . import strategies as P
from .runtime import compile_program

OUT_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "generated")

# the dot expression of Sec. 6.2 as printed there (float4 views; 64
# work-items per work-group folding 2048 vectors each; every work-item's
# vector written out)
SEC62_DOT = ("(asScalar 4 (join (mapWorkgroup (lam (zs1) (mapLocal (lam (zs2) (reduceSeq"
             " (lam (x a) (+ (* (fst x) (snd x)) a)) (broadcast 4 0) zs2)) (split 2048 zs1)))"
             " (split 131072 (zip (asVector 4 xs) (asVector 4 ys))))))")

HEADLINE_DOT = Strategy(seq_len=256, local_size=1024, order=STRIDED, wg_combine=TREE)
HEADLINE_GEMV = Strategy(seq_len=32, local_size=256, order=STRIDED, wg_combine=TREE,
                         rows_per_wg=4)


def _vec_inputs(n: int, et: str = "f32", names=("xs", "ys")) -> Dict:
    return {k: (et, (n,)) for k in names}


def programs() -> List[Tuple[str, str, Dict, str]]:
    """(name, expression text, inputs, num) of every catalogued program."""
    out = []

    def dot(name, s, n, num="f32"):
        out.append((name, P.dot_text(s, n), _vec_inputs(n, num), num))

    dot("dot_strided_tree", Strategy(seq_len=4, local_size=64, order=STRIDED), 4 * 64 * 37)
    dot("dot_contiguous_seq", Strategy(seq_len=16, local_size=32, order=CONTIGUOUS,
                                       wg_combine=SEQ), 16 * 32 * 23)
    dot("dot_kahan_f64", Strategy(seq_len=16, local_size=64, order=STRIDED, accum=KAHAN,
                                  final_f64=1), 16 * 64 * 13)
    dot("dot_sum2", Strategy(seq_len=16, local_size=64, order=STRIDED, accum=SUM2),
        16 * 64 * 13)
    dot("dot_u32", Strategy(seq_len=4, local_size=16, order=CONTIGUOUS), 4 * 16 * 29, "u32")
    dot("dot_v4_strided_tree", Strategy(seq_len=8, local_size=64, order=STRIDED, vec_width=4),
        4 * 8 * 64 * 11)
    dot("dot_headline_2p26", HEADLINE_DOT, 1 << 26)
    # Sec. 6.3 hoisting: every work-group's lane values in global memory
    # (toGlobal inside mapWorkgroup), one copy per work-group, folded in
    # lane order by the work-group; the sequential-combine strategy C=4,
    # L=64, contiguous
    add, mul_add = "(lam (e a) (+ e a))", "(lam (z a) (+ (* (fst z) (snd z)) a))"
    ng = 4 * 64 * 300
    out.append(("dot_global_lanes",
                f"(reduceSeq {add} 0 (mapWorkgroup (lam (ch) (reduceSeq {add} 0 ((toGlobal (lam (c)"
                f" (mapLocal (lam (row) (reduceSeq {mul_add} 0 row)) (split 4 c)))) ch)))"
                f" (split 256 (zip xs ys))))", _vec_inputs(ng), "f32"))
    s = Strategy(seq_len=8, local_size=128, order=STRIDED)
    out.append(("asum_strided_tree", P.asum_text(s, 8 * 128 * 19), _vec_inputs(8 * 128 * 19,
                                                                              names=("xs",)),
                "f32"))
    n62 = 1 << 22
    out.append(("dot_sec62_chunks", SEC62_DOT.replace("131072", str(64 * 2048)),
                _vec_inputs(n62), "f32"))
    g = Strategy(seq_len=16, local_size=64, order=STRIDED, rows_per_wg=2)
    out.append(("gemv_strided_tree", P.gemv_text(g, 96, 1024),
                {"A": ("f32", (96, 1024)), "x": ("f32", (1024,))}, "f32"))
    out.append(("gemv_headline_8192", P.gemv_text(HEADLINE_GEMV, 8192, 8192),
                {"A": ("f32", (8192, 8192)), "x": ("f32", (8192,))}, "f32"))
    out.append(("scal_global", "(mapGlobal (lam (e) (* alpha e)) xs)",
                {"alpha": ("f32", ()), "xs": ("f32", (1 << 20,))}, "f32"))
    # low-precision gemv: small (parity) and 16384 x 16384 (speed), and every
    # storage code through the generated decoders
    lp = Strategy(seq_len=4, local_size=64, order=STRIDED, rows_per_wg=2)
    big = Strategy(seq_len=16, local_size=1024, order=STRIDED, rows_per_wg=2)
    for fmt, et in (("bf16", "u16"), ("fp8", "u8")):
        ins = {"A": (et, (64, 256)), "x": ("f32", (256,))}
        bins = {"A": (et, (16384, 16384)), "x": ("f32", (16384,))}
        if fmt == "fp8":
            ins["scale"] = ("f32", (64,))
            bins["scale"] = ("f32", (16384,))
        out.append((f"gemv_{fmt}_strided_tree", P.gemv_text(lp, 64, 256, fmt), ins, "f32"))
        out.append((f"gemv_{fmt}_16384", P.gemv_text(big, 16384, 16384, fmt), bins, "f32"))
        ncodes = 1 << (16 if fmt == "bf16" else 8)
        out.append((f"decode_{fmt}_all", f"(mapGlobal (lam (c) ({fmt} c)) codes)",
                    {"codes": (et, (ncodes,))}, "f32"))
    return out


def path(name: str) -> str:
    return os.path.join(OUT_DIR, name + ".json")


def build_all(jobs: int = 8) -> List[str]:
    os.makedirs(OUT_DIR, exist_ok=True)
    progs = programs()
    with ThreadPoolExecutor(max_workers=min(jobs, len(progs))) as ex:
        return list(ex.map(lambda p: compile_program(p[1], p[2], os.path.join(OUT_DIR, p[0]),
                                                     num=p[3], name=p[0]), progs))


if __name__ == "__main__":
    for p in build_all():
        print(p)
