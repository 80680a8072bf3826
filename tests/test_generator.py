"""The expression generator on the CPU: nesting rules, and the translated
imperative program (run by tests/gen_interp.py) against the oracle's
evaluation of the same expression text, bit for bit."""

import numpy as np
import pytest

from oracle import eval_numpy
from oracle import strategies as S
from paper_1710_08332_amd.generator import CheckError, check, parse
from paper_1710_08332_amd.generator import translate as T
from tests import gen_interp as GI


def disc(seed, n):
    g = np.random.default_rng(seed)
    h = n // 2
    v = (np.where(g.random(h) < 0.5, -1, 1) * 2.0 ** g.uniform(-20, 20, h)).astype(np.float32)
    w = 2 * g.random(h, dtype=np.float32) - 1
    pad = [np.zeros(n % 2, np.float32)]
    p = g.permutation(n)
    return np.concatenate([v, v] + pad)[p], np.concatenate([w, -w] + pad)[p]


def same(a, b):
    return np.asarray(a).tobytes() == np.asarray(b).tobytes()


DOT_PLANS = [
    S.Plan(seq=4, lanes=8, order="strided", combine="tree"),
    S.Plan(seq=5, lanes=3, combine="seq"),
    S.Plan(seq=3, lanes=16, order="contiguous", combine="tree"),
    S.Plan(seq=3, lanes=4, combine="none", vec=4),
    S.Plan(seq=3, lanes=8, order="strided", combine="tree", vec=2),
    S.Plan(seq=2, lanes=4, order="strided", combine="seq", vec=4),
    S.Plan(seq=6, lanes=1),
    S.Plan(seq=2, lanes=2, accum="kahan", final_f64=True),
    S.Plan(seq=3, lanes=4, order="strided", accum="kahan"),
    S.Plan(seq=4, lanes=8, order="strided", accum="sum2"),
    S.Plan(seq=5, lanes=2, combine="seq", accum="sum2", final_f64=True),
]


@pytest.mark.parametrize("p", DOT_PLANS, ids=str)
def test_generated_dot_and_asum_match_the_oracle(p):
    n = p.chunk * 3
    x, y = disc(7, n)
    prog = T.translate(S.dot_expr(n, p), {"xs": ("f32", (n,)), "ys": ("f32", (n,))})
    got = GI.run(prog, {"xs": x, "ys": y})
    want = S.dot(x, y, p)
    assert same(got["out"][0], want)
    if p.accum == "plain":
        prog = T.translate(S.asum_expr(n, p), {"xs": ("f32", (n,))})
        assert same(GI.run(prog, {"xs": x})["out"][0], S.asum(x, p))
        g = np.random.default_rng(3)
        xi = g.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
        yi = g.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
        prog = T.translate(S.dot_expr(n, p), {"xs": ("u32", (n,)), "ys": ("u32", (n,))}, num="u32")
        assert same(GI.run(prog, {"xs": xi, "ys": yi})["out"][0], S.dot(xi, yi, p, num="u32"))


@pytest.mark.parametrize("p", [S.Plan(seq=4, lanes=8, order="strided", rows=2),
                               S.Plan(seq=3, lanes=4, combine="seq", rows=1, row_parts=2),
                               S.Plan(seq=2, lanes=16, order="contiguous", rows=4)], ids=str)
def test_generated_gemv_matches_the_oracle(p):
    m, k = 4 * p.rows, p.chunk * p.row_parts
    g = np.random.default_rng(11)
    A = g.standard_normal((m, k)).astype(np.float32)
    x = g.standard_normal(k).astype(np.float32)
    prog = T.translate(S.gemv_expr(m, k, p), {"A": ("f32", (m, k)), "x": ("f32", (k,))})
    assert same(GI.run(prog, {"A": A, "x": x})["out"], S.gemv(A, x, p))
    y0 = g.standard_normal(m).astype(np.float32)
    e = S.gemv_blas_expr(m, k, p)
    prog = T.translate(e, {"A": ("f32", (m, k)), "x": ("f32", (k,)), "alpha": ("f32", ()),
                           "beta": ("f32", ()), "yin": ("f32", (m,))})
    got = GI.run(prog, {"A": A, "x": x, "alpha": np.float32(0.5), "beta": np.float32(-2),
                        "yin": y0})["out"]
    assert same(got, S.gemv_blas(0.5, A, x, -2.0, y0, p))


def test_generated_scal_and_paper_listing_forms():
    x = disc(5, 64)[0]
    prog = T.translate("(mapGlobal (lam (e) (* alpha e)) xs)",
                       {"alpha": ("f32", ()), "xs": ("f32", (64,))})
    assert [k.kind for k in prog.kernels] == ["global"]
    assert same(GI.run(prog, {"alpha": np.float32(1.7), "xs": x})["out"], np.float32(1.7) * x)
    # the dot expression of Sec. 6.2 (float4 views, work-items' values written
    # out), smaller: 2 work-groups of 4 work-items folding 3 vectors each
    e = ("(asScalar 4 (join (mapWorkgroup (lam (zs1) (mapLocal (lam (zs2) (reduceSeq"
         " (lam (x a) (+ (* (fst x) (snd x)) a)) (broadcast 4 0) zs2)) (split 3 zs1)))"
         " (split 12 (zip (asVector 4 xs) (asVector 4 ys))))))")
    xs, ys = disc(6, 96)
    prog = T.translate(e, {"xs": ("f32", (96,)), "ys": ("f32", (96,))})
    want = eval_numpy.evaluate(e, {"xs": xs, "ys": ys})
    assert same(GI.run(prog, {"xs": xs, "ys": ys})["out"], want)
    assert same(want, S.dot_chunks(xs, ys, S.Plan(seq=3, lanes=4, combine="none", vec=4)))


@pytest.mark.parametrize("text", [
    "(mapLocal (lam (x) x) xs)",                                            # no work-group
    "(mapWorkgroup (lam (r) (mapLocal (lam (q) (mapLocal (lam (z) z) q)) r)) xs)",
    "(mapWorkgroup (lam (r) (mapWorkgroup (lam (q) q) r)) xs)",
    "(mapGlobal (lam (r) (mapLocal (lam (q) q) r)) xs)",
    "(mapSeq (lam (r) (mapGlobal (lam (q) q) r)) xs)",
    "(reduceSeq (lam (r a) (mapWorkgroup (lam (q) q) r)) 0 xs)",
])
def test_illegal_nestings_are_rejected(text):
    with pytest.raises(CheckError):
        check(parse(text))


def test_legal_nestings_are_accepted():
    # a sequential loop around mapLocal inside a work-group (gemv rows), and
    # sequential maps inside work-items
    for text in ["(mapWorkgroup (lam (rows) (map (lam (r) (mapLocal (lam (q) q) r)) rows)) xs)",
                 "(mapWorkgroup (lam (r) (mapLocal (lam (q) (mapSeq (lam (z) z) q)) r)) xs)",
                 "(mapGlobal (lam (r) (reduceSeq (lam (e a) (+ e a)) 0 r)) xs)"]:
        check(parse(text))


def test_catalogued_programs_match_the_oracle_on_the_cpu():
    # every program the build compiles, at its own sizes (the small ones; the
    # full-size ones share their shapes), run through the imperative form
    from paper_1710_08332_amd.generator import catalog
    g = np.random.default_rng(21)
    for name, text, inputs, num in catalog.programs():
        if max(int(np.prod(s)) for _, s in inputs.values()) > 70000:
            continue
        feed = {}
        for k, (et, shape) in inputs.items():
            if et == "u32":
                feed[k] = g.integers(0, 2 ** 32, shape, dtype=np.uint64).astype(np.uint32)
            elif et == "u16":                        # bf16 codes, no inf / NaN
                c = g.integers(0, 2 ** 16, shape).astype(np.uint16)
                c[(c & 0x7F80) == 0x7F80] = 0x3F80
                feed[k] = c
            elif et == "u8":                         # fp8 codes, no NaN
                c = g.integers(0, 256, shape).astype(np.uint8)
                c[(c & 0x7F) == 0x7F] = 0x38
                feed[k] = c
            else:
                feed[k] = (2 * g.random(shape) - 1).astype(np.float32)
        prog = T.translate(text, inputs, num=num, name=name)
        got = GI.run(prog, feed)["out"]
        want = np.atleast_1d(eval_numpy.evaluate(text, feed, num=num))
        assert same(got[:want.size], want), name


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_generated_low_precision_gemv_matches_the_oracle(fmt):
    from paper_1710_08332_amd import Strategy, STRIDED
    from paper_1710_08332_amd.generator import strategies as P
    s = Strategy(seq_len=4, local_size=16, order=STRIDED, rows_per_wg=2)
    m, k = 6, 64
    g = np.random.default_rng(17)
    x = g.standard_normal(k).astype(np.float32)
    if fmt == "bf16":
        codes = g.integers(0, 2 ** 16, (m, k)).astype(np.uint16)
        inputs = {"A": ("u16", (m, k)), "x": ("f32", (k,))}
        feed, scale = {"A": codes, "x": x}, None
    else:
        codes = g.integers(0, 256, (m, k)).astype(np.uint8)
        scale = g.random(m, dtype=np.float32) + np.float32(0.5)
        inputs = {"A": ("u8", (m, k)), "x": ("f32", (k,)), "scale": ("f32", (m,))}
        feed = {"A": codes, "x": x, "scale": scale}
    text = P.gemv_text(s, m, k, fmt)
    prog = T.translate(text, inputs)
    got = GI.run(prog, feed)["out"]
    want = S.gemv(codes, x, S.Plan(seq=4, lanes=16, order="strided", rows=2), a_format=fmt,
                  scale=scale)
    assert same(got, want) or (np.isnan(got) == np.isnan(want)).all() and \
        same(got[~np.isnan(got)], np.asarray(want)[~np.isnan(want)])


def test_translation_errors():
    from paper_1710_08332_amd.generator.translate import TranslateError
    with pytest.raises(TranslateError):      # arithmetic on storage codes
        T.translate("(map (lam (c) (+ c c)) xs)", {"xs": ("u16", (8,))})
    with pytest.raises(TranslateError):      # zip of different lengths
        T.translate("(zip xs ys)", {"xs": ("f32", (8,)), "ys": ("f32", (4,))})
    with pytest.raises(TranslateError):      # split that does not divide
        T.translate("(split 3 xs)", {"xs": ("f32", (8,))})
    with pytest.raises(TranslateError):      # 32-bit indices only
        T.translate("(mapGlobal (lam (e) (* e e)) xs)", {"xs": ("f32", (1 << 31,))})


from hypothesis import given, settings, strategies as st  # noqa: E402


@settings(max_examples=40, deadline=None)
@given(seq=st.integers(1, 6), lanes_log=st.integers(0, 4), order=st.sampled_from(["contiguous", "strided"]),
       combine=st.sampled_from(["tree", "seq", "none"]), vec=st.sampled_from([1, 2, 4]),
       accum=st.sampled_from(["plain", "kahan", "sum2"]), chunks=st.integers(1, 4),
       seed=st.integers(0, 2 ** 16))
def test_random_strategies_translate_to_the_oracle_value(seq, lanes_log, order, combine, vec,
                                                         accum, chunks, seed):
    # any strategy the oracle accepts: the generator's imperative program gives
    # the oracle's bits
    if accum != "plain" and (vec > 1 or combine == "none"):
        vec, combine = 1, "tree"
    p = S.Plan(seq=seq, lanes=1 << lanes_log, order=order, combine=combine, vec=vec, accum=accum)
    n = p.chunk * chunks
    x, y = disc(seed, n)
    prog = T.translate(S.dot_expr(n, p), {"xs": ("f32", (n,)), "ys": ("f32", (n,))})
    assert same(GI.run(prog, {"xs": x, "ys": y})["out"][0], S.dot(x, y, p))


def _nodes(cmds, acc=None):
    from paper_1710_08332_amd.generator import ir
    acc = acc if acc is not None else set()
    for c in cmds:
        acc.add(type(c).__name__)
        for attr in ("body", "main", "tail"):
            if hasattr(c, attr):
                _nodes(getattr(c, attr), acc)
    return acc


@pytest.mark.parametrize("p,want", [
    (S.Plan(seq=64, lanes=256, order="strided"), {"Lanes", "VLoad", "Blocked"}),
    (S.Plan(seq=32, lanes=256, order="contiguous", combine="seq"), {"Lanes", "Blocked"}),
    (S.Plan(seq=32, lanes=256, order="strided", accum="sum2"), {"Lanes", "VLoad", "Blocked"}),
    (S.Plan(seq=48, lanes=256, order="strided", accum="kahan", final_f64=True),
     {"Lanes", "VLoad", "Blocked"}),
    (S.Plan(seq=4, lanes=64, order="strided"), {"Blocked"}),              # 64 chunks: the fold
    (S.Plan(seq=2, lanes=16, order="strided", vec=4), {"Blocked"}),       # asScalar selectors
], ids=str)
def test_optimisation_passes_keep_the_oracle_value(p, want):
    # sizes that make the passes fire: coarsened lanes with 16-byte loads,
    # blocked folds, the blocked one-work-item fold of many chunk values
    # (whose asScalar reads select components by index)
    chunks = 2 if p.lanes >= 256 else (64 if p.vec == 1 else 16)
    n = p.chunk * chunks
    x, y = disc(90, n)
    prog = T.translate(S.dot_expr(n, p), {"xs": ("f32", (n,)), "ys": ("f32", (n,))})
    assert want <= _nodes([c for k in prog.kernels for c in k.body])
    assert same(GI.run(prog, {"xs": x, "ys": y})["out"][0], S.dot(x, y, p))


def test_optimised_gemv_rows_keep_the_oracle_value():
    p = S.Plan(seq=16, lanes=256, order="strided", rows=2)
    m, k = 4, p.chunk
    g = np.random.default_rng(91)
    A = g.standard_normal((m, k)).astype(np.float32)
    x = g.standard_normal(k).astype(np.float32)
    prog = T.translate(S.gemv_expr(m, k, p), {"A": ("f32", (m, k)), "x": ("f32", (k,))})
    assert {"Lanes", "VLoad", "Blocked"} <= _nodes([c for kk in prog.kernels for c in kk.body])
    assert same(GI.run(prog, {"A": A, "x": x})["out"], S.gemv(A, x, p))
    plain = T.translate(S.gemv_expr(m, k, p), {"A": ("f32", (m, k)), "x": ("f32", (k,))},
                        optimise=False)
    assert "Lanes" not in _nodes([c for kk in plain.kernels for c in kk.body])
    assert same(GI.run(plain, {"A": A, "x": x})["out"], S.gemv(A, x, p))


@pytest.mark.parametrize("fmt,lanes", [("bf16", 512), ("fp8", 1024)])
def test_optimised_low_precision_rows_keep_the_oracle_value(fmt, lanes):
    # 8 bf16 or 16 fp8 lanes per work-item, the codes read 16 bytes at a time
    from paper_1710_08332_amd import STRIDED, Strategy
    from paper_1710_08332_amd.generator import strategies as P
    s = Strategy(seq_len=2, local_size=lanes, order=STRIDED)
    m, k = 3, 2 * lanes
    g = np.random.default_rng(92)
    x = g.standard_normal(k).astype(np.float32)
    if fmt == "bf16":
        codes = g.integers(0, 2 ** 16, (m, k)).astype(np.uint16)
        codes[(codes & 0x7F80) == 0x7F80] = 0x3F80
        inputs = {"A": ("u16", (m, k)), "x": ("f32", (k,))}
        feed, scale = {"A": codes, "x": x}, None
    else:
        codes = g.integers(0, 256, (m, k)).astype(np.uint8)
        codes[(codes & 0x7F) == 0x7F] = 0x38
        scale = g.random(m, dtype=np.float32) + np.float32(0.5)
        inputs = {"A": ("u8", (m, k)), "x": ("f32", (k,)), "scale": ("f32", (m,))}
        feed = {"A": codes, "x": x, "scale": scale}
    prog = T.translate(P.gemv_text(s, m, k, fmt), inputs)
    body = [c for kk in prog.kernels for c in kk.body]
    assert {"Lanes", "VLoad"} <= _nodes(body)
    want = S.gemv(codes, x, S.Plan(seq=2, lanes=lanes, order="strided"), a_format=fmt,
                  scale=scale)
    assert same(GI.run(prog, feed)["out"], want)


@pytest.mark.parametrize("fmt,rows", [("bf16", 2), ("fp8", 4), ("bf16", 6)])
def test_paired_low_precision_rows_share_x_and_keep_the_oracle_value(fmt, rows, monkeypatch):
    # a work-group's rows of bf16 / fp8 codes run two at a time, so each x
    # read serves both: as many x loads per round as one row had, half the
    # rounds, the same bits
    from paper_1710_08332_amd import STRIDED, Strategy
    from paper_1710_08332_amd.generator import passes
    from paper_1710_08332_amd.generator import strategies as P
    lanes = 512
    s = Strategy(seq_len=2, local_size=lanes, order=STRIDED, rows_per_wg=rows)
    m, k = 2 * rows, 2 * lanes
    g = np.random.default_rng(93)
    x = g.standard_normal(k).astype(np.float32)
    if fmt == "bf16":
        codes = g.integers(0, 2 ** 16, (m, k)).astype(np.uint16)
        codes[(codes & 0x7F80) == 0x7F80] = 0x3F80
        inputs = {"A": ("u16", (m, k)), "x": ("f32", (k,))}
        feed, scale = {"A": codes, "x": x}, None
    else:
        codes = g.integers(0, 256, (m, k)).astype(np.uint8)
        codes[(codes & 0x7F) == 0x7F] = 0x38
        scale = g.random(m, dtype=np.float32) + np.float32(0.5)
        inputs = {"A": ("u8", (m, k)), "x": ("f32", (k,)), "scale": ("f32", (m,))}
        feed = {"A": codes, "x": x, "scale": scale}
    text = P.gemv_text(s, m, k, fmt)
    want = S.gemv(codes, x, S.Plan(seq=2, lanes=lanes, order="strided", rows=rows),
                  a_format=fmt, scale=scale)
    paired = T.translate(text, inputs)
    assert same(GI.run(paired, feed)["out"], want)
    monkeypatch.setattr(passes, "pair_rows", lambda cmds, *a, **kw: cmds)
    single = T.translate(text, inputs)
    assert same(GI.run(single, feed)["out"], want)

    def row_loops(prog):
        return [c.n for c in _flat(prog.kernels[0].body) if type(c).__name__ == "For"
                and c.var.startswith("k") and any(type(b).__name__ in ("ParFor", "Lanes")
                                                  for b in c.body)]
    names = {c.name for c in _flat(paired.kernels[0].body) if hasattr(c, "name")}
    assert any(n.endswith("_r1") for n in names)
    assert row_loops(paired) == [rows // 2] and row_loops(single) == [rows]
    # per load of A's codes, half as many loads of x
    def ratio(prog):
        loads = [c for c in _flat(prog.kernels[0].body) if type(c).__name__ in ("Load", "VLoad")]
        return (sum(c.buf == "x" for c in loads) / sum(c.buf == "A" for c in loads))
    assert ratio(paired) * 2 == ratio(single)


def _flat(cmds, acc=None):
    acc = acc if acc is not None else []
    for c in cmds:
        acc.append(c)
        for attr in ("body", "main", "tail"):
            if hasattr(c, attr):
                _flat(getattr(c, attr), acc)
    return acc


def test_binary32_rows_are_not_paired():
    # the hand-written kernels pair rows only for 1- and 2-byte elements
    p = S.Plan(seq=16, lanes=256, order="strided", rows=2)
    m, k = 4, p.chunk
    prog = T.translate(S.gemv_expr(m, k, p), {"A": ("f32", (m, k)), "x": ("f32", (k,))})
    names = {c.name for kk in prog.kernels for c in _flat(kk.body) if hasattr(c, "name")}
    assert not any(n.endswith("_r1") for n in names)


def test_a_reduction_over_rows_is_not_paired():
    # a reduceSeq over a work-group's rows carries its accumulator from row
    # to row: pairing would reorder its updates, so the pass leaves it alone
    import synthetic
    text = ("(mapWorkgroup (lam (rows) (reduceSeq (lam (row acc) (+ (reduceSeq (lam (e a)"
            " (+ e a)) 0 (mapLocal (lam (p) (* (bf16 (fst p)) (snd p))) (zip row x))) acc))"
            " 0 rows)) (split 2 A))")
    inputs = {"A": ("u16", (4, 256)), "x": ("f32", (256,))}
    prog = T.translate(text, inputs)
    names = {c.name for c in _flat(prog.kernels[0].body) if hasattr(c, "name")}
    assert not any(n.endswith("_r1") for n in names)
    g = np.random.default_rng(94)
    A = synthetic.quantise_bf16(g.standard_normal((4, 256)).astype(np.float32))
    x = g.standard_normal(256).astype(np.float32)
    feed = {"A": A, "x": x}
    want = np.atleast_1d(eval_numpy.evaluate(text, feed, num="f32"))
    assert same(GI.run(prog, feed)["out"], want)


# ------------------------------------------------ hoisting out of parallel loops (Sec. 6.3)
MULADD = "(lam (z a) (+ (* (fst z) (snd z)) a))"
ADD = "(lam (e a) (+ e a))"


def _global_lanes_in_groups(C, L, W):
    # every work-group's lane values in global memory (toGlobal inside
    # mapWorkgroup), folded in lane order by the work-group
    return (f"(reduceSeq {ADD} 0 (mapWorkgroup (lam (ch) (reduceSeq {ADD} 0 "
            f"((toGlobal (lam (c) (mapLocal (lam (row) (reduceSeq {MULADD} 0 row)) (split {C} c))))"
            f" ch))) (split {W} (zip xs ys))))")


def _global_lane_values(C, L, W):
    # each lane's value in global memory (toGlobal inside mapLocal inside
    # mapWorkgroup), then the lanes joined
    return (f"(reduceSeq {ADD} 0 (join (mapWorkgroup (lam (ch) (mapLocal (lam (row) "
            f"((toGlobal (lam (r) (reduceSeq {MULADD} 0 r))) row)) (split {C} ch)))"
            f" (split {W} (zip xs ys)))))")


@pytest.mark.parametrize("build", [_global_lanes_in_groups, _global_lane_values])
def test_global_temporaries_in_parallel_loops_are_scaled_by_the_iterations(build):
    C, L, G = 4, 8, 5
    W = C * L
    n = W * G
    text = build(C, L, W)
    x, y = disc(17, n)
    prog = T.translate(text, {"xs": ("f32", (n,)), "ys": ("f32", (n,))})
    ws = [b for b in prog.buffers if b.kind == "ws"]
    # one copy of the temporary per iteration of the enclosing parallel
    # loops: L lane values per work-group times G work-groups, or one value
    # per lane times L lanes times G work-groups (a single shared copy would
    # hold L values, or one)
    assert any(b.elems == G * L for b in ws), [(b.name, b.elems) for b in ws]
    assert same(GI.run(prog, {"xs": x, "ys": y})["out"][0],
                eval_numpy.evaluate(text, {"xs": x, "ys": y}))
    # the annotation changes no value: the same expression without it
    plain = text.replace("(toGlobal ", "(toPrivate ")
    assert same(eval_numpy.evaluate(plain, {"xs": x, "ys": y}),
                eval_numpy.evaluate(text, {"xs": x, "ys": y}))


def test_global_temporary_of_a_work_group_is_read_after_its_lanes_wrote_it():
    # the group-level fold reads the lane values other work-items wrote to
    # the work-group's copy: the oracle's sequential combine of the same lanes
    C, L, G = 3, 16, 7
    W = C * L
    text = _global_lanes_in_groups(C, L, W)
    x, y = disc(23, W * G)
    prog = T.translate(text, {"xs": ("f32", (W * G,)), "ys": ("f32", (W * G,))})
    got = GI.run(prog, {"xs": x, "ys": y})["out"][0]
    assert same(got, S.dot(x, y, S.Plan(seq=C, lanes=L, order="contiguous", combine="seq")))
