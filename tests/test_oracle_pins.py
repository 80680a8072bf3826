"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test pins one part of the oracle to something other than itself:
IEEE-754 closed forms, the index rules of Fig. 7, the equivalences of
Sec. 5.3, exact integer arithmetic, correctly rounded sums, the paper's own
blocked dot product (Sec. 2.2) and library decoders.
"""

import math
import struct
from fractions import Fraction

import numpy as np
import pytest

from oracle import eval_numpy, eval_scalar, exact, formats
from oracle import strategies as S
from oracle.dpia_lang import parse, to_text

EVALS = [eval_numpy.evaluate, eval_scalar.evaluate]


def bits(a):
    a = np.asarray(a)
    if a.dtype == np.float32:
        return a.view(np.uint32)
    if a.dtype == np.float64:
        return a.view(np.uint64)
    return a


def same_bits(a, b):
    return np.array_equal(bits(a), bits(b))


# ----------------------------------------------------------- binary32 rounding

@pytest.mark.parametrize("ev", EVALS)
def test_binary32_addition_closed_forms(ev):
    # 2^24 + 1 is a tie between 2^24 and 2^24 + 2: ties-to-even gives 2^24.
    # 2^24 + 3 is a tie between 2^24 + 2 and 2^24 + 4: even is 2^24 + 4.
    for b, want in [(1.0, 2.0 ** 24), (3.0, 2.0 ** 24 + 4), (2.0, 2.0 ** 24 + 2)]:
        r = ev("(+ a b)", {"a": np.float32(2 ** 24), "b": np.float32(b)})
        assert float(r) == want
    # 1 + 2^-24 rounds back to 1 (tie to even), 1 + 2^-23 is exact.
    r = ev("(+ a b)", {"a": np.float32(1), "b": np.float32(2.0 ** -24)})
    assert float(r) == 1.0
    r = ev("(+ a b)", {"a": np.float32(1), "b": np.float32(2.0 ** -23)})
    assert float(r) == 1.0 + 2.0 ** -23


def test_binary32_operations_agree_between_two_mechanisms():
    # eval_numpy rounds with numpy's binary32 ufuncs, eval_scalar with a
    # binary64 operation followed by one rounding (innocuous double rounding)
    g = np.random.default_rng(7)
    a = (g.standard_normal(2000) * 10.0 ** g.uniform(-40, 38, 2000)).astype(np.float32)
    b = (g.standard_normal(2000) * 10.0 ** g.uniform(-40, 38, 2000)).astype(np.float32)
    a[:50] = np.float32(1e-45) * np.arange(50, dtype=np.float32)   # subnormals
    for op in "+-*/":
        e = f"(map (lam (p) ({op} (fst p) (snd p))) (zip a b))"
        r1 = eval_numpy.evaluate(e, {"a": a, "b": b})
        r2 = eval_scalar.evaluate(e, {"a": a[:300], "b": b[:300]})
        with np.errstate(all="ignore"):
            want = {"+": np.add, "-": np.subtract, "*": np.multiply, "/": np.divide}[op](a, b)
        assert same_bits(r1, want)
        assert same_bits(r2, want[:300])


def test_subnormals_are_not_flushed():
    tiny = np.float32(2.0 ** -149)
    for ev in EVALS:
        assert float(ev("(+ a a)", {"a": tiny})) == 2.0 ** -148
        assert float(ev("(* a b)", {"a": np.float32(2.0 ** -126), "b": np.float32(0.5)})) == 2.0 ** -127


def test_u32_arithmetic_wraps():
    for ev in EVALS:
        r = ev("(* a b)", {"a": np.uint32(0x10000), "b": np.uint32(0x10001)})
        assert int(r) == (0x10000 * 0x10001) % 2 ** 32
        r = ev("(+ a b)", {"a": np.uint32(0xFFFFFFFF), "b": np.uint32(2)})
        assert int(r) == 1


# ----------------------------------------------------------- layout (Fig. 7)

@pytest.mark.parametrize("ev", EVALS)
def test_split_index_rule(ev):
    # element (i, j) of split n e is element i*n + j of e
    v = np.arange(48, dtype=np.uint32)
    for n in (1, 2, 3, 4, 6, 8, 12, 16, 24, 48):
        r = ev(f"(split {n} v)", {"v": v})
        assert r.shape == (48 // n, n)
        for i in range(48 // n):
            for j in range(n):
                assert r[i, j] == i * n + j


@pytest.mark.parametrize("ev", EVALS)
def test_join_index_rule(ev):
    # element i of join e is element (i div n, i mod n), n the inner length
    w = np.arange(35, dtype=np.uint32).reshape(5, 7) * np.uint32(3)
    r = ev("(join w)", {"w": w})
    for i in range(35):
        assert r[i] == w[i // 7, i % 7]


@pytest.mark.parametrize("ev", EVALS)
def test_split_join_laws(ev):
    g = np.random.default_rng(3)
    v = g.standard_normal(96).astype(np.float32)
    for n in (1, 2, 3, 4, 8, 12, 32, 96):
        assert same_bits(ev(f"(join (split {n} v))", {"v": v}), v)
    w = g.standard_normal((6, 16)).astype(np.float32)
    assert same_bits(ev("(split 16 (join w))", {"w": w}), w)


@pytest.mark.parametrize("ev", EVALS)
def test_zip_pair_projection_laws(ev):
    a = np.arange(10, dtype=np.uint32)
    b = np.arange(10, dtype=np.uint32) * np.uint32(7)
    assert np.array_equal(ev("(map (lam (p) (fst p)) (zip a b))", {"a": a, "b": b}), a)
    assert np.array_equal(ev("(map (lam (p) (snd p)) (zip a b))", {"a": a, "b": b}), b)
    r = ev("(pair a b)", {"a": a, "b": b})
    assert np.array_equal(r[0], a) and np.array_equal(r[1], b)


@pytest.mark.parametrize("ev", EVALS)
def test_transpose_index_rule(ev):
    w = np.arange(12, dtype=np.uint32).reshape(3, 4)
    r = ev("(transpose w)", {"w": w})
    assert r.shape == (4, 3)
    for i in range(4):
        for j in range(3):
            assert r[i, j] == w[j, i]
    assert np.array_equal(ev("(transpose (transpose w))", {"w": w}), w)


@pytest.mark.parametrize("ev", EVALS)
def test_codegen_worked_example(ev):
    # Sec. 4.3 derives, for the parallel map of the dot product,
    # out[i] = xs[i] * ys[i]
    g = np.random.default_rng(11)
    xs = g.standard_normal(33).astype(np.float32)
    ys = g.standard_normal(33).astype(np.float32)
    r = ev("(map (lam (x) (* (fst x) (snd x))) (zip xs ys))", {"xs": xs, "ys": ys})
    assert same_bits(r, xs * ys)


def test_blocked_dot_index_map():
    # The blocked strategy of eq. (2) gives work-item (i, j) the elements
    # 2048*128*i + 2048*j + k, k < 2048 (the reading of the listing in
    # Sec. 2.2 whose printed 128*j term contradicts "each processing 2048
    # elements"), at full paper sizes with two work-groups.
    n = 2 * 128 * 2048
    v = np.arange(n, dtype=np.uint32)
    r = eval_numpy.evaluate(
        "(mapWorkgroup (lam (zs1) (mapLocal (lam (zs2) zs2) (split 2048 zs1)))"
        " (split 262144 v))", {"v": v})
    assert r.shape == (2, 128, 2048)
    i, j, k = np.meshgrid(np.arange(2), np.arange(128), np.arange(2048), indexing="ij")
    assert np.array_equal(r, (2048 * 128 * i + 2048 * j + k).astype(np.uint32))


# ----------------------------------------------------------- Sec. 5.3 laws

def test_map_fusion_law():
    g = np.random.default_rng(5)
    v = g.standard_normal(64).astype(np.float32)
    for ev in EVALS:
        a = ev("(map (lam (x) (* x x)) (map (lam (y) (+ y y)) v))", {"v": v})
        b = ev("(map (lam (y) ((lam (x) (* x x)) (+ y y))) v)", {"v": v})
        assert same_bits(a, b)


def _rewrite(e, f):
    """Apply ``f`` bottom-up to every node of an expression."""
    from oracle.dpia_lang import App, Lam, Prim
    if isinstance(e, Lam):
        e = Lam(e.params, _rewrite(e.body, f))
    elif isinstance(e, Prim):
        e = Prim(e.name, tuple(_rewrite(a, f) for a in e.args))
    elif isinstance(e, App):
        e = App(_rewrite(e.fn, f), tuple(_rewrite(a, f) for a in e.args))
    return f(e)


def test_hierarchy_and_address_space_relabelling_changes_no_bits():
    # mapGlobal / mapWorkgroup / mapLocal / mapSeq all denote map, and
    # toGlobal / toLocal / toPrivate are the identity (Sec. 6.1)
    from oracle.dpia_lang import Prim
    g = np.random.default_rng(6)
    xs, ys = S_inputs(g, 1024)
    base = parse(S.dot_expr(1024, S.Plan(seq=8, lanes=16, combine="tree")))
    want = eval_numpy.evaluate(base, {"xs": xs, "ys": ys})

    def relabel(to):
        return lambda e: (Prim(to, e.args) if isinstance(e, Prim) and e.name.startswith("map")
                          else e)

    def strip_address_spaces(e):
        if isinstance(e, Prim) and e.name in ("toGlobal", "toLocal", "toPrivate"):
            return e.args[0]
        return e

    def swap_address_spaces(e):
        if isinstance(e, Prim) and e.name in ("toLocal", "toPrivate"):
            return Prim("toGlobal", e.args)
        return e

    variants = [_rewrite(base, relabel(m)) for m in ("map", "mapSeq", "mapGlobal", "mapLocal")]
    variants += [_rewrite(base, strip_address_spaces), _rewrite(base, swap_address_spaces)]
    assert all(to_text(v) != to_text(base) for v in variants)
    for t in variants:
        assert same_bits(eval_numpy.evaluate(t, {"xs": xs, "ys": ys}), want)


def test_temporary_storage_is_unobservable():
    # eq. (5): computing E into a temporary, then reading it, equals using E.
    # Here: reducing an array produced by map equals reducing with the map
    # fused into the operator (both visit the same values in the same order).
    g = np.random.default_rng(8)
    xs, ys = S_inputs(g, 300)
    a = eval_numpy.evaluate("(reduceSeq (lam (e a) (+ e a)) 0 (map (lam (z) (* (fst z) (snd z)))"
                            " (zip xs ys)))", {"xs": xs, "ys": ys})
    b = eval_numpy.evaluate("(reduceSeq (lam (z a) (+ (* (fst z) (snd z)) a)) 0 (zip xs ys))",
                            {"xs": xs, "ys": ys})
    assert same_bits(a, b)


def S_inputs(g, n):
    return (2 * g.random(n, dtype=np.float32) - 1), (2 * g.random(n, dtype=np.float32) - 1)


# ----------------------------------------------------------- reduce order

@pytest.mark.parametrize("ev", EVALS)
def test_reduce_is_a_left_fold_closed_form(ev):
    # A sequential fold of ones from 2^24 - 3 in binary32 counts up to 2^24
    # and then sticks: 2^24 + 1 rounds (tie to even) back to 2^24.
    ones = np.ones(9, dtype=np.float32)
    r = ev("(reduceSeq (lam (e a) (+ e a)) 16777213 v)", {"v": ones})
    assert float(r) == 2.0 ** 24
    # the fold visits index 0 first: with a huge element first, later small
    # ones are absorbed; with it last they are not
    v = np.array([2.0 ** 24, 1, 1, 1, 1], dtype=np.float32)
    assert float(ev("(reduceSeq (lam (e a) (+ e a)) 0 v)", {"v": v})) == 2.0 ** 24
    assert float(ev("(reduceSeq (lam (e a) (+ e a)) 0 v)", {"v": v[::-1].copy()})) == 2.0 ** 24 + 4
    # element first, accumulator second: (lam (e a) (- e a)) over [1, 2]
    # gives 2 - (1 - 0) = 1; the other argument order would give -3
    r = ev("(reduceSeq (lam (e a) (- e a)) 0 v)", {"v": np.array([1, 2], dtype=np.float32)})
    assert float(r) == 1.0


PLANS = [
    S.Plan(seq=s, lanes=l, order=o, combine=c)
    for s in (1, 4, 16, 64)
    for l in (1, 2, 16, 64)
    for o in ("contiguous", "strided")
    for c in ("tree", "seq")
]


def test_all_ones_sum_is_exact_for_every_strategy():
    # every partial sum is an integer below 2^24, so each strategy returns n
    n = 1 << 16
    ones = np.ones(n, dtype=np.float32)
    for p in PLANS:
        if n % p.chunk:
            continue
        assert float(S.dot(ones, ones, p)) == n
        assert float(S.asum(-ones, p)) == n


def test_purely_sequential_strategy_saturates_at_two_to_the_24():
    # one lane, one chunk, n elements: the fold of ones gets stuck at 2^24
    n = (1 << 24) + 4096
    ones = np.ones(n, dtype=np.float32)
    blocked = S.Plan(seq=4096, lanes=1)
    # blocked strategy: 4100 chunks of exactly 4096, final fold is exact too
    assert float(S.dot(ones, ones, blocked)) == n
    # the pure left fold, written directly
    v = np.ones(4096 + 8, dtype=np.float32)
    r = eval_numpy.evaluate("(reduceSeq (lam (e a) (+ e a)) 16773120 v)", {"v": v})
    assert float(r) == 2.0 ** 24


def test_integer_strategies_equal_the_brute_force_sum():
    # in the ring of integers modulo 2^32 every association gives the same
    # value, so each strategy must equal the exact sum of products mod 2^32
    g = np.random.default_rng(21)
    n = 4096
    x = g.integers(-2 ** 31, 2 ** 31, n, dtype=np.int64).astype(np.int32).view(np.uint32)
    y = g.integers(-2 ** 31, 2 ** 31, n, dtype=np.int64).astype(np.int32).view(np.uint32)
    want = sum(int(a) * int(b) for a, b in zip(x.tolist(), y.tolist())) % 2 ** 32
    for p in PLANS:
        if n % p.chunk:
            continue
        assert int(S.dot(x, y, p, num="u32")) == want


def test_exactly_representable_float_sums_are_exact_for_every_strategy():
    g = np.random.default_rng(22)
    n = 1 << 14
    x = g.integers(-8, 9, n).astype(np.float32)
    y = g.integers(-8, 9, n).astype(np.float32)
    want = int(np.dot(x.astype(np.int64), y.astype(np.int64)))
    for p in PLANS:
        if n % p.chunk:
            continue
        assert float(S.dot(x, y, p)) == want


def test_dot_error_within_fixed_order_bound():
    g = np.random.default_rng(23)
    n = 1 << 14
    x, y = S_inputs(g, n)
    s = exact.dot_exact(x, y)
    t = exact.dot_abs_terms(x, y)
    for p in PLANS:
        if n % p.chunk:
            continue
        h = exact.strategy_depth(n, p.seq, p.lanes, p.combine)
        err = abs(float(S.dot(x, y, p)) - s)
        assert err <= exact.gamma(h + 1) * t, (p, err)


def discriminating_dot_inputs(seed: int, n: int):
    """Products of magnitude up to 2^20 that cancel in pairs (exact dot = 0),
    shuffled: the computed value is nothing but accumulated rounding error,
    which depends on the association."""
    g = np.random.default_rng(seed)
    v = (np.where(g.random(n // 2) < 0.5, -1, 1) * 2.0 ** g.uniform(-20, 20, n // 2)).astype(np.float32)
    w = 2 * g.random(n // 2, dtype=np.float32) - 1
    perm = g.permutation(n)
    return np.concatenate([v, v])[perm], np.concatenate([w, -w])[perm]


def test_strategies_are_distinguishable():
    # Every pair of different strategies gives different bits on at least one
    # of four cancelling inputs.  This is what makes a bit-exact parity test
    # able to fail when a kernel runs another association than the one asked.
    plans = [S.Plan(seq=s, lanes=l, order=o, combine=c)
             for s, l in [(64, 16), (16, 64), (256, 16), (32, 32)]
             for o in ("contiguous", "strided") for c in ("tree", "seq")]
    n = 4096
    vals = []
    for seed in range(4):
        x, y = discriminating_dot_inputs(100 + seed, n)
        vals.append([float(S.dot(x, y, p)) for p in plans])
    for i in range(len(plans)):
        for j in range(i + 1, len(plans)):
            assert any(v[i] != v[j] for v in vals), (plans[i], plans[j])


# ----------------------------------------------------------- the paper's listing

def test_blocked_dot_matches_a_loop_nest_of_the_two_level_strategy():
    # Sec. 2.2 lowers eq. (2) to: per work-group i and work-item j a private
    # accumulator folds its block of elements, each result goes to
    # tmp[groups-of-j], and one sequential loop folds tmp.  Written here as
    # plain loops over binary32 numpy scalars (no layout primitives), with the
    # corrected block index i*L*C + j*C + k.
    g = np.random.default_rng(25)
    C, L, G = 32, 8, 6
    xs, ys = S_inputs(g, C * L * G)
    tmp = []
    for i in range(G):
        for j in range(L):
            acc = np.float32(0)
            for k in range(C):
                e = i * L * C + j * C + k
                acc = xs[e] * ys[e] + acc
            tmp.append(acc)
    out = np.float32(0)
    for t in tmp:
        out = out + t
    # The same strategy as a DPIA expression: eq. (2) with the outer reduce
    # folding all L*G work-item results in order.
    e = ("(reduceSeq (lam (e a) (+ e a)) 0 (join (mapWorkgroup (lam (zs1) (mapLocal"
         " (lam (zs2) (reduceSeq (lam (x a) (+ (* (fst x) (snd x)) a)) 0 zs2))"
         f" (split {C} zs1))) (split {C * L} (zip xs ys)))))")
    for ev in EVALS:
        assert same_bits(ev(e, {"xs": xs, "ys": ys}), out)


def test_strided_order_equals_vector_accumulator_form():
    # transpose (split L ch) row l = ch[l], ch[l+L], ...  The same per-lane
    # order with Fig. 5a primitives only: a reduce over the rows of
    # split L ch whose accumulator is the array of L lane sums, each step
    # updating every lane with its own element (like the float4 accumulators
    # of Sec. 6.2, here L wide).
    g = np.random.default_rng(26)
    C, L = 16, 8
    xs, ys = S_inputs(g, C * L)
    zeros = np.zeros(L, dtype=np.float32)
    via_transpose = ("(mapLocal (lam (s) (reduceSeq (lam (z a) (+ (* (fst z) (snd z)) a)) 0 s))"
                     f" (transpose (split {L} (zip xs ys))))")
    via_vector = (f"(reduceSeq (lam (row acc) (map (lam (q) (+ (* (fst (fst q)) (snd (fst q)))"
                  f" (snd q))) (zip row acc))) zeros (split {L} (zip xs ys)))")
    for ev in EVALS:
        a = ev(via_transpose, {"xs": xs, "ys": ys})
        b = ev(via_vector, {"xs": xs, "ys": ys, "zeros": zeros})
        assert same_bits(a, b)


# ----------------------------------------------------------- asum and gemv

def test_asum_equals_dot_of_magnitudes_with_ones():
    # |x| * 1 is exact, so abs x + a and (|x| * 1) + a round identically
    g = np.random.default_rng(27)
    n = 4096
    x = g.standard_normal(n).astype(np.float32)
    ones = np.ones(n, dtype=np.float32)
    for p in PLANS:
        if n % p.chunk:
            continue
        assert same_bits(S.asum(x, p), S.dot(np.abs(x), ones, p))
        assert same_bits(S.asum(x, p), S.asum(-x, p))


def test_gemv_identity_and_integer_rows():
    g = np.random.default_rng(28)
    m = k = 64
    A = np.eye(m, k, dtype=np.float32)
    x = g.standard_normal(k).astype(np.float32)
    for p in (S.Plan(seq=4, lanes=16, rows=2), S.Plan(seq=16, lanes=4, order="strided", combine="seq"),
              S.Plan(seq=2, lanes=16, rows=4, row_parts=2)):
        assert same_bits(S.gemv(A, x, p), x)
    Ai = g.integers(-2 ** 31, 2 ** 31, (8, 32), dtype=np.int64).astype(np.int32).view(np.uint32)
    xi = g.integers(-2 ** 31, 2 ** 31, 32, dtype=np.int64).astype(np.int32).view(np.uint32)
    want = [sum(int(a) * int(b) for a, b in zip(Ai[r].tolist(), xi.tolist())) % 2 ** 32 for r in range(8)]
    for p in (S.Plan(seq=4, lanes=8, rows=2), S.Plan(seq=8, lanes=2, order="strided", rows=4, row_parts=2)):
        assert [int(v) for v in S.gemv(Ai, xi, p, num="u32")] == want


def test_gemv_rows_are_dot_products_of_the_same_strategy():
    g = np.random.default_rng(29)
    m, k = 8, 256
    A = g.standard_normal((m, k)).astype(np.float32)
    x = (2 * g.random(k, dtype=np.float32) - 1)
    p = S.Plan(seq=16, lanes=16, order="strided", combine="tree", rows=4)
    y = S.gemv(A, x, p)
    for r in range(m):
        assert same_bits(y[r], S.dot(A[r], x, S.Plan(seq=16, lanes=16, order="strided")))
    want = exact.gemv_exact(A, x)
    bound = [exact.gamma(16 + 8 + 2) * exact.dot_abs_terms(A[r], x) for r in range(m)]
    assert np.all(np.abs(y - want) <= bound)


def test_gemv_two_row_parts_fold_halves_in_order():
    g = np.random.default_rng(30)
    m, k = 4, 128
    A = g.standard_normal((m, k)).astype(np.float32)
    x = g.standard_normal(k).astype(np.float32)
    half = S.Plan(seq=8, lanes=8)
    y = S.gemv(A, x, S.Plan(seq=8, lanes=8, row_parts=2, rows=2))
    for r in range(m):
        h0 = S.dot(A[r, :64], x[:64], half)
        h1 = S.dot(A[r, 64:], x[64:], half)
        assert same_bits(y[r], (np.float32(0) + h0) + h1)


def test_low_precision_gemv_decodes_then_accumulates_in_binary32():
    g = np.random.default_rng(31)
    m, k = 4, 64
    codes16 = g.integers(0, 2 ** 16, (m, k)).astype(np.uint16)
    codes16[(codes16 & 0x7F80) == 0x7F80] = 0x3F80   # no inf/nan
    x = g.standard_normal(k).astype(np.float32)
    p = S.Plan(seq=4, lanes=16)
    y = S.gemv(codes16, x, p, a_format="bf16")
    Af = formats.bf16_decode(codes16)
    assert same_bits(y, S.gemv(Af, x, p))
    codes8 = g.integers(0, 256, (m, k)).astype(np.uint8)
    codes8[(codes8 & 0x7F) == 0x7F] = 0x38           # no NaN
    scale = g.random(m, dtype=np.float32) + np.float32(0.5)
    y8 = S.gemv(codes8, x, p, a_format="fp8", scale=scale)
    rows = S.gemv(formats.fp8_decode(codes8), x, p)
    assert same_bits(y8, scale * rows)
    for ev in EVALS[1:]:
        e = S.gemv_expr(m, k, p, "fp8")
        assert same_bits(ev(e, {"A": codes8, "x": x, "scale": scale}), y8)


# ----------------------------------------------------------- decoders

def test_bf16_decoder_exhaustive_against_torch():
    import torch
    codes = np.arange(2 ** 16, dtype=np.uint32).astype(np.uint16)
    ours = formats.bf16_decode(codes)
    theirs = torch.from_numpy(codes.view(np.int16)).view(torch.bfloat16).float().numpy()
    nan = np.isnan(theirs)
    assert np.array_equal(np.isnan(ours), nan)
    assert same_bits(ours[~nan], theirs[~nan])


def test_fp8_decoder_exhaustive_against_torch():
    import torch
    codes = np.arange(256, dtype=np.uint8)
    ours = formats.fp8_decode(codes)
    theirs = torch.from_numpy(codes).view(torch.float8_e4m3fn).float().numpy()
    nan = np.isnan(theirs)
    assert np.array_equal(np.isnan(ours), nan)
    assert nan.sum() == 2                         # S.1111.111 only
    assert same_bits(ours[~nan], theirs[~nan])
    assert ours[0x7E] == 448.0 and ours[0x01] == 2.0 ** -9


# ----------------------------------------------------------- Kahan variant

def _kahan_reference(x, y, C, L):
    """Kahan / TwoSum on Fractions of the binary32 values, with each binary32
    rounding applied explicitly: an exact-arithmetic restatement used to
    confirm the expression's operation order (one lane block, tree combine)."""
    def r32(q):
        return Fraction(struct.unpack("<f", struct.pack("<f", float(q)))[0])
    lanes = []
    for lane in range(L):
        s, c = Fraction(0), Fraction(0)
        for k in range(C):
            e = lane * C + k
            p = r32(Fraction(float(x[e])) * Fraction(float(y[e])))
            yk = r32(p - c)
            t = r32(s + yk)
            c = r32(r32(t - s) - yk)
            s = t
        lanes.append((s, c))

    def merge(left, right):
        s1, c1 = left
        s2, c2 = right
        s = r32(s1 + s2)
        bp = r32(s - s1)
        e = r32(r32(s1 - r32(s - bp)) + r32(s2 - bp))
        return s, r32(r32(c1 + c2) - e)

    zero = (Fraction(0), Fraction(0))
    while len(lanes) > 1:
        lanes = [merge(merge(zero, lanes[2 * i]), lanes[2 * i + 1]) for i in range(len(lanes) // 2)]
    return lanes[0]


def test_kahan_expression_follows_the_stated_steps():
    g = np.random.default_rng(32)
    C, L = 16, 4
    x = (g.standard_normal(C * L) * 10.0 ** g.uniform(-3, 3, C * L)).astype(np.float32)
    y = (g.standard_normal(C * L)).astype(np.float32)
    p = S.Plan(seq=C, lanes=L, accum="kahan", combine="tree")
    r = S.dot(x, y, p)
    # one chunk: the chunk pair is merged into (0, 0) by the final fold, and
    # the result is s - c, all in binary32
    s, c = _kahan_reference(x, y, C, L)
    zero_merge = _kahan_reference_merge((Fraction(0), Fraction(0)), (s, c))
    want = np.float32(float(zero_merge[0])) - np.float32(float(zero_merge[1]))
    assert same_bits(r, want)
    e = S.dot_expr(C * L, p)
    assert same_bits(eval_scalar.evaluate(e, {"xs": x, "ys": y}), r)


def _r64(q):
    # Fraction -> nearest binary64 (CPython divides the integers correctly rounded)
    return Fraction(float(q))


@pytest.mark.parametrize("ev", EVALS)
def test_kahan_binary64_final_fold_closed_forms(ev):
    # The binary64 fold of the chunk values: acc = (f64 s - f64 c) + acc, from
    # +0, in chunk order (a Kahan pair's value is s - c).
    # (a) one lane folding 1 then 2^-30: the sum 1 + 2^-30 rounds to 1 in
    #     binary32 and Kahan keeps the lost part as c = -2^-30, so the pair is
    #     (1, -2^-30) and the binary64 value is exactly 1 + 2^-30.  A sign
    #     flip (s + c) gives 1 - 2^-30; dropping c, or subtracting in binary32
    #     before widening, gives 1.
    p = S.Plan(seq=2, lanes=1, accum="kahan", final_f64=True)
    xs = np.array([1.0, 2.0 ** -30], np.float32)
    ys = np.ones(2, np.float32)
    r = ev(S.dot_expr(2, p), {"xs": xs, "ys": ys})
    assert np.asarray(r).dtype == np.float64
    assert float(r) == 1.0 + 2.0 ** -30
    # two such chunks: 2 + 2^-29, exact in binary64
    r2 = ev(S.dot_expr(4, p), {"xs": np.tile(xs, 2), "ys": np.ones(4, np.float32)})
    assert float(r2) == 2.0 + 2.0 ** -29
    # (b) the fold runs in chunk order: chunk values 1, 2^53, -2^53.  In order,
    #     2^53 + 1 is a tie that rounds to 2^53 (even), so the result is +0.
    #     Folded from the last chunk (or as 1 + (2^53 - 2^53)) it would be 1.
    q = S.Plan(seq=1, lanes=1, accum="kahan", final_f64=True)
    xs = np.array([1.0, 2.0 ** 53, -2.0 ** 53], np.float32)
    r3 = ev(S.dot_expr(3, q), {"xs": xs, "ys": np.ones(3, np.float32)})
    assert np.asarray(r3).view(np.uint64) == 0
    r4 = ev(S.dot_expr(3, q), {"xs": xs[::-1].copy(), "ys": np.ones(3, np.float32)})
    assert float(r4) == 1.0
    # (c) a chunk's c meets the next chunk in binary64: (1, -2^-30) then a
    #     chunk (-1, 0) gives exactly 2^-30 (dropping c would give 0)
    xs = np.array([1.0, 2.0 ** -30, -1.0, 0.0], np.float32)
    r5 = ev(S.dot_expr(4, p), {"xs": xs, "ys": np.ones(4, np.float32)})
    assert float(r5) == 2.0 ** -30


def _kahan_chunk_pairs(x, y, C, L):
    """Each chunk's merged Kahan pair (lane folds, tree combine, then merged
    into the zero pair as the first step of the outer fold), in Fractions."""
    W = C * L
    zero = (Fraction(0), Fraction(0))
    return [_kahan_reference_merge(zero, _kahan_reference(x[g * W:(g + 1) * W],
                                                          y[g * W:(g + 1) * W], C, L))
            for g in range(len(x) // W)]


def test_kahan_final_folds_over_many_chunks_follow_the_stated_steps():
    # Random chunk pairs with nonzero c: the binary32 TwoSum fold then s - c,
    # and the binary64 fold of s - c, restated over Fractions with each
    # rounding explicit, agree bit for bit with the oracle.
    g = np.random.default_rng(35)
    C, L, G = 8, 4, 9
    n = C * L * G
    x = (np.where(g.random(n) < 0.5, -1, 1) * 10.0 ** g.uniform(-4, 4, n)).astype(np.float32)
    y = (np.where(g.random(n) < 0.5, -1, 1) * 10.0 ** g.uniform(-4, 4, n)).astype(np.float32)
    pairs = _kahan_chunk_pairs(x, y, C, L)
    assert sum(c != 0 for _, c in pairs) >= G // 2          # the c parts matter here
    # binary32: TwoSum-merge the chunk pairs in order from the zero pair
    # (the first merge into the zero pair is the identity on these pairs)
    acc = pairs[0]
    for pr in pairs[1:]:
        acc = _kahan_reference_merge(acc, pr)
    want32 = np.float32(float(acc[0])) - np.float32(float(acc[1]))
    got32 = S.dot(x, y, S.Plan(seq=C, lanes=L, accum="kahan"))
    assert same_bits(got32, want32)
    # binary64: acc = (s - c) + acc, each operation rounded to binary64
    a64 = Fraction(0)
    for s, c in pairs:
        a64 = _r64(_r64(s - c) + a64)
    got64 = S.dot(x, y, S.Plan(seq=C, lanes=L, accum="kahan", final_f64=True))
    assert np.asarray(got64).dtype == np.float64
    assert float(got64) == float(a64)
    # and the order matters on these data: folding from the last chunk differs
    b64 = Fraction(0)
    for s, c in reversed(pairs):
        b64 = _r64(_r64(s - c) + b64)
    c64 = Fraction(0)
    for s, c in pairs:
        c64 = _r64(_r64(s + c) + c64)
    assert float(b64) != float(a64) or float(c64) != float(a64)
    assert float(c64) != float(a64)


def _kahan_reference_merge(left, right):
    def r32(q):
        return Fraction(struct.unpack("<f", struct.pack("<f", float(q)))[0])
    s1, c1 = left
    s2, c2 = right
    s = r32(s1 + s2)
    bp = r32(s - s1)
    e = r32(r32(s1 - r32(s - bp)) + r32(s2 - bp))
    return s, r32(r32(c1 + c2) - e)


def test_twosum_merge_is_error_free():
    # TwoSum: s + e equals s1 + s2 exactly, so the merged pair keeps the
    # exact value (s1 - c1) + (s2 - c2) up to the rounding of c1 + c2 - e
    g = np.random.default_rng(34)
    for _ in range(200):
        s1, s2 = (np.float32(v) for v in g.standard_normal(2) * 10.0 ** g.uniform(-8, 8, 2))
        s = s1 + s2
        bp = s - s1
        e = (s1 - (s - bp)) + (s2 - bp)
        assert Fraction(float(s)) + Fraction(float(e)) == Fraction(float(s1)) + Fraction(float(s2))
    # the oracle's merge on pairs (s2, 0) after (s1, 0) yields (s, -e)
    for _ in range(50):
        s1, s2 = (np.float32(v) for v in g.standard_normal(2) * 10.0 ** g.uniform(-8, 8, 2))
        e_text = f"(reduceSeq {S.KAHAN_MERGE} (pair 0 0) (zip v w))"
        v = np.array([s1, s2], np.float32)
        w = np.zeros(2, np.float32)
        rs, rc = eval_numpy.evaluate(e_text, {"v": v, "w": w})
        assert Fraction(float(rs)) - Fraction(float(rc)) == Fraction(float(s1)) + Fraction(float(s2))


def test_kahan_is_far_more_accurate_than_plain_on_cancelling_data():
    g = np.random.default_rng(33)
    n = 1 << 14
    mag = 10.0 ** g.uniform(-4, 4, n)
    x = (np.where(g.random(n) < 0.5, -1, 1) * mag).astype(np.float32)
    y = (np.where(g.random(n) < 0.5, -1, 1) * 10.0 ** g.uniform(-4, 4, n)).astype(np.float32)
    s = exact.dot_exact(x, y)
    t = exact.dot_abs_terms(x, y)
    plain = S.Plan(seq=256, lanes=16)
    kahan = S.Plan(seq=256, lanes=16, accum="kahan")
    kahan64 = S.Plan(seq=256, lanes=16, accum="kahan", final_f64=True)
    e_plain = abs(float(S.dot(x, y, plain)) - s) / t
    e_k = abs(float(S.dot(x, y, kahan)) - s) / t
    r64 = S.dot(x, y, kahan64)
    assert r64.dtype == np.float64
    e_k64 = abs(float(r64) - s) / t
    # compensated summation: error about 2u + O(n u^2) of sum |t| plus one
    # rounding of each product (u sum |t|): a normwise bound of 4u here
    assert e_k <= 4 * 2.0 ** -24
    assert e_k64 <= 4 * 2.0 ** -24
    assert e_k <= e_plain


# ----------------------------------------------------------- printer / parser

def test_printer_round_trips():
    for p in PLANS[:12]:
        e = S.dot_expr(p.chunk * 2, p)
        assert to_text(parse(e)) == e


# ----------------------------------------------------------- golden fixtures

def _golden_index_maps():
    path = __file__.replace("test_oracle_pins.py", "golden/paper_index_examples.txt")
    out = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, _cite, formula = (p.strip() for p in line.split("|"))
        out[name] = formula
    return out


def test_golden_paper_index_maps():
    maps = _golden_index_maps()
    # codegen_map_dot: element i of the zipped, mapped array uses index i
    xs = np.arange(16, dtype=np.uint32)
    r = eval_numpy.evaluate("(map (lam (x) (fst x)) (zip xs ys))", {"xs": xs, "ys": xs})
    for i in range(16):
        assert r[i] == xs[eval(maps["codegen_map_dot"], {"i": i})]
    # blocked dot, at the paper's sizes (2 groups)
    n = 2 * 128 * 2048
    v = np.arange(n, dtype=np.uint32)
    lanes = eval_numpy.evaluate("(mapWorkgroup (lam (zs1) (mapLocal (lam (zs2) zs2)"
                                " (split 2048 zs1))) (split 262144 v))", {"v": v})
    flat_tmp = eval_numpy.evaluate("(join (mapWorkgroup (lam (zs1) (mapLocal (lam (zs2) zs2)"
                                   " (split 2048 zs1))) (split 262144 v)))", {"v": v})
    g = np.random.default_rng(0)
    for _ in range(200):
        i, j, k = int(g.integers(2)), int(g.integers(128)), int(g.integers(2048))
        assert lanes[i, j, k] == eval(maps["blocked_dot_element"], {"i": i, "j": j, "k": k})
        assert np.array_equal(flat_tmp[eval(maps["blocked_dot_tmp"], {"i": i, "j": j})], lanes[i, j])
    # hoisting: join of per-iteration temporaries places (i, j) at 1024*i + j
    w = np.arange(3 * 1024, dtype=np.uint32).reshape(3, 1024)
    joined = eval_numpy.evaluate("(join w)", {"w": w})
    for i in range(3):
        for j in (0, 5, 1023):
            assert joined[eval(maps["hoisted_tmp"], {"i": i, "j": j})] == w[i, j]


def test_zero_extension_is_invisible_to_plain_folds():
    # A ragged length is read as the input extended with zeros.  Pin: the
    # extended evaluation equals the same strategy evaluated on the same
    # values placed in a longer zero-filled vector by hand, and the
    # extension adds exactly nothing (integer-valued data: exact sums).
    g = np.random.default_rng(35)
    for n in (1, 7, 100, 1000, 4097):
        x = g.integers(-8, 9, n).astype(np.float32)
        y = g.integers(-8, 9, n).astype(np.float32)
        for p in (S.Plan(seq=16, lanes=16), S.Plan(seq=5, lanes=3, combine="seq", order="strided")):
            m = S.extended_length(n, p.chunk)
            xz = np.zeros(m, np.float32)
            yz = np.zeros(m, np.float32)
            xz[:n], yz[:n] = x, y
            assert same_bits(S.dot(x, y, p), S.dot(xz, yz, p))
            assert float(S.dot(x, y, p)) == float(np.dot(x.astype(np.int64), y.astype(np.int64)))
            assert same_bits(S.asum(x, p), S.asum(xz, p))
    # the padding never yields -0 even when every product is -0
    x = -np.ones(10, np.float32)
    y = np.zeros(10, np.float32)
    assert np.float32(S.dot(x, y, S.Plan(seq=4, lanes=4))).view(np.uint32) == 0
    with pytest.raises(ValueError):
        S.dot(np.ones(10, np.float32), np.ones(10, np.float32), S.Plan(seq=4, lanes=4, accum="kahan"))


def test_scal_is_one_rounded_product_per_element():
    # scal maps alpha * x over the vector: each element is one binary32
    # product (numpy's own binary32 multiply), for both evaluators
    g = np.random.default_rng(36)
    x = (g.standard_normal(500) * 2.0 ** g.uniform(-30, 30, 500)).astype(np.float32)
    a = np.float32(1.7)
    assert same_bits(S.scal(a, x), a * x)
    assert same_bits(eval_scalar.evaluate(S.scal_expr(), {"alpha": a, "xs": x[:50]}), a * x[:50])
    assert same_bits(S.scal(np.float32(1), x), x)
    assert same_bits(S.scal(np.float32(-2), x), np.float32(-2) * x)


def test_blas_gemv_reduces_to_gemv_and_to_exact_integers():
    # y := alpha A x + beta y.  (1) alpha = 1, beta = 0 is the plain gemv
    # (1 * v = v exactly).  (2) alpha = -2 scales exactly (power of two, no
    # overflow).  (3) With small integers every product and sum is exactly
    # representable, so the result equals the integer arithmetic.  (4) beta = 0
    # never reads y: NaN in y does not reach the result.
    g = np.random.default_rng(37)
    m, k = 8, 96
    p = S.Plan(seq=3, lanes=16, rows=2, row_parts=2)
    A = g.standard_normal((m, k)).astype(np.float32)
    x = g.standard_normal(k).astype(np.float32)
    y0 = g.standard_normal(m).astype(np.float32)
    plain = S.gemv(A, x, p)
    assert same_bits(S.gemv_blas(1.0, A, x, 0.0, y0, p), plain)
    assert same_bits(S.gemv_blas(-2.0, A, x, 0.0, y0, p), np.float32(-2) * plain)
    nan_y = np.full(m, np.nan, np.float32)
    assert same_bits(S.gemv_blas(1.5, A, x, 0.0, nan_y, p), S.gemv_blas(1.5, A, x, 0.0, y0, p))
    Ai = g.integers(-8, 9, (m, k))
    xi = g.integers(-8, 9, k)
    yi = g.integers(-100, 101, m)
    want = 3 * (Ai @ xi) - 5 * yi
    got = S.gemv_blas(3.0, Ai.astype(np.float32), xi.astype(np.float32), -5.0,
                      yi.astype(np.float32), p)
    assert np.array_equal(np.asarray(got, np.float64), want.astype(np.float64))
    # both evaluators, fp8 rows: alpha * (scale * rowsum) + beta * y
    codes8 = g.integers(0, 256, (m, k)).astype(np.uint8)
    codes8[(codes8 & 0x7F) == 0x7F] = 0x38
    scale = g.random(m, dtype=np.float32) + np.float32(0.5)
    r8 = S.gemv(codes8, x, p, a_format="fp8", scale=scale)
    a, b = np.float32(0.7), np.float32(-1.3)
    y8 = S.gemv_blas(a, codes8, x, b, y0, p, a_format="fp8", scale=scale)
    assert same_bits(y8, (a * r8) + (b * y0))
    e = S.gemv_blas_expr(m, k, p, "fp8")
    assert same_bits(eval_scalar.evaluate(e, {"A": codes8, "x": x, "scale": scale, "alpha": a,
                                              "beta": b, "yin": y0}), y8)


# ----------------------------------------------------------- vector strategies

@pytest.mark.parametrize("ev", EVALS)
def test_as_vector_and_as_scalar_move_indices_only(ev):
    # asVector n: vector i holds elements i*n .. i*n+n-1; asScalar n: element
    # i is component i mod n of vector i div n; one undoes the other.
    x = np.arange(24, dtype=np.float32) * np.float32(0.5)
    v = ev("(map (lam (q) q) (asVector 4 xs))", {"xs": x})
    assert np.array_equal(np.asarray(v), x.reshape(6, 4))
    assert same_bits(ev("(asScalar 4 (asVector 4 xs))", {"xs": x}), x)
    assert same_bits(ev("(asScalar 3 (map (lam (q) (+ q q)) (asVector 3 xs)))", {"xs": x}), x + x)
    b = ev("(broadcast 5 (* a a))", {"a": np.float32(3)})
    assert same_bits(b, np.full(5, 9, np.float32))
    with pytest.raises(ValueError):
        ev("(asVector 5 xs)", {"xs": x})
    with pytest.raises(ValueError):       # a vector plus a number is not defined
        ev("(map (lam (q) (+ q 1)) (asVector 4 xs))", {"xs": x})


def _loops_vector_dot(xs, ys, V, L, C, order, combine):
    """The vector strategy as plain loops over binary32 numpy scalars: lane l
    of chunk g keeps V component sums; component j of step k reads vector
    g*L*C + l*C + k (contiguous) or g*L*C + k*L + l (strided), element
    V*vector + j.  combine "none" writes every lane's components out;
    "seq" folds lanes 0..L-1 per component.  Then one fold over the list."""
    G = len(xs) // (V * L * C)
    out = []
    for g in range(G):
        lanes = []
        for l in range(L):
            acc = [np.float32(0)] * V
            for k in range(C):
                vi = g * L * C + (l * C + k if order == "contiguous" else k * L + l)
                for j in range(V):
                    e = V * vi + j
                    acc[j] = xs[e] * ys[e] + acc[j]
            lanes.append(acc)
        if combine == "none":
            for acc in lanes:
                out.extend(acc)
        else:
            comp = [np.float32(0)] * V
            for acc in lanes:
                for j in range(V):
                    comp[j] = acc[j] + comp[j]
            out.extend(comp)
    r = np.float32(0)
    for t in out:
        r = t + r
    return r


@pytest.mark.parametrize("order", ["contiguous", "strided"])
@pytest.mark.parametrize("combine", ["none", "seq"])
@pytest.mark.parametrize("V", [1, 2, 4])
def test_vector_strategies_match_plain_loops(order, combine, V):
    # Sec. 6.2's dot expression keeps a float4 accumulator per work-item over
    # asVector 4 views and writes every work-item's value out; the oracle's
    # vector strategies against the same computation written as loops.
    xs, ys = discriminating_dot_inputs(50 + V, V * 8 * 6 * 5)
    p = S.Plan(seq=6, lanes=8, order=order, combine=combine, vec=V)
    want = _loops_vector_dot(xs, ys, V, 8, 6, order, combine)
    assert same_bits(S.dot(xs, ys, p), want)
    e = S.dot_expr(len(xs), p)
    assert same_bits(eval_scalar.evaluate(e, {"xs": xs, "ys": ys}), want)


def test_vector_tree_is_the_scalar_tree_per_component():
    # Component j of a V-wide strategy is the scalar strategy on the
    # elements j, j+V, ...: the chunk values of the vector strategy are, per
    # chunk and component, the scalar chunk values of the de-interleaved
    # inputs, folded in chunk-then-component order.
    V, L, C, G = 4, 8, 5, 3
    xs, ys = discriminating_dot_inputs(61, V * L * C * G)
    for order in ("contiguous", "strided"):
        pv = S.Plan(seq=C, lanes=L, order=order, combine="tree", vec=V)
        p1 = S.Plan(seq=C, lanes=L, order=order, combine="tree")
        chunk_expr = (f"(mapWorkgroup (lam (ch) {S._chunk_value('ch', p1, S.MUL_ADD)})"
                      f" (split {L * C} (zip xs ys)))")
        per_comp = [eval_numpy.evaluate(chunk_expr, {"xs": xs[j::V], "ys": ys[j::V]})
                    for j in range(V)]
        r = np.float32(0)
        for g in range(G):
            for j in range(V):
                r = per_comp[j][g] + r
        assert same_bits(S.dot(xs, ys, pv), r), order


def test_vector_lanes_are_adjacent_scalar_lanes():
    # Uncombined strategies: a strided V-wide strategy with L lanes reads and
    # folds exactly like the scalar strided one with V*L lanes (vector lane
    # l component j = scalar lane V*l + j), and a contiguous V-wide one like
    # the scalar strided strategy with V lanes on chunks of one lane's row.
    V, L, C = 4, 8, 6
    xs, ys = discriminating_dot_inputs(62, V * L * C * 7)
    strided_v = S.dot(xs, ys, S.Plan(seq=C, lanes=L, order="strided", combine="none", vec=V))
    assert same_bits(strided_v, S.dot(xs, ys, S.Plan(seq=C, lanes=V * L, order="strided",
                                                     combine="none")))
    contig_v = S.dot(xs, ys, S.Plan(seq=C, lanes=L, order="contiguous", combine="none", vec=V))
    assert same_bits(contig_v, S.dot(xs, ys, S.Plan(seq=C, lanes=V, order="strided",
                                                    combine="none")))
    assert not same_bits(strided_v, contig_v)


def test_vector_strategies_integer_and_all_ones():
    # Exact cases: 32-bit integers (every strategy equals the modular sum) and
    # all ones with exactly representable partial sums (result = n).
    g = np.random.default_rng(63)
    n = 4 * 8 * 16 * 3
    xi = g.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    yi = g.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    want = int(sum(int(a) * int(b) for a, b in zip(xi, yi)) % (1 << 32))
    ones = np.ones(n, np.float32)
    for order in ("contiguous", "strided"):
        for combine in ("tree", "seq", "none"):
            p = S.Plan(seq=16, lanes=8, order=order, combine=combine, vec=4)
            assert int(S.dot(xi, yi, p, num="u32")) == want
            assert float(S.dot(ones, ones, p)) == n
            assert float(S.asum(-ones, p)) == n


def test_chunk_values_fold_to_the_result():
    # The outer fold of the chunk values is the strategy's value, and the
    # uncombined chunk values are the lanes' own folds (plain loops).
    xs, ys = discriminating_dot_inputs(64, 4 * 8 * 6 * 5)
    for p in (S.Plan(seq=6, lanes=8, combine="none", vec=4), S.Plan(seq=6, lanes=32),
              S.Plan(seq=24, lanes=8, order="strided", combine="seq", vec=2)):
        c = S.dot_chunks(xs, ys, p)
        r = np.float32(0)
        for v in c:
            r = v + r
        assert same_bits(S.dot(xs, ys, p), r)
    c = S.dot_chunks(xs, ys, S.Plan(seq=6, lanes=8, combine="none", vec=4))
    for i in (0, 1, 37, len(c) - 1):       # lane (g, l), component j of vector lane
        g, l, j = i // 32, (i // 4) % 8, i % 4
        acc = np.float32(0)
        for k in range(6):
            e = 4 * (g * 48 + l * 6 + k) + j
            acc = xs[e] * ys[e] + acc
        assert same_bits(c[i], acc)


# ----------------------------------------------------------- Sum2

def test_sum2_keeps_the_error_of_a_dominant_term():
    # products 2^30, 1, -2^30 folded in order: the exact sum is 1.  The plain
    # fold loses the 1 (2^30 + 1 rounds to 2^30); Kahan's step also loses it
    # (its correction -1 is absorbed when -2^30 + 1 rounds); Sum2's TwoSum
    # keeps it in c, so s + c = 0 + 1.
    xs = np.array([2.0 ** 30, 1.0, -2.0 ** 30], np.float32)
    ys = np.ones(3, np.float32)
    for ev in EVALS:
        for acc, want in (("sum2", 1.0), ("kahan", 0.0), ("plain", 0.0)):
            p = S.Plan(seq=3, lanes=1, accum=acc)
            assert float(ev(S.dot_expr(3, p), {"xs": xs, "ys": ys})) == want, (acc, ev)
        p = S.Plan(seq=3, lanes=1, accum="sum2", final_f64=True)
        assert float(ev(S.dot_expr(3, p), {"xs": xs, "ys": ys})) == 1.0


def test_sum2_meets_its_error_bound_where_plain_and_kahan_do_not():
    # Cancelling products (every rounded product has its exact negation in
    # the input, so their exact sum S is 0): Sum2's result is within
    # u|S| + gamma_h^2 * sum|p| (Ogita, Rump, Oishi 2005, Prop. 4.5, with h the
    # strategy's depth in place of n - 1), i.e. essentially 0.  The plain and
    # Kahan folds of the same strategies leave that bound (on some of them:
    # a plain fold can cancel exactly by chance).
    outside = 0
    for p in (S.Plan(seq=64, lanes=16, order="strided", accum="sum2"),
              S.Plan(seq=32, lanes=8, combine="seq", accum="sum2"),
              S.Plan(seq=16, lanes=64, accum="sum2", final_f64=True),
              S.Plan(seq=512, lanes=2, combine="seq", accum="sum2")):
        n = p.chunk * 6
        xs, ys = discriminating_dot_inputs(70, n)
        prods = (xs * ys).astype(np.float64)     # rounded products, exact in binary64
        assert math.fsum(prods.tolist()) == 0.0
        h = exact.strategy_depth(n, p.seq, p.lanes, p.combine) + 2
        bound = 2 * exact.gamma(h) ** 2 * math.fsum(np.abs(prods).tolist())
        assert abs(float(S.dot(xs, ys, p))) <= bound, p
        for acc in ("plain", "kahan"):
            q = S.Plan(seq=p.seq, lanes=p.lanes, order=p.order, combine=p.combine, accum=acc)
            outside += abs(float(S.dot(xs, ys, q))) > 10 * bound
    assert outside >= 5


def test_sum2_evaluators_agree_and_exact_cases():
    g = np.random.default_rng(71)
    x = (g.standard_normal(96) * 2.0 ** g.uniform(-20, 20, 96)).astype(np.float32)
    y = g.standard_normal(96).astype(np.float32)
    p = S.Plan(seq=6, lanes=4, order="strided", accum="sum2")
    e = S.dot_expr(96, p)
    assert same_bits(eval_scalar.evaluate(e, {"xs": x, "ys": y}),
                     eval_numpy.evaluate(e, {"xs": x, "ys": y}))
    ones = np.ones(p.chunk * 4, np.float32)
    assert float(S.dot(ones, ones, p)) == p.chunk * 4
