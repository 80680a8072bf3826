"""The two oracle evaluators agree bit for bit on random small strategies,
and the oracle stays independent of the HIP library."""

import ast
import os

import numpy as np
from hypothesis import given, settings, strategies as st

from oracle import eval_numpy, eval_scalar
from oracle import strategies as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pow2 = st.sampled_from([1, 2, 4, 8])


@st.composite
def plans(draw, kahan=False):
    lanes = draw(pow2)
    return S.Plan(seq=draw(st.sampled_from([1, 2, 3, 4, 8])), lanes=lanes,
                  order=draw(st.sampled_from(["contiguous", "strided"])),
                  combine=draw(st.sampled_from(["tree", "seq"])),
                  accum="kahan" if kahan else "plain",
                  final_f64=draw(st.booleans()) if kahan else False)


def _bits(a):
    a = np.asarray(a)
    return a.view(np.uint64) if a.dtype == np.float64 else (a.view(np.uint32) if a.dtype == np.float32 else a)


@settings(max_examples=60, deadline=None)
@given(plans(), st.integers(1, 4), st.integers(0, 2 ** 31), st.sampled_from(["f32", "u32"]))
def test_dot_and_asum_evaluators_agree(plan, chunks, seed, num):
    g = np.random.default_rng(seed)
    n = plan.chunk * chunks
    if num == "f32":
        x = (g.standard_normal(n) * 2.0 ** g.uniform(-12, 12, n)).astype(np.float32)
        y = g.standard_normal(n).astype(np.float32)
    else:
        x = g.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
        y = g.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    e = S.dot_expr(n, plan)
    a = eval_numpy.evaluate(e, {"xs": x, "ys": y}, num)
    b = eval_scalar.evaluate(e, {"xs": x, "ys": y}, num)
    assert np.array_equal(_bits(a), _bits(b))
    if num == "f32":
        e = S.asum_expr(n, plan)
        assert np.array_equal(_bits(eval_numpy.evaluate(e, {"xs": x})),
                              _bits(eval_scalar.evaluate(e, {"xs": x})))


@settings(max_examples=30, deadline=None)
@given(plans(kahan=True), st.integers(1, 3), st.integers(0, 2 ** 31))
def test_kahan_evaluators_agree(plan, chunks, seed):
    g = np.random.default_rng(seed)
    n = plan.chunk * chunks
    x = (g.standard_normal(n) * 10.0 ** g.uniform(-4, 4, n)).astype(np.float32)
    y = (g.standard_normal(n) * 10.0 ** g.uniform(-4, 4, n)).astype(np.float32)
    e = S.dot_expr(n, plan)
    a = eval_numpy.evaluate(e, {"xs": x, "ys": y})
    b = eval_scalar.evaluate(e, {"xs": x, "ys": y})
    assert a.dtype == (np.float64 if plan.final_f64 else np.float32)
    assert np.array_equal(_bits(a), _bits(b))


@settings(max_examples=30, deadline=None)
@given(plans(), st.integers(1, 3), st.sampled_from([1, 2]), st.sampled_from([1, 2]),
       st.sampled_from(["f32", "bf16", "fp8"]), st.integers(0, 2 ** 31))
def test_gemv_evaluators_agree(plan, groups, rows, parts, fmt, seed):
    from dataclasses import replace
    plan = replace(plan, rows=rows, row_parts=parts)
    g = np.random.default_rng(seed)
    m = rows * groups
    k = plan.chunk * parts
    x = g.standard_normal(k).astype(np.float32)
    inputs = {"x": x}
    if fmt == "f32":
        inputs["A"] = g.standard_normal((m, k)).astype(np.float32)
    elif fmt == "bf16":
        a = g.integers(0, 2 ** 16, (m, k)).astype(np.uint16)
        a[(a & 0x7F80) == 0x7F80] = 0
        inputs["A"] = a
    else:
        a = g.integers(0, 256, (m, k)).astype(np.uint8)
        a[(a & 0x7F) == 0x7F] = 0
        inputs["A"] = a
        inputs["scale"] = g.random(m, dtype=np.float32)
    e = S.gemv_expr(m, k, plan, fmt)
    assert np.array_equal(_bits(eval_numpy.evaluate(e, inputs)), _bits(eval_scalar.evaluate(e, inputs)))


def test_oracle_imports_nothing_from_the_hip_library():
    odir = os.path.join(ROOT, "oracle")
    for fn in os.listdir(odir):
        if not fn.endswith(".py"):
            continue
        tree = ast.parse(open(os.path.join(odir, fn)).read())
        for node in ast.walk(tree):
            names = []
            if isinstance(node, ast.Import):
                names = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                names = [node.module or ""]
            for nm in names:
                assert not nm.startswith("paper_1710_08332_amd"), (fn, nm)
                assert not nm.startswith("synthetic"), (fn, nm)
                assert nm not in ("torch", "ctypes"), (fn, nm)
