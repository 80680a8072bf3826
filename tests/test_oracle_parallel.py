"""The parallel evaluation of the oracle (oracle/parallel.py: the outermost
map split over worker processes, the outer fold once) gives the serial
oracle's bits for every strategy shape and for ragged lengths."""

import numpy as np
import pytest

import synthetic
from oracle import parallel as P
from oracle import strategies as S

PLANS = [
    S.Plan(seq=16, lanes=16, order="contiguous", combine="tree"),
    S.Plan(seq=8, lanes=32, order="strided", combine="seq"),
    S.Plan(seq=4, lanes=8, order="strided", combine="none"),
    S.Plan(seq=8, lanes=4, order="contiguous", combine="tree", vec=4),
    S.Plan(seq=32, lanes=1, order="contiguous", combine="seq"),
]
# one length that every plan's chunk divides (the chunks are 128 .. 256
# numbers), less a ragged tail: each plan zero-extends it to its own chunk
N = 37 * 256 - 5


def _bits(v):
    return np.asarray(v, np.float32).view(np.uint32)


@pytest.fixture(scope="module")
def inputs():
    g = synthetic.rng(77)
    x = synthetic.log_uniform_signed(g, N, -6, 6)   # discriminating magnitudes
    y = synthetic.uniform_pm1(g, N)
    # rows of 125 (one part of W = 128) and of 253 (two parts)
    A = {1: synthetic.log_uniform_signed(g, (40, 125), -6, 6),
         2: synthetic.log_uniform_signed(g, (40, 253), -6, 6)}
    xv = {1: synthetic.uniform_pm1(g, 125), 2: synthetic.uniform_pm1(g, 253)}
    return x, y, A, xv


@pytest.fixture(scope="module")
def pool(inputs):
    x, y, A, xv = inputs
    arrays = {"A1": A[1], "v1": xv[1], "A2": A[2], "v2": xv[2]}
    for i, p in enumerate(PLANS):
        n = S.extended_length(N, p.chunk)
        arrays[f"x{i}"] = S._zero_extend(x, n)
        arrays[f"y{i}"] = S._zero_extend(y, n)
    with P.Evaluator(arrays, workers=3) as ev:
        yield ev


@pytest.mark.parametrize("i", range(len(PLANS)),
                         ids=[f"C{p.seq}L{p.lanes}{p.order[0]}{p.combine}V{p.vec}" for p in PLANS])
def test_parallel_dot_and_asum_equal_the_serial_oracle(pool, inputs, i):
    x, y, _, _ = inputs
    plan = PLANS[i]
    assert _bits(pool.dot(plan, f"x{i}", f"y{i}")) == _bits(S.dot(x, y, plan))
    assert _bits(pool.asum(plan, f"x{i}")) == _bits(S.asum(x, plan))


@pytest.mark.parametrize("rows,parts", [(1, 1), (4, 1), (2, 2)])
def test_parallel_gemv_equals_the_serial_oracle(pool, inputs, rows, parts):
    _, _, A, xv = inputs
    plan = S.Plan(seq=8, lanes=16, order="strided", combine="tree", rows=rows, row_parts=parts)
    got = pool.gemv(plan, f"A{parts}", f"v{parts}")
    assert np.array_equal(_bits(got), _bits(S.gemv(A[parts], xv[parts], plan)))


def test_ranges_cover_the_iterations_in_order():
    for items, unit, parts in [(100, 10, 3), (7, 4, 16), (4096, 256, 16), (1, 1, 4)]:
        spans = P.ranges(items, unit, parts)
        assert spans[0][0] == 0 and spans[-1][1] == items
        assert all(a % unit == 0 and a < b for a, b in spans)
        assert all(spans[i][1] == spans[i + 1][0] for i in range(len(spans) - 1))
        assert len(spans) <= parts


def test_only_plain_zero_extended_reductions_are_split(pool):
    with pytest.raises(ValueError):
        pool.dot(S.Plan(seq=4, lanes=4, accum="kahan"), "x0", "y0")
    with pytest.raises(ValueError):
        pool.dot(S.Plan(seq=3, lanes=7), "x0", "y0")     # 21 does not divide the length
