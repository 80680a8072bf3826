"""The library's strategy printer against the oracle's expression builder:
for each descriptor both texts, evaluated by the oracle, give the same bits."""

import numpy as np
import pytest

import paper_1710_08332_amd as dp
from oracle import eval_numpy
from oracle import strategies as S
from paper_1710_08332_amd.generator import strategies as P
from tests.gpu_util import to_plan
from tests.test_generator import disc, same

C_, T_ = dp.CONTIGUOUS, dp.STRIDED
DESCS = [
    dp.Strategy(seq_len=4, local_size=8, order=T_),
    dp.Strategy(seq_len=3, local_size=5, order=C_, wg_combine=dp.SEQ),
    dp.Strategy(seq_len=2, local_size=16, order=C_),
    dp.Strategy(seq_len=3, local_size=4, order=C_, wg_combine=dp.NONE, vec_width=4),
    dp.Strategy(seq_len=2, local_size=8, order=T_, vec_width=2),
    dp.Strategy(seq_len=5, local_size=1),
    dp.Strategy(seq_len=2, local_size=4, order=T_, accum=dp.KAHAN, final_f64=1),
    dp.Strategy(seq_len=4, local_size=2, accum=dp.KAHAN),
    dp.Strategy(seq_len=4, local_size=4, order=T_, accum=dp.SUM2),
    dp.Strategy(seq_len=2, local_size=8, wg_combine=dp.SEQ, accum=dp.SUM2, final_f64=1),
]


@pytest.mark.parametrize("s", DESCS, ids=str)
def test_printed_reductions_equal_the_oracle_expressions(s):
    p = to_plan(s)
    n = p.chunk * 3
    x, y = disc(13, n)
    got = eval_numpy.evaluate(P.dot_text(s, n), {"xs": x, "ys": y})
    assert same(got, S.dot(x, y, p))
    if s.accum == dp.PLAIN:
        assert same(eval_numpy.evaluate(P.asum_text(s, n), {"xs": x}), S.asum(x, p))
        assert same(eval_numpy.evaluate(P.dot_chunks_text(s, n), {"xs": x, "ys": y}),
                    S.dot_chunks(x, y, p))


@pytest.mark.parametrize("s", [dp.Strategy(seq_len=4, local_size=8, order=T_, rows_per_wg=2),
                               dp.Strategy(seq_len=3, local_size=4, wg_combine=dp.SEQ,
                                           row_parts=2)], ids=str)
def test_printed_gemv_equals_the_oracle_expression(s):
    p = to_plan(s)
    m, k = 2 * s.rows_per_wg, p.chunk * p.row_parts
    g = np.random.default_rng(2)
    A = g.standard_normal((m, k)).astype(np.float32)
    x = g.standard_normal(k).astype(np.float32)
    assert same(eval_numpy.evaluate(P.gemv_text(s, m, k), {"A": A, "x": x}), S.gemv(A, x, p))


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_printed_low_precision_gemv_equals_the_oracle_expression(fmt):
    # the printer fuses the decode into the lane step; the oracle decodes
    # with a map first: the same values
    s = dp.Strategy(seq_len=4, local_size=8, order=T_, rows_per_wg=2)
    p = to_plan(s)
    m, k = 4, p.chunk
    g = np.random.default_rng(3)
    x = g.standard_normal(k).astype(np.float32)
    if fmt == "bf16":
        codes = g.integers(0, 2 ** 16, (m, k)).astype(np.uint16)
        codes[(codes & 0x7F80) == 0x7F80] = 0x3F80
        inp, scale = {"A": codes, "x": x}, None
    else:
        codes = g.integers(0, 256, (m, k)).astype(np.uint8)
        codes[(codes & 0x7F) == 0x7F] = 0x38
        scale = g.random(m, dtype=np.float32) + np.float32(0.5)
        inp = {"A": codes, "x": x, "scale": scale}
    got = eval_numpy.evaluate(P.gemv_text(s, m, k, fmt), inp)
    assert same(got, S.gemv(codes, x, p, a_format=fmt, scale=scale))
