"""The expression texts the generator compiles ahead of time (the catalogue)
against the oracle's own expression builders (CPU only).

The GPU tests compare each generated kernel with the oracle's builder for
the same descriptor.  Here, first, every catalogued text is checked to be the
library printer's output for that descriptor and size; then, for each
descriptor, the printer's text at a reduced size of the same structure (the
same C, L, R, V, order, combine and accumulation; fewer chunks or rows) is
evaluated by the oracle and compared bit for bit with the oracle builder's
expression on discriminating inputs."""

import numpy as np
import pytest

import paper_1710_08332_amd as dp
from oracle import eval_numpy
from oracle import strategies as S
from paper_1710_08332_amd.generator import catalog
from paper_1710_08332_amd.generator import strategies as P
from tests.gpu_util import to_plan
from tests.test_generator import disc, same

St = dp.Strategy
T_, C_ = dp.STRIDED, dp.CONTIGUOUS

# name -> (kind, descriptor, full-size arguments of the printer)
CATALOGUE = {
    "dot_strided_tree": ("dot", St(seq_len=4, local_size=64, order=T_), (4 * 64 * 37,)),
    "dot_contiguous_seq": ("dot", St(seq_len=16, local_size=32, order=C_, wg_combine=dp.SEQ),
                           (16 * 32 * 23,)),
    "dot_kahan_f64": ("dot", St(seq_len=16, local_size=64, order=T_, accum=dp.KAHAN,
                                final_f64=1), (16 * 64 * 13,)),
    "dot_sum2": ("dot", St(seq_len=16, local_size=64, order=T_, accum=dp.SUM2), (16 * 64 * 13,)),
    "dot_u32": ("dot", St(seq_len=4, local_size=16, order=C_), (4 * 16 * 29,)),
    "dot_v4_strided_tree": ("dot", St(seq_len=8, local_size=64, order=T_, vec_width=4),
                            (4 * 8 * 64 * 11,)),
    "dot_headline_2p26": ("dot", catalog.HEADLINE_DOT, (1 << 26,)),
    "asum_strided_tree": ("asum", St(seq_len=8, local_size=128, order=T_), (8 * 128 * 19,)),
    "gemv_strided_tree": ("gemv", St(seq_len=16, local_size=64, order=T_, rows_per_wg=2),
                          (96, 1024)),
    "gemv_headline_8192": ("gemv", catalog.HEADLINE_GEMV, (8192, 8192)),
    "gemv_bf16_strided_tree": ("gemv_bf16", St(seq_len=4, local_size=64, order=T_,
                                               rows_per_wg=2), (64, 256)),
    "gemv_fp8_strided_tree": ("gemv_fp8", St(seq_len=4, local_size=64, order=T_,
                                             rows_per_wg=2), (64, 256)),
    "gemv_bf16_16384": ("gemv_bf16", St(seq_len=16, local_size=1024, order=T_, rows_per_wg=2),
                        (16384, 16384)),
    "gemv_fp8_16384": ("gemv_fp8", St(seq_len=16, local_size=1024, order=T_, rows_per_wg=2),
                       (16384, 16384)),
}


def _print(kind, s, args):
    if kind == "dot":
        return P.dot_text(s, *args)
    if kind == "asum":
        return P.asum_text(s, *args)
    fmt = {"gemv": "f32", "gemv_bf16": "bf16", "gemv_fp8": "fp8"}[kind]
    return P.gemv_text(s, *args, fmt) if fmt != "f32" else P.gemv_text(s, *args)


def test_every_catalogued_text_is_the_printer_output_for_its_descriptor():
    texts = {name: text for name, text, _, _ in catalog.programs()}
    assert set(CATALOGUE) <= set(texts)
    # the rest are not printed from descriptors: the paper's own Sec. 6.2
    # expression, a map (scal), the decoders and a hoisting case
    assert set(texts) - set(CATALOGUE) == {"dot_sec62_chunks", "scal_global",
                                           "decode_bf16_all", "decode_fp8_all",
                                           "dot_global_lanes"}
    for name, (kind, s, args) in CATALOGUE.items():
        assert texts[name] == _print(kind, s, args), name


def test_the_sec62_text_is_the_oracle_builder_for_its_strategy():
    # the paper's expression as catalogued, evaluated by the oracle, against
    # the oracle builder's uncombined V = 4 strategy at the same sizes
    text = dict((n, t) for n, t, _, _ in catalog.programs())["dot_sec62_chunks"]
    plan = S.Plan(seq=2048, lanes=64, order="contiguous", combine="none", vec=4)
    n = 2 * plan.chunk
    x, y = disc(21, n)
    assert same(eval_numpy.evaluate(text, {"xs": x, "ys": y}), S.dot_chunks(x, y, plan))


@pytest.mark.parametrize("name", sorted(CATALOGUE))
def test_catalogued_descriptor_at_a_reduced_size_equals_the_oracle_builder(name):
    kind, s, _ = CATALOGUE[name]
    p = to_plan(s)
    g = np.random.default_rng(len(name))
    if kind in ("dot", "asum"):
        n = 3 * p.chunk
        if name == "dot_u32":
            x = g.integers(0, 2 ** 32, n, dtype=np.uint32)
            y = g.integers(0, 2 ** 32, n, dtype=np.uint32)
            got = eval_numpy.evaluate(P.dot_text(s, n), {"xs": x, "ys": y}, "u32")
            assert same(got, S.dot(x, y, p, num="u32"))
            return
        x, y = disc(11, n)
        if kind == "asum":
            assert same(eval_numpy.evaluate(P.asum_text(s, n), {"xs": x}), S.asum(x, p))
        else:
            assert same(eval_numpy.evaluate(P.dot_text(s, n), {"xs": x, "ys": y}),
                        S.dot(x, y, p))
        return
    m, k = 2 * s.rows_per_wg, p.chunk * p.row_parts
    x = (g.standard_normal(k) * 2.0 ** g.uniform(-8, 8, k)).astype(np.float32)
    if kind == "gemv":
        A = (g.standard_normal((m, k)) * 2.0 ** g.uniform(-8, 8, (m, k))).astype(np.float32)
        got = eval_numpy.evaluate(P.gemv_text(s, m, k), {"A": A, "x": x})
        assert same(got, S.gemv(A, x, p))
    elif kind == "gemv_bf16":
        codes = g.integers(0, 2 ** 16, (m, k)).astype(np.uint16)
        codes[(codes & 0x7F80) == 0x7F80] = 0x3F80          # no inf / NaN codes
        got = eval_numpy.evaluate(P.gemv_text(s, m, k, "bf16"), {"A": codes, "x": x})
        assert same(got, S.gemv(codes, x, p, a_format="bf16"))
    else:
        codes = g.integers(0, 256, (m, k)).astype(np.uint8)
        codes[(codes & 0x7F) == 0x7F] = 0x38                 # no NaN codes
        scale = (g.random(m) + 0.5).astype(np.float32)
        got = eval_numpy.evaluate(P.gemv_text(s, m, k, "fp8"),
                                  {"A": codes, "x": x, "scale": scale})
        assert same(got, S.gemv(codes, x, p, a_format="fp8", scale=scale))
