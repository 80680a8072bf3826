"""Parity of the HIP path (called through the C ABI) with the CPU oracle.

Every comparison is bit for bit: for binary32 and integer strategies the
strategy fixes every rounding, so the GPU must reproduce the oracle's value
of the same DPIA expression exactly.  Inputs come from ``synthetic`` (the
seeded generators both sides share) plus cancelling inputs on which
different associations give different bits."""

import numpy as np
import pytest

import paper_1710_08332_amd as dp
import synthetic
from oracle import exact, formats
from oracle import strategies as S
from tests.gpu_util import (assert_same_bits, cuda, discriminating, gpu_asum, gpu_dot, gpu_gemv,
                            to_plan)

pytestmark = pytest.mark.gpu

C_, T_ = dp.CONTIGUOUS, dp.STRIDED
TREE, SEQ = dp.TREE, dp.SEQ

# (seq_len C, local_size L, order, combine) spanning: one lane, lanes inside
# one thread, teams smaller than / equal to / larger than a wavefront,
# non-power-of-two lanes (sequential combine), C not a multiple of the
# vector width, and the config-1 strategy (C=256, L=16, contiguous, tree).
STRATS = [
    (256, 16, C_, TREE), (256, 16, T_, TREE), (256, 16, C_, SEQ), (256, 16, T_, SEQ),
    (1, 1, C_, SEQ), (7, 1, C_, TREE), (3, 4, T_, TREE), (5, 2, C_, TREE), (6, 2, T_, SEQ),
    (4, 64, C_, TREE), (4, 64, T_, TREE), (16, 256, T_, TREE), (16, 256, C_, TREE),
    (8, 128, C_, SEQ), (8, 512, T_, TREE), (2, 1024, C_, TREE), (2, 4096, T_, TREE),
    (3, 12, T_, SEQ), (9, 3, C_, SEQ), (64, 1024, T_, SEQ), (33, 32, C_, TREE),
    (1024, 8, T_, TREE), (8192, 2, C_, TREE), (64, 256, T_, TREE),
]


def _ids(s):
    C, L, o, c = s
    return f"C{C}-L{L}-{'str' if o == T_ else 'con'}-{'tree' if c == TREE else 'seq'}"


@pytest.mark.parametrize("strat", STRATS, ids=_ids)
@pytest.mark.parametrize("passes", [1, 2])
def test_dot_and_asum_bit_exact(strat, passes):
    C, L, order, comb = strat
    s = dp.Strategy(seq_len=C, local_size=L, order=order, wg_combine=comb, passes=passes)
    W = C * L
    G = max(1, min(37, (1 << 18) // W))         # several tiles and a ragged tail
    n = W * G
    x, y = synthetic.dot_inputs(n, synthetic.SEEDS["small"])
    plan = to_plan(s)
    assert_same_bits(gpu_dot(x, y, s), S.dot(x, y, plan), f"dot uniform n={n}")
    xd, yd = discriminating(7, n)
    assert_same_bits(gpu_dot(xd, yd, s), S.dot(xd, yd, plan), f"dot cancelling n={n}")
    assert_same_bits(gpu_asum(x, s), S.asum(x, plan), f"asum n={n}")


# Small teams over many chunks: several teams share a work-group (few chunks
# are spread one wavefront per work-group, so the small cases above run
# unpacked) and the last work-group and the last chunk are only partly
# filled.
@pytest.mark.parametrize("strat", [(4, 16, C_, TREE), (4, 16, T_, TREE), (2, 32, T_, SEQ),
                                   (16, 16, C_, TREE), (16, 16, C_, SEQ)], ids=_ids)
@pytest.mark.parametrize("passes", [1, 2])
def test_packed_small_teams_with_ragged_last_workgroup(strat, passes):
    C, L, order, comb = strat
    s = dp.Strategy(seq_len=C, local_size=L, order=order, wg_combine=comb, passes=passes)
    W = C * L
    n = W * 4101 + W // 3 + 1
    x, y = synthetic.dot_inputs(n, synthetic.SEEDS["small"])
    plan = to_plan(s)
    assert_same_bits(gpu_dot(x, y, s), S.dot(x, y, plan), f"dot packed n={n}")
    xd, yd = discriminating(11, n)
    assert_same_bits(gpu_dot(xd, yd, s), S.dot(xd, yd, plan), f"dot packed cancelling n={n}")
    assert_same_bits(gpu_asum(x, s), S.asum(x, plan), f"asum packed n={n}")


def test_config1_dot_and_asum_at_full_size():
    # N = 2^20, split 4096 -> mapWorkgroup (split 256 -> mapLocal reduceSeq)
    # -> tree in local memory -> second-pass reduceSeq
    n = 1 << 20
    x, y = synthetic.dot_inputs(n, synthetic.SEEDS["small"])
    for passes in (2, 1):
        s = dp.Strategy(seq_len=256, local_size=16, order=C_, wg_combine=TREE, passes=passes)
        plan = to_plan(s)
        assert_same_bits(gpu_dot(x, y, s), S.dot(x, y, plan), "config-1 dot")
        assert_same_bits(gpu_asum(x, s), S.asum(x, plan), "config-1 asum")


@pytest.mark.parametrize("max_grid", [1, 2, 3, 7, 64])
def test_physical_grid_changes_no_bits(max_grid):
    n = 1 << 18
    xd, yd = discriminating(11, n)
    for passes in (1, 2):
        base = dp.Strategy(seq_len=64, local_size=64, order=T_, passes=passes)
        want = S.dot(xd, yd, to_plan(base))
        assert_same_bits(gpu_dot(xd, yd, base.with_(max_grid=max_grid)), want, f"grid {max_grid}")


def test_repeated_calls_are_bit_identical_and_reuse_the_workspace():
    import torch
    n = 1 << 20
    xd, yd = discriminating(12, n)
    s = dp.Strategy(seq_len=128, local_size=64, order=C_, passes=1)
    want = S.dot(xd, yd, to_plan(s))
    xt, yt = torch.from_numpy(xd).cuda(), torch.from_numpy(yd).cuda()
    ws = dp.workspace(s, dp.OP_DOT, dp.F32, 0, n)
    outs = [dp.dot(xt, yt, s, ws=ws) for _ in range(20)]
    torch.cuda.synchronize()
    for o in outs:
        assert_same_bits(o.cpu().numpy()[0], want, "repeat")


def test_many_chunk_results_fold_across_staging_blocks():
    # G = 5000 chunk results > one LDS staging block of the final fold
    s = dp.Strategy(seq_len=4, local_size=4, order=T_, wg_combine=SEQ)
    n = 16 * 5000
    xd, yd = discriminating(13, n)
    for passes in (1, 2):
        assert_same_bits(gpu_dot(xd, yd, s.with_(passes=passes)),
                         S.dot(xd, yd, to_plan(s)), f"G=5000 passes={passes}")


def test_empty_vector_gives_positive_zero():
    s = dp.Strategy(seq_len=4, local_size=16)
    for passes in (1, 2):
        r = gpu_dot(np.zeros(0, np.float32), np.zeros(0, np.float32), s.with_(passes=passes))
        assert r.view(np.uint32) == 0
        assert gpu_asum(np.zeros(0, np.float32), s.with_(passes=passes)).view(np.uint32) == 0


@pytest.mark.parametrize("strat", STRATS[:12], ids=_ids)
def test_integer_dot_is_exact(strat):
    C, L, order, comb = strat
    s = dp.Strategy(seq_len=C, local_size=L, order=order, wg_combine=comb)
    n = C * L * 11
    g = np.random.default_rng(5)
    x = synthetic.integers_u32(g, n)
    y = synthetic.integers_u32(g, n)
    want = sum(int(a) * int(b) for a, b in zip(x.tolist(), y.tolist())) % 2 ** 32
    got = gpu_dot(x, y, s)
    assert int(got) == want
    assert int(got) == int(S.dot(x, y, to_plan(s), num="u32"))


@pytest.mark.parametrize("strat", [(256, 16, C_, TREE), (64, 256, T_, TREE), (16, 64, C_, SEQ),
                                   (5, 4, T_, SEQ), (32, 128, T_, TREE)], ids=_ids)
@pytest.mark.parametrize("final_f64", [0, 1])
@pytest.mark.parametrize("accum", [dp.KAHAN, dp.SUM2], ids=["kahan", "sum2"])
def test_kahan_dot_bit_exact(strat, final_f64, accum):
    C, L, order, comb = strat
    s = dp.Strategy(seq_len=C, local_size=L, order=order, wg_combine=comb, accum=accum,
                    final_f64=final_f64)
    n = C * L * 19
    x, y = synthetic.kahan_dot_inputs(n, synthetic.SEEDS["precision"])
    want = S.dot(x, y, to_plan(s))
    for passes in (1, 2):
        got = gpu_dot(x, y, s.with_(passes=passes))
        assert_same_bits(got, want, "kahan")
    if final_f64:
        got32 = gpu_dot(x, y, s, out_dtype=__import__("torch").float32)
        assert_same_bits(got32, np.float32(want), "kahan f64 rounded to f32")
    err = abs(float(want) - exact.dot_exact(x, y)) / exact.dot_abs_terms(x, y)
    assert err < 1e-6


GEMV_STRATS = [
    dict(seq_len=64, local_size=16, order=T_, wg_combine=TREE, rows_per_wg=1),
    dict(seq_len=8, local_size=128, order=C_, wg_combine=SEQ, rows_per_wg=2),
    dict(seq_len=16, local_size=64, order=T_, wg_combine=TREE, rows_per_wg=4, row_parts=2),
    dict(seq_len=3, local_size=5, order=C_, wg_combine=SEQ, rows_per_wg=1),
    dict(seq_len=32, local_size=256, order=T_, wg_combine=TREE, rows_per_wg=1),
    dict(seq_len=4, local_size=256, order=C_, wg_combine=TREE, rows_per_wg=1, row_parts=2),
    dict(seq_len=512, local_size=2, order=T_, wg_combine=TREE, rows_per_wg=8),
    dict(seq_len=32, local_size=128, order=C_, wg_combine=TREE, rows_per_wg=2),   # LDS staged
    dict(seq_len=16, local_size=64, order=C_, wg_combine=SEQ, rows_per_wg=1, row_parts=2),
]


@pytest.mark.parametrize("kw", GEMV_STRATS, ids=lambda k: "-".join(f"{a[:3]}{b}" for a, b in k.items()))
@pytest.mark.parametrize("fmt", ["f32", "bf16", "fp8", "i32"])
def test_gemv_bit_exact(kw, fmt):
    s = dp.Strategy(**kw)
    plan = to_plan(s)
    k = s.seq_len * s.local_size * s.row_parts
    m = s.rows_per_wg * 13
    A, x = synthetic.gemv_inputs(m, k, synthetic.SEEDS["scale"])
    if fmt == "f32":
        assert_same_bits(gpu_gemv(A, x, s), S.gemv(A, x, plan), "gemv f32")
    elif fmt == "bf16":
        codes = synthetic.quantise_bf16(A)
        assert_same_bits(gpu_gemv(codes, x, s, a_dtype=dp.BF16),
                         S.gemv(codes, x, plan, a_format="bf16"), "gemv bf16")
    elif fmt == "fp8":
        codes, scale = synthetic.quantise_fp8_rows(A)
        assert_same_bits(gpu_gemv(codes, x, s, a_dtype=dp.FP8_E4M3, scale=scale),
                         S.gemv(codes, x, plan, a_format="fp8", scale=scale), "gemv fp8")
    else:
        g = np.random.default_rng(9)
        Ai = synthetic.integers_u32(g, (m, k))
        xi = synthetic.integers_u32(g, k)
        assert_same_bits(gpu_gemv(Ai, xi, s), S.gemv(Ai, xi, plan, num="u32"), "gemv i32")


def test_gemv_leading_dimension_larger_than_k():
    s = dp.Strategy(seq_len=16, local_size=16, order=T_)
    m, k, lda = 24, 256, 300
    A, x = synthetic.gemv_inputs(m, lda, 3)
    import torch
    At = torch.from_numpy(A).cuda()[:, :k]
    y = dp.gemv(At, torch.from_numpy(x[:k].copy()).cuda(), s)
    torch.cuda.synchronize()
    assert_same_bits(y.cpu().numpy(), S.gemv(np.ascontiguousarray(A[:, :k]), x[:k], to_plan(s)),
                     "gemv lda")


def test_fp8_decoding_exhaustive_through_gemv():
    # row r holds code r in column 0 and +0 codes elsewhere, x = 1: every
    # lane adds exact zeros to code r's value, so y[r] is the decoded value
    s = dp.Strategy(seq_len=1, local_size=16, order=T_)
    A = np.zeros((256, 16), np.uint8)
    A[:, 0] = np.arange(256, dtype=np.uint8)
    x = np.ones(16, np.float32)
    scale = np.ones(256, np.float32)
    y = gpu_gemv(A, x, s, a_dtype=dp.FP8_E4M3, scale=scale)
    table = formats.FP8_E4M3_TABLE + np.float32(0)      # -0 + 0 = +0
    nan = np.isnan(table)
    assert np.array_equal(np.isnan(y), nan)
    assert_same_bits(y[~nan], table[~nan], "fp8 table")
    want = S.gemv(A, x, to_plan(s), a_format="fp8", scale=scale)
    assert np.array_equal(np.isnan(want), nan)
    assert_same_bits(y[~nan], want[~nan], "fp8 oracle")


def test_bf16_decoding_exhaustive_through_gemv():
    s = dp.Strategy(seq_len=1, local_size=16, order=T_, rows_per_wg=4)
    A = np.zeros((65536, 16), np.uint16)
    A[:, 0] = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    x = np.ones(16, np.float32)
    y = gpu_gemv(A, x, s, a_dtype=dp.BF16)
    with np.errstate(invalid="ignore"):
        table = formats.bf16_decode(A[:, 0]) + np.float32(0)
    nan = np.isnan(table)
    assert np.array_equal(np.isnan(y), nan)
    assert_same_bits(y[~nan], table[~nan], "bf16 table")


def test_config2_dot_and_gemv_at_full_size():
    # dot N = 2^26 and gemv 8192 x 8192, the measured workload's strategies
    import bench
    n = 1 << 26
    x, y = synthetic.dot_inputs(n, synthetic.SEEDS["scale"])
    s = bench.DOT_STRATEGY
    assert_same_bits(gpu_dot(x, y, s), S.dot(x, y, to_plan(s)), "dot 2^26")
    A, xv = synthetic.gemv_inputs(8192, 8192, synthetic.SEEDS["scale"])
    g = bench.GEMV_STRATEGY
    assert_same_bits(gpu_gemv(A, xv, g), S.gemv(A, xv, to_plan(g)), "gemv 8192^2")


@pytest.mark.parametrize("kw", [dict(seq_len=256, local_size=1024, order=T_),
                                dict(seq_len=64, local_size=16, order=C_, wg_combine=SEQ),
                                dict(seq_len=32, local_size=128, order=T_, accum=dp.KAHAN),
                                dict(seq_len=32, local_size=128, order=T_, accum=dp.SUM2),
                                dict(seq_len=32, local_size=128, order=C_, accum=dp.KAHAN,
                                     final_f64=1)], ids=str)
def test_chunks_then_fold_equals_one_call(kw):
    import torch
    s = dp.Strategy(**kw)
    n = s.seq_len * s.local_size * 23
    x, y = discriminating(17, n)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    c = dp.chunks(dp.OP_DOT, s, xt, yt)
    r = dp.fold(dp.OP_DOT, s, c, n, dp.F32)
    torch.cuda.synchronize()
    want = S.dot(x, y, to_plan(s))
    assert_same_bits(r.cpu().numpy()[0], want, "chunks+fold")
    assert_same_bits(gpu_dot(x, y, s), want, "dot")
    if s.accum == dp.PLAIN:
        ca = dp.chunks(dp.OP_ASUM, s, xt)
        ra = dp.fold(dp.OP_ASUM, s, ca, n, dp.F32)
        torch.cuda.synchronize()
        assert_same_bits(ra.cpu().numpy()[0], S.asum(x, to_plan(s)), "asum chunks+fold")


def test_sweep_strategies_bit_exact_at_full_size():
    # the 24-strategy sweeps the autotuner chooses from: dot N = 2^26 and
    # gemv 16384 x 16384, every candidate bit-exact against the oracle
    import torch
    from paper_1710_08332_amd import autotune as T
    seed = synthetic.SEEDS["sweep"]
    n = 1 << 26
    x, y = synthetic.dot_inputs(n, seed)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    cands = T.sweep_dot(n)
    assert len(cands) == 24
    for s in cands:
        got = dp.dot(xt, yt, s).cpu().numpy()[0]
        assert_same_bits(got, S.dot(x, y, to_plan(s)), f"sweep dot {s}")
    del xt, yt
    m = k = 16384
    A, xv = synthetic.gemv_inputs(m, k, seed)
    At, xvt = torch.from_numpy(A).cuda(), torch.from_numpy(xv).cuda()
    gc = T.sweep_gemv(m, k)
    assert len(gc) == 24
    for s in gc:
        got = dp.gemv(At, xvt, s).cpu().numpy()
        assert_same_bits(got, S.gemv(A, xv, to_plan(s)), f"sweep gemv {s}")


RAGGED = [(256, 16, C_, TREE), (64, 256, T_, TREE), (5, 4, T_, SEQ), (8, 128, C_, SEQ),
          (33, 32, C_, TREE), (16, 1024, T_, TREE)]


@pytest.mark.parametrize("strat", RAGGED, ids=_ids)
@pytest.mark.parametrize("extra", [1, 3, 37, 4095])
def test_ragged_lengths_are_zero_extended(strat, extra):
    C, L, order, comb = strat
    W = C * L
    n = W * 3 + (extra % W if extra % W else 1)
    for passes in (1, 2):
        s = dp.Strategy(seq_len=C, local_size=L, order=order, wg_combine=comb, passes=passes)
        x, y = discriminating(19 + extra, n)
        assert_same_bits(gpu_dot(x, y, s), S.dot(x, y, to_plan(s)), f"ragged dot n={n}")
        assert_same_bits(gpu_asum(x, s), S.asum(x, to_plan(s)), f"ragged asum n={n}")


def test_short_vectors_smaller_than_one_chunk():
    s = dp.Strategy(seq_len=64, local_size=256, order=T_)
    for n in (1, 2, 5, 255, 257, 1000):
        x, y = discriminating(23, n)
        assert_same_bits(gpu_dot(x, y, s), S.dot(x, y, to_plan(s)), f"short n={n}")


@pytest.mark.parametrize("kw", [dict(seq_len=4, local_size=256, order=T_),
                                dict(seq_len=4, local_size=256, order=C_, wg_combine=SEQ),
                                dict(seq_len=2, local_size=256, order=T_, row_parts=2, rows_per_wg=4),
                                dict(seq_len=16, local_size=64, order=C_, row_parts=2)], ids=str)
@pytest.mark.parametrize("k", [1, 37, 1000, 1001, 1023])
def test_gemv_ragged_rows(kw, k):
    import torch
    s = dp.Strategy(**kw)
    if k > s.seq_len * s.local_size * s.row_parts:
        pytest.skip("row longer than the strategy")
    m = 4 * s.rows_per_wg * 3
    lda = -(-k // 4) * 4                         # rows 16-byte aligned
    A, x = synthetic.gemv_inputs(m, lda, 29)
    At = torch.from_numpy(A).cuda()[:, :k]
    xt = torch.from_numpy(np.ascontiguousarray(x[:k])).cuda()
    y = dp.gemv(At, xt, s)
    torch.cuda.synchronize()
    assert_same_bits(y.cpu().numpy(), S.gemv(np.ascontiguousarray(A[:, :k]), x[:k], to_plan(s)),
                     f"gemv k={k}")


def _batch_instances(seed, count_red, count_gemv, max_log_n=14, max_mk=300):
    """Seeded instances: dot or asum (coin) with log-uniform lengths, and
    gemvs with uniform m, k; plus the strategy list they index."""
    import torch
    g = np.random.default_rng(seed)
    strategies = [dp.Strategy(seq_len=16, local_size=256, order=T_),
                  dp.Strategy(seq_len=4, local_size=64, order=C_, wg_combine=SEQ),
                  dp.Strategy(seq_len=64, local_size=1024, order=T_),
                  dp.Strategy(seq_len=8, local_size=16, order=C_),
                  dp.Strategy(seq_len=20, local_size=16, order=T_, wg_combine=SEQ),
                  dp.Strategy(seq_len=4, local_size=64, order=T_, row_parts=2)]
    insts, host = [], []
    for _ in range(count_red):
        n = int(2 ** g.uniform(8, max_log_n))
        op = dp.OP_DOT if g.random() < 0.5 else dp.OP_ASUM
        si = int(g.integers(0, 5))
        x = (g.standard_normal(n) * 2.0 ** g.uniform(-10, 10, n)).astype(np.float32)
        y = synthetic.uniform_pm1(g, n)
        d = {"op": op, "strategy": si, "x": torch.from_numpy(x).cuda(),
             "out": torch.empty(1, device="cuda")}
        if op == dp.OP_DOT:
            d["y"] = torch.from_numpy(y).cuda()
        insts.append(d)
        host.append((op, si, x, y))
    for _ in range(count_gemv):
        m, k = int(g.integers(1, max_mk)), int(g.integers(1, max_mk))
        si = int(g.choice([0, 1, 3, 5]))
        s = strategies[si]
        if k > s.seq_len * s.local_size * s.row_parts:
            si = 0
        lda = -(-k // 4) * 4
        A = np.zeros((m, lda), np.float32)
        A[:, :k] = synthetic.normal(g, (m, k))
        x = synthetic.uniform_pm1(g, k)
        At = torch.from_numpy(A).cuda()[:, :k]
        insts.append({"op": dp.OP_GEMV, "strategy": si, "A": At, "x": torch.from_numpy(x).cuda(),
                      "out": torch.empty(m, device="cuda")})
        host.append((dp.OP_GEMV, si, np.ascontiguousarray(A[:, :k]), x))
    return insts, host, strategies


@pytest.mark.parametrize("one_launch", [False, True], ids=["two_launches", "one_launch"])
def test_batched_instances_equal_single_calls_and_the_oracle(one_launch):
    import torch
    insts, host, strategies = _batch_instances(31, 150, 40)
    plan = dp.BatchPlan(insts, strategies)
    ws = plan.workspace()
    plan.upload(ws)
    plan.run(ws, one_launch=one_launch)
    torch.cuda.synchronize()
    for d, (op, si, a, b) in zip(insts, host):
        s = strategies[si]
        got = d["out"].cpu().numpy()
        if op == dp.OP_GEMV:
            single = dp.gemv(d["A"], d["x"], s).cpu().numpy()
            want = S.gemv(a, b, to_plan(s))
        elif op == dp.OP_DOT:
            single = dp.dot(d["x"], d["y"], s).cpu().numpy()
            want = np.atleast_1d(S.dot(a, b, to_plan(s)))
        else:
            single = dp.asum(d["x"], s).cpu().numpy()
            want = np.atleast_1d(S.asum(a, to_plan(s)))
        assert_same_bits(got, single, f"batched vs single op={op} s={si}")
        assert_same_bits(got, want, f"batched vs oracle op={op} s={si}")


@pytest.mark.parametrize("one_launch", [False, True], ids=["two_launches", "one_launch"])
def test_batched_run_in_a_graph_replays_exactly(one_launch):
    import torch
    insts, host, strategies = _batch_instances(37, 60, 20)
    plan = dp.BatchPlan(insts, strategies)
    ws = plan.workspace()
    plan.upload(ws)
    plan.run(ws, one_launch=one_launch)
    torch.cuda.synchronize()
    eager = [d["out"].clone() for d in insts]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        for d in insts:
            d["out"].fill_(-1.0)
        with torch.cuda.graph(graph, stream=side):
            plan.run(ws, one_launch=one_launch)
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(3):
        for d in insts:
            d["out"].fill_(float(rep) + 7.0)          # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for d, e in zip(insts, eager):
            assert_same_bits(d["out"].cpu().numpy(), e.cpu().numpy(), f"replay {rep}")



def test_single_calls_in_a_graph_replay_exactly():
    # dot (2-pass, 1-pass with its arrival counter, Kahan to binary64), asum
    # and gemv captured in one graph: every replay reproduces the eager bits
    import torch
    n = (1 << 20) + 77
    x, y = synthetic.dot_inputs(n, synthetic.SEEDS["small"])
    A, xv = synthetic.gemv_inputs(96, 3000, synthetic.SEEDS["scale"])
    xt, yt, At, xvt = cuda(x), cuda(y), cuda(A), cuda(xv)
    calls = []
    for s, kind in ((dp.Strategy(seq_len=256, local_size=16, order=C_, passes=2), "dot"),
                    (dp.Strategy(seq_len=64, local_size=256, order=T_, passes=1), "dot"),
                    (dp.Strategy(seq_len=32, local_size=128, order=T_, passes=1, accum=dp.KAHAN,
                                 final_f64=1), "dot"),
                    (dp.Strategy(seq_len=128, local_size=64, order=T_, passes=2), "asum"),
                    (dp.Strategy(seq_len=64, local_size=64, order=T_, rows_per_wg=2), "gemv")):
        if kind == "gemv":
            out = torch.empty(96, dtype=torch.float32, device="cuda")
            calls.append((lambda s=s, out=out: dp.gemv(At, xvt, s, y=out), out))
            continue
        op = dp.OP_DOT if kind == "dot" else dp.OP_ASUM
        # compensated strategies take whole chunks only: a 2^20 prefix
        xs, ys = (xt[:1 << 20], yt[:1 << 20]) if s.accum != dp.PLAIN else (xt, yt)
        ws = dp.workspace(s, op, dp.F32, 0, xs.numel())
        od = torch.float64 if s.final_f64 else torch.float32
        out = torch.empty(1, dtype=od, device="cuda")
        if kind == "dot":
            calls.append((lambda s=s, out=out, ws=ws, xs=xs, ys=ys:
                          dp.dot(xs, ys, s, out=out, ws=ws), out))
        else:
            calls.append((lambda s=s, out=out, ws=ws: dp.asum(xt, s, out=out, ws=ws), out))
    for fn, _ in calls:
        fn()
    torch.cuda.synchronize()
    eager = [o.clone() for _, o in calls]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            for fn, _ in calls:
                fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(3):
        for _, o in calls:
            o.fill_(float(rep) - 5.0)                 # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for i, ((_, o), e) in enumerate(zip(calls, eager)):
            assert torch.equal(o.cpu().view(torch.uint8), e.cpu().view(torch.uint8)), \
                f"replay {rep} call {i}"


def test_dots_and_gemvs_on_two_graph_branches_replay_exactly():
    # the headline step's strategies with the dots on one graph branch and the
    # gemvs (three copies of A in turn) on another, joined at the end: every
    # replay reproduces the eager bits, which equal the oracle's
    import torch
    dot_s = dp.Strategy(seq_len=256, local_size=1024, order=T_, wg_combine=TREE, passes=1)
    gemv_s = dp.Strategy(seq_len=32, local_size=256, order=T_, wg_combine=TREE, rows_per_wg=4)
    n, m, k, steps = (1 << 22) + 77, 256, 8192, 6
    x, y = synthetic.dot_inputs(n, synthetic.SEEDS["small"])
    A, xv = synthetic.gemv_inputs(m, k, synthetic.SEEDS["scale"])
    xt, yt, xvt = cuda(x), cuda(y), cuda(xv)
    Ats = [cuda(A) for _ in range(3)]
    out = torch.empty(1, dtype=torch.float32, device="cuda")
    yg = torch.empty(m, dtype=torch.float32, device="cuda")
    ws = dp.workspace(dot_s, dp.OP_DOT, dp.F32, 0, n)
    dp.dot(xt, yt, dot_s, out=out, ws=ws)
    dp.gemv(Ats[0], xvt, gemv_s, y=yg)
    torch.cuda.synchronize()
    assert_same_bits(out.cpu().numpy()[0], S.dot(x, y, to_plan(dot_s)), "eager dot")
    assert_same_bits(yg.cpu().numpy(), S.gemv(A, xv, to_plan(gemv_s)), "eager gemv")
    eager = (out.clone(), yg.clone())
    main, branch = torch.cuda.Stream(), torch.cuda.Stream()
    main.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(main):
        with torch.cuda.graph(graph, stream=main):
            branch.wait_stream(main)
            for _ in range(steps):
                dp.dot(xt, yt, dot_s, out=out, ws=ws)
            with torch.cuda.stream(branch):
                for j in range(steps):
                    dp.gemv(Ats[j % 3], xvt, gemv_s, y=yg)
            main.wait_stream(branch)
    torch.cuda.current_stream().wait_stream(main)
    torch.cuda.synchronize()
    for rep in range(4):
        out.fill_(float(rep) - 5.0)                    # eager work between replays
        yg.fill_(float(rep) + 3.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), eager[0].view(torch.int32)), f"dot, replay {rep}"
        assert torch.equal(yg.view(torch.int32), eager[1].view(torch.int32)), f"gemv, replay {rep}"
    # the 1-pass arrival counter is left at zero by every call
    assert not ws[-256:].any(), "arrival-counter block left non-zero"


@pytest.mark.parametrize("kw", [dict(seq_len=16, local_size=256, order=T_),
                                dict(seq_len=64, local_size=64, order=C_),     # staged, tile 64
                                dict(seq_len=96, local_size=128, order=C_),    # staged, tile 32
                                dict(seq_len=16, local_size=64, order=C_),     # staged, tile 16
                                dict(seq_len=48, local_size=48, order=C_),     # 240 threads: direct
                                dict(seq_len=3, local_size=5, order=T_),
                                dict(seq_len=1, local_size=1, order=C_)], ids=str)
@pytest.mark.parametrize("n", [1, 1000, 4097, (1 << 20) + 3])
def test_scal_bit_exact_and_in_place(kw, n):
    import torch
    s = dp.Strategy(**kw)
    g = np.random.default_rng(41)
    x = (g.standard_normal(n) * 2.0 ** g.uniform(-30, 30, n)).astype(np.float32)
    a = np.float32(-1.3)
    xt = torch.from_numpy(x).cuda()
    y = dp.scal(float(a), xt, s)
    torch.cuda.synchronize()
    want = S.scal(a, x)
    assert_same_bits(y.cpu().numpy(), want, "scal")
    dp.scal(float(a), xt, s, y=xt)          # in place
    torch.cuda.synchronize()
    assert_same_bits(xt.cpu().numpy(), want, "scal in place")


@pytest.mark.parametrize("kw", [GEMV_STRATS[0], GEMV_STRATS[2], GEMV_STRATS[5]],
                         ids=lambda k: "-".join(f"{a[:3]}{b}" for a, b in k.items()))
@pytest.mark.parametrize("fmt", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (-0.75, 0.0), (1.3, -2.1), (0.5, 1.0)])
def test_gemv_blas_bit_exact(kw, fmt, alpha, beta):
    import torch
    s = dp.Strategy(**kw)
    plan = to_plan(s)
    k = s.seq_len * s.local_size * s.row_parts - 3            # ragged rows too
    m = s.rows_per_wg * 11
    A, x = synthetic.gemv_inputs(m, k, synthetic.SEEDS["scale"])
    y0 = np.random.default_rng(12).standard_normal(m).astype(np.float32)
    scale = None
    if fmt == "f32":
        src, adt = A, dp.F32
    elif fmt == "bf16":
        src, adt = synthetic.quantise_bf16(A), dp.BF16
    else:
        (src, scale), adt = synthetic.quantise_fp8_rows(A), dp.FP8_E4M3
    lda = -(-k // 16) * 16
    Ap = np.zeros((m, lda), src.dtype)
    Ap[:, :k] = src
    At = torch.from_numpy(Ap.view(np.int16) if Ap.dtype == np.uint16 else Ap).cuda()[:, :k]
    # beta == 0: the old y is never read, so NaN there must not show
    yt = torch.from_numpy(y0 if beta != 0 else np.full(m, np.nan, np.float32)).cuda()
    st = torch.from_numpy(scale).cuda() if scale is not None else None
    dp.gemv_blas(alpha, At, torch.from_numpy(x).cuda(), beta, yt, s, row_scale=st, a_dtype=adt)
    torch.cuda.synchronize()
    want = S.gemv_blas(alpha, src, x, beta, y0, plan, a_format=fmt, scale=scale)
    assert_same_bits(yt.cpu().numpy(), want, f"gemv_blas {fmt}")


VEC_STRATS = [
    dict(seq_len=16, local_size=64, order=C_, wg_combine=dp.NONE, vec_width=4),  # Sec. 6.2 form
    dict(seq_len=8, local_size=256, order=T_, wg_combine=TREE, vec_width=4),
    dict(seq_len=5, local_size=128, order=C_, wg_combine=TREE, vec_width=4),
    dict(seq_len=7, local_size=12, order=T_, wg_combine=SEQ, vec_width=2),
    dict(seq_len=9, local_size=1024, order=T_, wg_combine=TREE, vec_width=2),
    dict(seq_len=6, local_size=32, order=C_, wg_combine=SEQ, vec_width=4),
    dict(seq_len=4, local_size=64, order=T_, wg_combine=dp.NONE, vec_width=4),
    dict(seq_len=3, local_size=16, order=C_, wg_combine=dp.NONE),
    dict(seq_len=4, local_size=64, order=T_, wg_combine=dp.NONE),
    dict(seq_len=33, local_size=1, order=C_, wg_combine=dp.NONE, vec_width=4),
]


@pytest.mark.parametrize("kw", VEC_STRATS, ids=lambda k: "-".join(f"{a[:3]}{b}" for a, b in k.items()))
@pytest.mark.parametrize("passes", [1, 2])
@pytest.mark.parametrize("ragged", [0, 1])
def test_vector_and_uncombined_strategies_bit_exact(kw, passes, ragged):
    import torch
    s = dp.Strategy(passes=passes, **kw)
    p = to_plan(s)
    n = p.chunk * 17 - ragged * (p.chunk // 3 + 5)
    x, y = discriminating(23 + ragged, n)
    assert_same_bits(gpu_dot(x, y, s), S.dot(x, y, p), "dot")
    assert_same_bits(gpu_asum(x, s), S.asum(x, p), "asum")
    g = np.random.default_rng(5)
    xi, yi = synthetic.integers_u32(g, n), synthetic.integers_u32(g, n)
    assert_same_bits(gpu_dot(xi, yi, s), S.dot(xi, yi, p, num="u32"), "i32 dot")
    # the chunk values element by element, then the fold
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    c = dp.chunks(dp.OP_DOT, s, xt, yt)
    torch.cuda.synchronize()
    want = np.asarray(S.dot_chunks(x, y, p), np.float32)
    assert_same_bits(c.cpu().numpy()[:4 * len(want)].view(np.float32), want, "chunk values")


def test_paper_vector_dot_at_full_size():
    # the dot expression of Sec. 6.2: float4 views, 64 work-items per work-group
    # each folding 2048 vectors, every work-item's value written out; then the
    # ordered fold.  N = 2^26.
    import torch
    s = dp.Strategy(seq_len=2048, local_size=64, order=C_, wg_combine=dp.NONE, vec_width=4)
    p = to_plan(s)
    n = 1 << 26
    x, y = synthetic.dot_inputs(n, synthetic.SEEDS["scale"])
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    c = dp.chunks(dp.OP_DOT, s, xt, yt)
    r = dp.dot(xt, yt, s)
    torch.cuda.synchronize()
    want = np.asarray(S.dot_chunks(x, y, p), np.float32)
    assert len(want) == 128 * 64 * 4
    assert_same_bits(c.cpu().numpy().view(np.float32), want, "Sec. 6.2 chunk values")
    assert_same_bits(r.cpu().numpy()[0], S.dot(x, y, p), "Sec. 6.2 dot")


# ------------------------------------------------------------ generated kernels

def _generated(name):
    from paper_1710_08332_amd.generator import catalog, runtime
    return runtime.Generated(catalog.path(name))


def _meta(name):
    import json
    from paper_1710_08332_amd.generator import catalog
    with open(catalog.path(name)) as f:
        return json.load(f)


@pytest.mark.parametrize("name,strategy", [
    ("dot_strided_tree", dict(seq_len=4, local_size=64, order=T_)),
    ("dot_contiguous_seq", dict(seq_len=16, local_size=32, order=C_, wg_combine=SEQ)),
    ("dot_kahan_f64", dict(seq_len=16, local_size=64, order=T_, accum=dp.KAHAN, final_f64=1)),
    ("dot_sum2", dict(seq_len=16, local_size=64, order=T_, accum=dp.SUM2)),
    ("dot_u32", dict(seq_len=4, local_size=16, order=C_)),
    ("dot_v4_strided_tree", dict(seq_len=8, local_size=64, order=T_, vec_width=4)),
    ("asum_strided_tree", dict(seq_len=8, local_size=128, order=T_)),
])
def test_generated_reductions_equal_oracle_and_library(name, strategy):
    # a descriptor printed as its expression, compiled by the generator: the
    # same bits as the oracle's expression for the descriptor and as the
    # library's hand-written kernels for it
    import torch
    meta = _meta(name)
    n = meta["inputs"]["xs"][1][0]
    s = dp.Strategy(**strategy)
    if meta["num"] == "u32":
        g = np.random.default_rng(8)
        x, y = synthetic.integers_u32(g, n), synthetic.integers_u32(g, n)
        feed = {"xs": cuda(x.view(np.int32)), "ys": cuda(y.view(np.int32))}
    else:
        x, y = discriminating(29, n)
        feed = {"xs": cuda(x), "ys": cuda(y)}
    prog = _generated(name)
    out = prog.run(feed)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    # expected: the oracle's own expression for the descriptor (its builder,
    # not the library's printed text)
    if name.startswith("asum"):
        want = S.asum(x, to_plan(s))
    else:
        want = S.dot(x, y, to_plan(s), num=meta["num"])
    res = got["out"][0]
    if meta["num"] == "u32":
        res = res.view(np.uint32)
    assert_same_bits(res, want, f"{name} vs oracle")
    if name.startswith("asum"):
        lib = gpu_asum(x, s)
    else:
        lib = gpu_dot(x, y, s, out_dtype=torch.float64 if s.final_f64 else None)
    assert_same_bits(res, lib, f"{name} vs library kernel")
    prog.close()


def test_generated_sec62_dot_equals_library_chunks():
    import torch
    meta = _meta("dot_sec62_chunks")
    n = meta["inputs"]["xs"][1][0]
    x, y = synthetic.dot_inputs(n, synthetic.SEEDS["scale"])
    prog = _generated("dot_sec62_chunks")
    out = prog.run({"xs": cuda(x), "ys": cuda(y)})
    s = dp.Strategy(seq_len=2048, local_size=64, order=C_, wg_combine=dp.NONE, vec_width=4)
    c = dp.chunks(dp.OP_DOT, s, cuda(x), cuda(y))
    torch.cuda.synchronize()
    got = out["out"].cpu().numpy()
    assert_same_bits(got, c.cpu().numpy().view(np.float32), "Sec. 6.2 generated vs library")
    # the oracle's builder for the same strategy (C=2048, L=64, V=4, no
    # work-group combine): its chunk values, lane by lane
    assert_same_bits(got, S.dot_chunks(x, y, to_plan(s)), "Sec. 6.2 generated vs oracle")
    prog.close()


def test_generated_gemv_and_scal():
    import torch
    A, x = synthetic.gemv_inputs(96, 1024, synthetic.SEEDS["scale"])
    prog = _generated("gemv_strided_tree")
    y = prog.run({"A": cuda(A), "x": cuda(x)})["out"]
    s = dp.Strategy(seq_len=16, local_size=64, order=T_, rows_per_wg=2)
    torch.cuda.synchronize()
    assert_same_bits(y.cpu().numpy(), gpu_gemv(A, x, s), "generated gemv vs library")
    assert_same_bits(y.cpu().numpy(), S.gemv(A, x, to_plan(s)), "generated gemv vs oracle")
    prog.close()
    xs = discriminating(4, 1 << 20)[0]
    prog = _generated("scal_global")
    r = prog.run({"alpha": cuda(np.array([1.3], np.float32)), "xs": cuda(xs)})["out"]
    torch.cuda.synchronize()
    assert_same_bits(r.cpu().numpy(), S.scal(np.float32(1.3), xs), "generated scal")
    prog.close()


def test_generated_headline_dot_and_gemv_at_full_size():
    import torch
    from paper_1710_08332_amd.generator import catalog
    x, y = synthetic.dot_inputs(1 << 26, synthetic.SEEDS["scale"])
    prog = _generated("dot_headline_2p26")
    r = prog.run({"xs": cuda(x), "ys": cuda(y)})["out"]
    torch.cuda.synchronize()
    assert_same_bits(r.cpu().numpy()[0], gpu_dot(x, y, catalog.HEADLINE_DOT), "generated dot")
    assert_same_bits(r.cpu().numpy()[0], S.dot(x, y, to_plan(catalog.HEADLINE_DOT)),
                     "generated dot vs oracle")
    prog.close()
    A, xv = synthetic.gemv_inputs(8192, 8192, synthetic.SEEDS["scale"])
    prog = _generated("gemv_headline_8192")
    g = prog.run({"A": cuda(A), "x": cuda(xv)})["out"]
    torch.cuda.synchronize()
    assert_same_bits(g.cpu().numpy(), gpu_gemv(A, xv, catalog.HEADLINE_GEMV), "generated gemv")
    assert_same_bits(g.cpu().numpy(), S.gemv(A, xv, to_plan(catalog.HEADLINE_GEMV)),
                     "generated gemv vs oracle")
    prog.close()


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_generated_decoders_cover_every_code(fmt):
    # the generator's decoders, written from the format definitions, against
    # the oracle's decode of every storage code (NaN codes: NaN on both sides)
    import torch
    n = 1 << (16 if fmt == "bf16" else 8)
    codes = np.arange(n, dtype=np.uint16 if fmt == "bf16" else np.uint8)
    prog = _generated(f"decode_{fmt}_all")
    dev = cuda(codes.view(np.int16) if fmt == "bf16" else codes)
    got = prog.run({"codes": dev})["out"]
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    want = (formats.bf16_decode if fmt == "bf16" else formats.fp8_decode)(codes)
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    assert_same_bits(got[~nan], want[~nan], f"{fmt} decode")
    prog.close()


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_generated_low_precision_gemv_equals_oracle_and_library(fmt):
    import torch
    s = dp.Strategy(seq_len=4, local_size=64, order=T_, rows_per_wg=2)
    A, x = synthetic.gemv_inputs(64, 256, synthetic.SEEDS["scale"])
    if fmt == "bf16":
        codes, scale, adt = synthetic.quantise_bf16(A), None, dp.BF16
        feed = {"A": cuda(codes.view(np.int16)), "x": cuda(x)}
    else:
        (codes, scale), adt = synthetic.quantise_fp8_rows(A), dp.FP8_E4M3
        feed = {"A": cuda(codes), "x": cuda(x), "scale": cuda(scale)}
    prog = _generated(f"gemv_{fmt}_strided_tree")
    y = prog.run(feed)["out"]
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    assert_same_bits(got, S.gemv(codes, x, to_plan(s), a_format=fmt, scale=scale),
                     f"generated {fmt} gemv vs oracle")
    assert_same_bits(got, gpu_gemv(codes, x, s, a_dtype=adt, scale=scale),
                     f"generated {fmt} gemv vs library")
    prog.close()


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_generated_low_precision_gemv_at_full_size_with_paired_rows(fmt):
    # 16384 x 16384, two rows per work-group run together by the generated
    # kernel: bit-exact against the library, and against the oracle on a
    # sample of rows (rows are independent)
    import torch
    s = dp.Strategy(seq_len=16, local_size=1024, order=T_, rows_per_wg=2)
    A, x = synthetic.gemv_inputs(16384, 16384, synthetic.SEEDS["precision"])
    if fmt == "bf16":
        codes, scale, adt = synthetic.quantise_bf16(A), None, dp.BF16
        feed = {"A": cuda(codes.view(np.int16)), "x": cuda(x)}
    else:
        (codes, scale), adt = synthetic.quantise_fp8_rows(A), dp.FP8_E4M3
        feed = {"A": cuda(codes), "x": cuda(x), "scale": cuda(scale)}
    del A
    prog = _generated(f"gemv_{fmt}_16384")
    got = prog.run(feed)["out"].cpu().numpy()
    torch.cuda.synchronize()
    prog.close()
    assert_same_bits(got, gpu_gemv(codes, x, s, a_dtype=adt, scale=scale),
                     f"generated {fmt} 16384^2 vs library")
    rows = np.random.default_rng(5).choice(16384, 48, replace=False)
    want = S.gemv(codes[rows], x, to_plan(s.with_(rows_per_wg=1)), a_format=fmt,
                  scale=None if scale is None else scale[rows])
    assert_same_bits(got[rows], want, f"generated {fmt} 16384^2 vs oracle, sampled rows")


@pytest.mark.parametrize("kw", [dict(seq_len=4, local_size=256, order=T_),
                                dict(seq_len=2, local_size=512, order=T_, wg_combine=SEQ)],
                         ids=["C4-L256-tree", "C2-L512-seq"])
def test_fp8_gemv_with_four_rows_per_team(kw):
    # enough rows that fp8 teams take 4 rows at a time (one or two
    # work-groups per compute unit), with a ragged last work-group
    s = dp.Strategy(**kw)
    teams_per_wg = 256 // (kw["local_size"] // 16)     # 16 fp8 lanes per work-item
    m, k = 300 * teams_per_wg * 4 + 5, kw["seq_len"] * kw["local_size"]   # 301 work-groups
    A, x = synthetic.gemv_inputs(m, k, synthetic.SEEDS["precision"])
    codes, scale = synthetic.quantise_fp8_rows(A)
    got = gpu_gemv(codes, x, s, a_dtype=dp.FP8_E4M3, scale=scale)
    assert_same_bits(got, S.gemv(codes, x, to_plan(s), a_format="fp8", scale=scale),
                     f"fp8 gemv m={m} {kw}")


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
@pytest.mark.parametrize("kw", [dict(seq_len=32, local_size=64, order=C_),
                                dict(seq_len=64, local_size=32, order=C_, wg_combine=SEQ),
                                dict(seq_len=32, local_size=32, order=C_, row_parts=2)], ids=str)
@pytest.mark.parametrize("k", [2048, 2047, 1001, 37])
def test_contiguous_low_precision_gemv_staged_and_ragged(fmt, kw, k):
    # contiguous bf16 / fp8 rows staged through LDS (C a multiple of 32),
    # rows ending inside a 16-byte unit of codes; lda keeps rows aligned
    import torch
    s = dp.Strategy(**kw)
    if k > s.seq_len * s.local_size * s.row_parts:
        pytest.skip("row longer than the strategy")
    m = 4 * 3 + 1
    lda = -(-k // 16) * 16
    A, x = synthetic.gemv_inputs(m, lda, 31)
    if fmt == "bf16":
        codes, scale, adt = synthetic.quantise_bf16(A), None, dp.BF16
        At = torch.from_numpy(np.ascontiguousarray(codes.view(np.int16))).cuda()[:, :k]
    else:
        (codes, scale), adt = synthetic.quantise_fp8_rows(A), dp.FP8_E4M3
        At = torch.from_numpy(np.ascontiguousarray(codes)).cuda()[:, :k]
    xt = torch.from_numpy(np.ascontiguousarray(x[:k])).cuda()
    st = torch.from_numpy(scale).cuda() if scale is not None else None
    y = dp.gemv(At, xt, s, row_scale=st, a_dtype=adt)
    torch.cuda.synchronize()
    want = S.gemv(np.ascontiguousarray(codes[:, :k]), x[:k], to_plan(s), a_format=fmt,
                  scale=scale)
    assert_same_bits(y.cpu().numpy(), want, f"{fmt} contiguous gemv k={k} {kw}")


def test_generated_global_temporaries_hoisted_out_of_work_groups():
    # toGlobal inside mapWorkgroup: one copy of the lane values per
    # work-group (Sec. 6.3), written by the lanes, folded by the work-group;
    # 300 work-groups at once would corrupt a shared copy
    import torch
    meta = _meta("dot_global_lanes")
    n = meta["inputs"]["xs"][1][0]
    ws = [b for b in meta["buffers"] if b["kind"] == "ws"]
    assert any(b["elems"] == 300 * 64 for b in ws)
    x, y = discriminating(31, n)
    prog = _generated("dot_global_lanes")
    out = prog.run({"xs": cuda(x), "ys": cuda(y)})
    torch.cuda.synchronize()
    want = S.dot(x, y, S.Plan(seq=4, lanes=64, order="contiguous", combine="seq"))
    assert_same_bits(out["out"].cpu().numpy()[0], want, "hoisted global lanes vs oracle")
    prog.close()
