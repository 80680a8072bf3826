"""GPU parity of kernel paths that only wide teams, large matrices or many
instances reach: compensated accumulators merged across wavefronts through
LDS (teams of 128 and 256 threads), the fp8 gemv that reduces 4 rows per team
with 64-element batches, a batch of instances drawn like the benchmark's
(lengths up to 2^20, gemv sides up to 4096), and staged contiguous folds
with an odd number of tiles, the outer fold of many chunk values at the
boundaries of the steps it copies them in, and staged contiguous lanes fed
by loader wavefronts (also in one pass, with many chunk values, and
tree-combined teams split over work-groups), and strided lanes fed the same
way; binary32 gemv rows of one thread each in the strided order, staged
through LDS.

Every comparison is bit for bit against the oracle on the same inputs.  Where
the full problem is too large for the oracle, it is evaluated on sampled
rows: gemv rows are the iterations of a map, so a subset of rows has the
same values alone as inside the whole matrix."""

import numpy as np
import pytest

import paper_1710_08332_amd as dp
import synthetic
from oracle import exact
from oracle import strategies as S
from tests.gpu_util import assert_same_bits, cuda, discriminating, gpu_asum, gpu_dot, to_plan

pytestmark = pytest.mark.gpu

C_, T_ = dp.CONTIGUOUS, dp.STRIDED


# ------------------------------------------------ compensated, wide teams
# (C, L, order, combine): strided L=1024 is a team of 256 threads (4
# wavefronts, the long-vector precision strategy), L=512 one of 128; the
# contiguous L=256 team is 4 wavefronts staged through LDS; the sequential
# combine over 1024 lanes reads every lane pair from LDS.
WIDE_COMP = [(256, 1024, T_, dp.TREE), (256, 512, T_, dp.TREE), (64, 256, C_, dp.TREE),
             (16, 1024, T_, dp.SEQ)]


@pytest.mark.parametrize("strat", WIDE_COMP, ids=lambda s: f"C{s[0]}-L{s[1]}-{s[2]}-{s[3]}")
@pytest.mark.parametrize("final_f64", [0, 1])
@pytest.mark.parametrize("accum", [dp.KAHAN, dp.SUM2], ids=["kahan", "sum2"])
def test_compensated_dots_with_teams_wider_than_a_wavefront(strat, final_f64, accum):
    import torch
    C, L, order, comb = strat
    s = dp.Strategy(seq_len=C, local_size=L, order=order, wg_combine=comb, accum=accum,
                    final_f64=final_f64)
    n = 3 * C * L
    print(f"compensated accum={accum} f64={final_f64} C={C} L={L} n={n}", flush=True)
    x, y = synthetic.kahan_dot_inputs(n, synthetic.SEEDS["precision"])
    want = S.dot(x, y, to_plan(s))
    for passes in (1, 2):
        assert_same_bits(gpu_dot(x, y, s.with_(passes=passes)), want, f"passes={passes}")
    if final_f64:
        assert_same_bits(gpu_dot(x, y, s, out_dtype=torch.float32), np.float32(want),
                         "binary64 fold rounded to binary32")
    # cancelling products: the result is rounding error alone
    xd, yd = discriminating(61, n)
    assert_same_bits(gpu_dot(xd, yd, s), S.dot(xd, yd, to_plan(s)), "cancelling")
    err = abs(float(want) - exact.dot_exact(x, y)) / exact.dot_abs_terms(x, y)
    assert err < 1e-6


# ------------------------------------------------ fp8 gemv, rows per team
def _fp8_rows_per_team(s, m, cus=256):
    """The rows one team reduces at once for an fp8 matrix (the library's
    rule, restated): 4 when that gives 1..2 work-groups per compute unit."""
    team = s.local_size // 16
    lg = max(1, 256 // (team * s.rows_per_wg))
    per_wg4 = lg * s.rows_per_wg * 4
    wgs4 = -(-m // per_wg4)
    return 4 if cus <= wgs4 <= 2 * cus else 2


@pytest.mark.parametrize("C,L", [(64, 256), (128, 128), (32, 512)])
def test_fp8_gemv_rows_per_team_at_full_size(C, L):
    # 16384 x 16384 fp8 rows with per-row scales; C >= 64 takes the
    # 64-element batches, and (C=64, L=256) and (C=32, L=512) reduce 4 rows
    # per team on a 256-CU device, (C=128, L=128) 2.
    import torch
    m = k = 16384
    s = dp.Strategy(seq_len=C, local_size=L, order=T_, wg_combine=dp.TREE)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    print(f"fp8 gemv C={C} L={L} rows per team {_fp8_rows_per_team(s, m, cus)}", flush=True)
    g = synthetic.rng(synthetic.SEEDS["precision"] + C)
    A = synthetic.normal(g, (m, k))
    x = synthetic.uniform_pm1(g, k)
    codes, scale = synthetic.quantise_fp8_rows(A)
    del A
    y = dp.gemv(cuda(codes), cuda(x), s, row_scale=cuda(scale), a_dtype=dp.FP8_E4M3)
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    # every row of the first and last team blocks, and a seeded sample
    rows = np.unique(np.concatenate([np.arange(0, 128), np.arange(m - 128, m),
                                     np.sort(g.choice(m, 256, replace=False))]))
    want = S.gemv(codes[rows], x, to_plan(s), a_format="fp8", scale=scale[rows])
    assert_same_bits(got[rows], want, f"fp8 C={C} L={L}")


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_row_blocked_gemv_with_a_ragged_last_block(fmt):
    # m not a multiple of the rows a work-group takes at once: the last
    # block's missing rows are skipped, the others exact
    s = dp.Strategy(seq_len=64, local_size=256, order=T_, wg_combine=dp.TREE)
    m, k = 16384 + 40, 16384 - 100
    g = synthetic.rng(77)
    A = synthetic.normal(g, (m, k))
    x = synthetic.uniform_pm1(g, k)
    import torch
    lda = k + (-k) % 16
    if fmt == "bf16":
        codes, scale, adt = synthetic.quantise_bf16(A), None, dp.BF16
    else:
        (codes, scale), adt = synthetic.quantise_fp8_rows(A), dp.FP8_E4M3
    del A
    pad = np.zeros((m, lda), codes.dtype)
    pad[:, :k] = codes
    At = cuda(pad.view(np.int16) if pad.dtype == np.uint16 else pad)[:, :k]
    y = dp.gemv(At, cuda(x), s, row_scale=cuda(scale) if scale is not None else None,
                a_dtype=adt)
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    rows = np.unique(np.concatenate([np.arange(m - 200, m), g.choice(m, 128, replace=False)]))
    want = S.gemv(np.ascontiguousarray(codes[rows]), x, to_plan(s), a_format=fmt,
                  scale=scale[rows] if scale is not None else None)
    assert_same_bits(got[rows], want, f"{fmt} ragged block")


# ------------------------------------------------ staged folds, odd tiles
# Contiguous binary32 folds staged through LDS in 32-element tiles: C*V/32
# tiles per lane row.  With few chunks (fewer wavefronts than compute units)
# the dot keeps two tiles in flight; odd tile counts (1, 3, 5) end on the
# first register set, and a single tile has no second one at all.
ODD_TILES = [dict(seq_len=32, local_size=64, order=C_),
             dict(seq_len=96, local_size=64, order=C_),
             dict(seq_len=160, local_size=128, order=C_, wg_combine=dp.SEQ),
             dict(seq_len=8, local_size=64, order=C_, vec_width=4),
             dict(seq_len=24, local_size=64, order=C_, vec_width=4, wg_combine=dp.NONE),
             dict(seq_len=40, local_size=256, order=C_)]


@pytest.mark.parametrize("kw", ODD_TILES, ids=str)
@pytest.mark.parametrize("chunks", [1, 7, 100])
def test_staged_contiguous_folds_with_odd_tile_counts(kw, chunks):
    import torch
    s = dp.Strategy(**kw)
    W = s.seq_len * s.local_size * max(1, s.vec_width)
    n = W * chunks - (W // 3 if chunks > 1 else 0)          # a ragged last chunk too
    print(f"odd tiles {kw} chunks={chunks} n={n}", flush=True)
    x, y = discriminating(83 + chunks, n)
    plan = to_plan(s)
    assert_same_bits(gpu_dot(x, y, s), S.dot(x, y, plan), "dot")
    assert_same_bits(gpu_asum(x, s), S.asum(x, plan), "asum")
    xt, yt = cuda(x), cuda(y)
    c = dp.chunks(dp.OP_DOT, s, xt, yt)
    torch.cuda.synchronize()
    vals = c.cpu().numpy().view(np.float32)[:dp.num_chunks(s, n) * dp.values_per_chunk(s)]
    assert_same_bits(vals, S.dot_chunks(x, y, plan), "chunk values")


# ------------------------------------------------ batches at benchmark sizes
def _bench_like_instances(seed, n_red, n_gemv):
    """Instances drawn as the benchmark draws them (op by a seeded coin,
    n = floor(2^U(8, 20)); gemv m, k uniform in 64..4096), each with a
    batch-eligible strategy of its size class picked by a seeded draw."""
    import torch
    from paper_1710_08332_amd import autotune as T
    g = synthetic.rng(seed)
    strategies, insts, host = [], [], []

    def pick(cls):
        cands = T.batch_candidates(cls)
        s = cands[int(g.integers(0, len(cands)))]
        if s not in strategies:
            strategies.append(s)
        return strategies.index(s)

    for _ in range(n_red):
        op = dp.OP_DOT if g.random() < 0.5 else dp.OP_ASUM
        n = int(2 ** g.uniform(8, 20))
        x = synthetic.uniform_pm1(g, n)
        y = synthetic.uniform_pm1(g, n)
        d = {"op": op, "x": torch.from_numpy(x).cuda(), "out": torch.empty(1, device="cuda")}
        if op == dp.OP_DOT:
            d["y"] = torch.from_numpy(y).cuda()
        d["strategy"] = pick(T.size_class(d))
        insts.append(d)
        host.append((op, x, y))
    for _ in range(n_gemv):
        m, k = int(g.integers(64, 4097)), int(g.integers(64, 4097))
        lda = -(-k // 4) * 4
        A = np.zeros((m, lda), np.float32)
        A[:, :k] = synthetic.uniform_pm1(g, (m, k))
        x = synthetic.uniform_pm1(g, k)
        d = {"op": dp.OP_GEMV, "A": torch.from_numpy(A).cuda()[:, :k],
             "x": torch.from_numpy(x).cuda(), "out": torch.empty(m, device="cuda")}
        d["strategy"] = pick(T.size_class(d))
        insts.append(d)
        host.append((dp.OP_GEMV, np.ascontiguousarray(A[:, :k]), x))
    return insts, host, strategies


@pytest.mark.parametrize("one_launch", [False, True], ids=["two_launches", "one_launch"])
def test_batch_at_benchmark_sizes_equals_the_oracle(one_launch):
    import torch
    insts, host, strategies = _bench_like_instances(synthetic.SEEDS["batch"] + 1, 120, 8)
    print(f"batch {len(insts)} instances, {len(strategies)} strategies, "
          f"one_launch={one_launch}", flush=True)
    plan = dp.BatchPlan(insts, strategies)
    ws = plan.workspace()
    plan.upload(ws)
    plan.run(ws, one_launch=one_launch)
    torch.cuda.synchronize()
    for i, (d, (op, a, b)) in enumerate(zip(insts, host)):
        p = to_plan(strategies[d["strategy"]])
        got = d["out"].cpu().numpy()
        if op == dp.OP_GEMV:
            want = S.gemv(a, b, p)
        elif op == dp.OP_DOT:
            want = np.atleast_1d(S.dot(a, b, p))
        else:
            want = np.atleast_1d(S.asum(a, p))
        assert_same_bits(got, want, f"instance {i} op={op}")
    plan.close()


def test_batch_runs_back_to_back_clear_their_counters():
    # Reductions of many tiles each (W = 256, 16 chunks per tile: up to 64
    # arrivals per instance) mixed with one-tile ones and gemvs, run six
    # times in a row on one stream, on two workspaces, by both engines in
    # turn: every one-launch run starts from the counters the previous run
    # left at zero, and every run gives the single calls' bits.
    import torch
    g = synthetic.rng(91)
    strategies = [dp.Strategy(seq_len=4, local_size=64, order=T_),
                  dp.Strategy(seq_len=16, local_size=256, order=C_, wg_combine=dp.SEQ),
                  dp.Strategy(seq_len=8, local_size=64, order=T_)]
    insts = []
    for i in range(48):
        op = (dp.OP_DOT, dp.OP_ASUM, dp.OP_GEMV)[i % 3]
        si = i % 2 if op != dp.OP_GEMV else 2
        if op == dp.OP_GEMV:
            m, k = int(g.integers(1, 700)), int(g.integers(1, 513))
            lda = -(-k // 4) * 4
            A = torch.zeros((m, lda), device="cuda")
            A[:, :k] = torch.from_numpy(synthetic.normal(g, (m, k))).cuda()
            insts.append({"op": op, "strategy": si, "A": A[:, :k],
                          "x": torch.from_numpy(synthetic.uniform_pm1(g, k)).cuda(),
                          "out": torch.empty(m, device="cuda")})
            continue
        n = int(2 ** g.uniform(8, 18)) if i % 4 else (1 << 18) - int(g.integers(0, 200))
        d = {"op": op, "strategy": si, "out": torch.empty(1, device="cuda"),
             "x": torch.from_numpy(synthetic.log_uniform_signed(g, n)).cuda()}
        if op == dp.OP_DOT:
            d["y"] = torch.from_numpy(synthetic.uniform_pm1(g, n)).cuda()
        insts.append(d)
    single = []
    for d in insts:
        s = strategies[d["strategy"]]
        if d["op"] == dp.OP_GEMV:
            single.append(dp.gemv(d["A"], d["x"], s).cpu().numpy())
        elif d["op"] == dp.OP_DOT:
            single.append(dp.dot(d["x"], d["y"], s).cpu().numpy())
        else:
            single.append(dp.asum(d["x"], s).cpu().numpy())
    plan = dp.BatchPlan(insts, strategies)
    ws_a, ws_b = plan.workspace(), plan.workspace()
    plan.upload(ws_a)
    plan.upload(ws_b)
    runs = ((ws_a, True), (ws_a, True), (ws_b, True), (ws_a, False), (ws_a, True), (ws_b, False))
    for run, (ws, one) in enumerate(runs):
        print(f"batch back-to-back run {run} one_launch={one}", flush=True)
        for d in insts:
            d["out"].fill_(float("nan"))
        plan.run(ws, one_launch=one)
        torch.cuda.synchronize()
        for i, (d, want) in enumerate(zip(insts, single)):
            assert_same_bits(d["out"].cpu().numpy(), want, f"run {run} instance {i}")
    plan.close()


# ------------------------------------------------ the outer fold, step edges
# The fold copies the chunk values into LDS a step at a time (256 values per
# step for a 64-thread work-group folding inside a 1-pass launch, 1024 for
# the 256-thread fold kernel of 2 passes and for wide 1-pass work-groups),
# with the next step's loads in flight while the current one is folded.  G
# around those sizes, with chunk values of 4 bytes (plain) and 8 (Kahan and
# Sum2 pairs, folded in binary64), on inputs whose sum depends on the order.
FOLD_STRATS = [
    # W = 1: one chunk per element, 64-thread work-groups
    dict(seq_len=1, local_size=1, order=T_, wg_combine=dp.SEQ),
    # W = 1024: a 256-thread team per chunk
    dict(seq_len=1, local_size=1024, order=T_),
]


@pytest.mark.parametrize("G", [1, 255, 256, 257, 1023, 1024, 1025, 2048, 2049, 3333])
@pytest.mark.parametrize("kw", FOLD_STRATS, ids=["W1", "W1024"])
@pytest.mark.parametrize("accum", [dp.PLAIN, dp.KAHAN, dp.SUM2], ids=["plain", "kahan", "sum2"])
def test_outer_fold_at_the_edges_of_its_steps(G, kw, accum):
    s = dp.Strategy(**kw, accum=accum, final_f64=1 if accum != dp.PLAIN else 0)
    W = kw["seq_len"] * kw["local_size"]
    if W > 1 and G > 1100:
        pytest.skip("the wide chunks reach the same steps at G <= 1025")
    n = G * W
    print(f"outer fold G={G} W={W} accum={accum}", flush=True)
    xd, yd = discriminating(70 + G % 13, n)
    want = S.dot(xd, yd, to_plan(s))
    for passes in (1, 2):
        assert_same_bits(gpu_dot(xd, yd, s.with_(passes=passes)), want,
                         f"G={G} W={W} passes={passes}")


# ------------------------------------------------ loader wavefronts
# Contiguous strategies with one 64-lane team per chunk and fewer chunks than
# compute units are folded by work-groups whose other wavefronts only load
# (whole lane rows of a multiple of the loaders' depth in tiles); a ragged
# last chunk is folded whole by one wavefront.  Tree and uncombined,
# scalar and V = 4 lanes, dot and asum, both pass counts; the chunk values
# of uncombined strategies element by element.
# (Tiles of 64 elements per lane row; uncombined chunks are split over 4, 2
# or 1 work-groups of 16, 32 or 64 lanes as the chunk count allows.)
FED = {
    "C256-tree": dict(seq_len=256, local_size=64, order=C_),                      # 4 tiles
    "C512-none": dict(seq_len=512, local_size=64, order=C_, wg_combine=dp.NONE),  # 8 tiles
    "C1024-none": dict(seq_len=1024, local_size=64, order=C_, wg_combine=dp.NONE),
    "C64-V4-tree": dict(seq_len=64, local_size=64, order=C_, vec_width=4),          # 4 tiles
    "sec62": dict(seq_len=2048, local_size=64, order=C_, vec_width=4, wg_combine=dp.NONE),
}


@pytest.mark.parametrize("chunks,short", [(1, 0), (3, 0), (37, 0), (37, 24), (100, 0),
                                          (200, 1000), (255, 0)])
@pytest.mark.parametrize("name", sorted(FED))
def test_contiguous_lanes_fed_by_loader_wavefronts(name, chunks, short):
    import torch
    s = dp.Strategy(**FED[name])
    W = s.seq_len * s.local_size * s.vec_width
    if W * chunks > (1 << 24):
        pytest.skip("the long rows reach the same path with fewer chunks")
    n = W * chunks - short
    print(f"fed {name} chunks={chunks} n={n}", flush=True)
    x, y = discriminating(80 + chunks, n)
    p = to_plan(s)
    for passes in (1, 2):
        sp = s.with_(passes=passes)
        assert_same_bits(gpu_dot(x, y, sp), S.dot(x, y, p), f"dot passes={passes}")
        assert_same_bits(gpu_asum(x, sp), S.asum(x, p), f"asum passes={passes}")
    if s.wg_combine == dp.NONE:
        c = dp.chunks(dp.OP_DOT, s, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
        torch.cuda.synchronize()
        assert_same_bits(c.cpu().numpy().view(np.float32), S.dot_chunks(x, y, p),
                         "chunk values")


@pytest.mark.parametrize("accum", [dp.KAHAN, dp.SUM2], ids=["kahan", "sum2"])
@pytest.mark.parametrize("final_f64", [0, 1])
def test_compensated_lanes_fed_by_loader_wavefronts(accum, final_f64):
    s = dp.Strategy(seq_len=256, local_size=64, order=C_, accum=accum, final_f64=final_f64)
    n = s.seq_len * s.local_size * 41
    x, y = synthetic.kahan_dot_inputs(n, synthetic.SEEDS["precision"])
    want = S.dot(x, y, to_plan(s))
    for passes in (1, 2):
        assert_same_bits(gpu_dot(x, y, s.with_(passes=passes)), want, f"passes={passes}")
    xd, yd = discriminating(90, n)
    assert_same_bits(gpu_dot(xd, yd, s), S.dot(xd, yd, to_plan(s)), "cancelling")


# ------------------------------------------------ one pass, many chunk values
# 1-pass uncombined strategies fed by loader wavefronts, with thousands of
# chunk values folded by the last work-group: chunk counts that split each
# chunk over 1, 2 or 4 work-groups, a ragged last chunk, scalar and V = 4
# lanes, dot and asum; twice in a row on one workspace, which the launch
# leaves with its arrival-counter block at zero.
ONE_PASS = {
    "C256-V4": dict(seq_len=256, local_size=64, order=C_, vec_width=4, wg_combine=dp.NONE),
    "C1024-V1": dict(seq_len=1024, local_size=64, order=C_, wg_combine=dp.NONE),
}


@pytest.mark.parametrize("chunks,short", [(40, 0), (100, 0), (200, 0), (255, 777)])
@pytest.mark.parametrize("name", sorted(ONE_PASS))
def test_one_pass_fed_launches_with_many_chunk_values(name, chunks, short):
    import torch
    s = dp.Strategy(**ONE_PASS[name], passes=1)
    W = s.seq_len * s.local_size * s.vec_width
    n = W * chunks - short
    print(f"one pass {name} chunks={chunks} n={n}", flush=True)
    x, y = discriminating(95 + chunks, n)
    p = to_plan(s)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    ws = dp.workspace(s, dp.OP_DOT, dp.F32, 0, n)
    want = S.dot(x, y, p)
    for rep in range(2):
        r = dp.dot(xt, yt, s, ws=ws)
        torch.cuda.synchronize()
        assert_same_bits(r.cpu().numpy()[0], want, f"dot call {rep}")
    assert_same_bits(gpu_dot(x, y, s.with_(passes=2)), want, "dot, 2 passes")
    assert_same_bits(gpu_asum(x, s), S.asum(x, p), "asum")
    assert not ws[-256:].any(), "arrival-counter block left non-zero"


# ------------------------------------------------ split tree teams
# Tree-combined contiguous teams of 64, 128 and 256 lanes with few chunks:
# their lanes are split over 2 to 8 work-groups, each reduces its slice to a
# node of the team's tree, and the last slice of a chunk applies the upper
# levels.  Bit-exact against the oracle; the chunk values from dpia_chunks
# (no workspace, so no split) equal the split launch's, and the per-chunk
# arrival counts are left at zero.
SPLIT = {
    "L64-C1024": dict(seq_len=1024, local_size=64, order=C_),
    "L128-C512": dict(seq_len=512, local_size=128, order=C_),
    "L256-C1024": dict(seq_len=1024, local_size=256, order=C_),
    "L256-C8192": dict(seq_len=8192, local_size=256, order=C_),
}


@pytest.mark.parametrize("chunks,short", [(1, 0), (5, 0), (31, 0), (31, 333), (60, 0),
                                          (100, 0)])
@pytest.mark.parametrize("name", sorted(SPLIT))
def test_split_tree_teams(name, chunks, short):
    import torch
    s = dp.Strategy(**SPLIT[name])
    W = s.seq_len * s.local_size
    if W * chunks > (1 << 25):
        pytest.skip("the long rows reach the same path with fewer chunks")
    n = W * chunks - short
    print(f"split tree {name} chunks={chunks} n={n}", flush=True)
    x, y = discriminating(110 + chunks, n)
    p = to_plan(s)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    want = S.dot(x, y, p)
    for passes in (1, 2):
        sp = s.with_(passes=passes)
        ws = dp.workspace(sp, dp.OP_DOT, dp.F32, 0, n)
        for rep in range(2):
            r = dp.dot(xt, yt, sp, ws=ws)
            torch.cuda.synchronize()
            assert_same_bits(r.cpu().numpy()[0], want, f"dot passes={passes} call {rep}")
        items = -(-n // W)
        counts = -(-items * 4 // 256) * 256         # the split region ends with them
        partial = -(-items * 4 // 256) * 256
        assert not ws[-counts:].any(), "per-chunk arrival counts left non-zero"
        assert not ws[partial:partial + 256].any(), "arrival counter left non-zero"
        assert_same_bits(gpu_asum(x, sp), S.asum(x, p), f"asum passes={passes}")
    c = dp.chunks(dp.OP_DOT, s, xt, yt)
    torch.cuda.synchronize()
    assert_same_bits(c.cpu().numpy().view(np.float32), S.dot_chunks(x, y, p), "chunk values")


@pytest.mark.parametrize("accum", [dp.KAHAN, dp.SUM2], ids=["kahan", "sum2"])
def test_split_tree_teams_compensated(accum):
    s = dp.Strategy(seq_len=1024, local_size=256, order=C_, accum=accum, final_f64=1)
    n = s.seq_len * s.local_size * 9
    x, y = synthetic.kahan_dot_inputs(n, synthetic.SEEDS["precision"])
    want = S.dot(x, y, to_plan(s))
    for passes in (1, 2):
        assert_same_bits(gpu_dot(x, y, s.with_(passes=passes)), want, f"passes={passes}")


# ------------------------------------------------ strided slices
# Scalar strided strategies with few chunks: each work-group folds a slice
# of 16, 32 or 64 lanes, one per thread, from 64-step tiles that loader
# wavefronts bring into LDS (step j of all lanes is one contiguous row);
# tree-combined chunks end in the split combine.  Ragged last chunks are
# folded by lane folds of one lane per thread.
STRIDED = {
    "L256-C8192-tree": dict(seq_len=8192, local_size=256, order=T_),
    "L64-C1024-tree": dict(seq_len=1024, local_size=64, order=T_),
    "L128-C512-none": dict(seq_len=512, local_size=128, order=T_, wg_combine=dp.NONE),
    "L512-C256-tree": dict(seq_len=256, local_size=512, order=T_),
}


@pytest.mark.parametrize("chunks,short", [(1, 0), (3, 0), (13, 5), (30, 0), (60, 1000)])
@pytest.mark.parametrize("name", sorted(STRIDED))
def test_strided_slices_fed_by_loader_wavefronts(name, chunks, short):
    import torch
    s = dp.Strategy(**STRIDED[name])
    W = s.seq_len * s.local_size
    if W * chunks > (1 << 25):
        pytest.skip("the long rows reach the same path with fewer chunks")
    n = W * chunks - short
    print(f"strided slices {name} chunks={chunks} n={n}", flush=True)
    x, y = discriminating(130 + chunks, n)
    p = to_plan(s)
    for passes in (1, 2):
        sp = s.with_(passes=passes)
        assert_same_bits(gpu_dot(x, y, sp), S.dot(x, y, p), f"dot passes={passes}")
        assert_same_bits(gpu_asum(x, sp), S.asum(x, p), f"asum passes={passes}")
    c = dp.chunks(dp.OP_DOT, s, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    assert_same_bits(c.cpu().numpy().view(np.float32), S.dot_chunks(x, y, p), "chunk values")


# ------------------------------------------------ strided gemv rows, one thread each
# A binary32 gemv in the strided order with L = 1, 2 or 4 lanes per row has
# one thread per row, holding all the row's lanes: it is folded through the
# contiguous LDS staging with L components.  One or two row parts, k that
# leaves the last part short, m not a multiple of the rows per work-group,
# and an odd k (L = 1: rows not 16-byte aligned, so not staged).
@pytest.mark.parametrize("L", [1, 2, 4])
@pytest.mark.parametrize("k,parts", [(4096, 1), (4096 - 40, 1), (2 * 2048 + 32, 2),
                                     (4096 - 3, 1)])
def test_strided_gemv_rows_of_one_thread_staged(L, k, parts):
    if k % L:
        pytest.skip("rows must stay aligned for L-lane loads (the call rejects this lda)")
    C = -(-k // (L * parts))
    C = -(-C // 32) * 32                  # whole 32-element tiles per row part
    s = dp.Strategy(seq_len=C, local_size=L, order=T_, rows_per_wg=4, row_parts=parts)
    m = 300                               # 256 rows per work-group: a partial last one
    print(f"strided gemv L={L} k={k} parts={parts} C={C}", flush=True)
    g = np.random.default_rng(L * 7 + k)
    A = (g.standard_normal((m, k)) * 2.0 ** g.uniform(-8, 8, (m, k))).astype(np.float32)
    x = (g.standard_normal(k) * 2.0 ** g.uniform(-8, 8, k)).astype(np.float32)
    from tests.gpu_util import gpu_gemv
    assert_same_bits(gpu_gemv(A, x, s), S.gemv(A, x, to_plan(s)), f"L={L} k={k}")


# Gemv rows fed by loader wavefronts: teams of one thread (strided L = 1, 2
# or 4 lanes as the thread's components, or one contiguous lane), strided
# teams of 2 threads of 4 lanes each, and contiguous teams of L threads, binary32 A, whole row parts with lanes of at
# least 64 tiles of 64 elements; 16, 32 or 64 lane rows per work-group.
# (m, k, C, L, order, combine, parts, lda padding)
FED_GEMV = {
    "L2-tree-16rows": (256, 16384, 8192, 2, T_, dp.TREE, 1, 0),
    "L1-2parts": (320, 16384, 8192, 1, T_, dp.TREE, 2, 0),
    "L4-tree": (64, 4096, 1024, 4, T_, dp.TREE, 1, 0),
    "L2-seq": (48, 8192, 4096, 2, T_, dp.SEQ, 1, 0),
    "L4-seq-2parts": (32, 8192, 1024, 4, T_, dp.SEQ, 2, 0),
    "contig-L1-2parts": (32, 8192, 4096, 1, C_, dp.TREE, 2, 0),
    "contig-L1": (16, 4096, 4096, 1, C_, dp.TREE, 1, 0),
    "L2-padded-rows": (64, 4096, 2048, 2, T_, dp.TREE, 1, 12),
    "L4-32rows": (8192, 4096, 1024, 4, T_, dp.TREE, 1, 0),
    # contiguous teams of L threads, one lane each
    "contig-L2-tree": (128, 16384, 8192, 2, C_, dp.TREE, 1, 0),
    "contig-L16": (16, 65536, 4096, 16, C_, dp.TREE, 1, 0),
    "contig-L8-2parts-seq": (16, 65536, 4096, 8, C_, dp.SEQ, 2, 0),
    "contig-L64": (4, 262144, 4096, 64, C_, dp.TREE, 1, 0),
    "contig-L32-padded": (8, 131072, 4096, 32, C_, dp.TREE, 1, 8),
    "contig-L4-64rows": (4096, 16384, 4096, 4, C_, dp.SEQ, 1, 0),
    "contig-L2-2parts-padded": (32, 16384, 4096, 2, C_, dp.TREE, 2, 12),
    "contig-L4-tree": (16, 16384, 4096, 4, C_, dp.TREE, 1, 0),
    # strided teams of 2 threads of 4 lanes each, sharing a row tile
    "strided-L8-tree": (64, 8192, 1024, 8, T_, dp.TREE, 1, 0),
    "strided-L8-2parts-seq": (32, 8192, 512, 8, T_, dp.SEQ, 2, 0),
    "strided-L8-2parts-padded": (16, 16384, 1024, 8, T_, dp.TREE, 2, 20),
    "strided-L8-32rows": (8192, 4096, 512, 8, T_, dp.TREE, 1, 0),
}


@pytest.mark.parametrize("name", list(FED_GEMV))
def test_gemv_rows_fed_by_loader_wavefronts(name):
    import torch
    m, k, C, L, order, comb, parts, pad = FED_GEMV[name]
    import math
    s = dp.Strategy(seq_len=C, local_size=L, order=order, wg_combine=comb,
                    rows_per_wg=math.gcd(16, m), row_parts=parts)
    print(f"fed gemv {name}: m={m} k={k} C={C} L={L} parts={parts} pad={pad}", flush=True)
    g = np.random.default_rng(m + k + C + L)
    A = (g.standard_normal((m, k)) * 2.0 ** g.uniform(-12, 12, (m, k))).astype(np.float32)
    x = (g.standard_normal(k) * 2.0 ** g.uniform(-12, 12, k)).astype(np.float32)
    # rows with cancelling products: every row's value is its rounding error
    xa, ya = discriminating(m * 3 + 1, k)
    A[0], x[:] = xa, ya
    A[1] = -xa
    Ap = np.zeros((m, k + pad), np.float32)
    Ap[:, :k] = A
    At = cuda(Ap)[:, :k]
    y = dp.gemv(At, cuda(x), s)
    torch.cuda.synchronize()
    assert_same_bits(y.cpu().numpy(), S.gemv(A, x, to_plan(s)), name)


def test_gemv_blas_rows_of_one_thread_fed():
    import torch
    m, k = 32, 8192
    s = dp.Strategy(seq_len=4096, local_size=2, order=T_, rows_per_wg=16)
    g = np.random.default_rng(77)
    A = (g.standard_normal((m, k)) * 2.0 ** g.uniform(-6, 6, (m, k))).astype(np.float32)
    x = g.standard_normal(k).astype(np.float32)
    y0 = g.standard_normal(m).astype(np.float32)
    yt = cuda(y0.copy())
    dp.gemv_blas(1.5, cuda(A), cuda(x), -0.75, yt, s)
    torch.cuda.synchronize()
    want = S.gemv_blas(np.float32(1.5), A, x, np.float32(-0.75), y0, to_plan(s))
    assert_same_bits(yt.cpu().numpy(), want, "gemv_blas fed")


# Fed gemv work-groups looping over several row groups (the strategy caps the
# grid at 2 work-groups): the ring, the x rows and the combine regions are
# reused from one row group to the next.  (m, k, C, L, order, combine, parts)
FED_GEMV_LOOP = {
    "L2-rows-of-one": (96, 4096, 2048, 2, T_, dp.TREE, 1),
    "L8-teams-of-two-seq": (64, 8192, 512, 8, T_, dp.SEQ, 2),
    "contig-L2-x-rows": (48, 16384, 4096, 2, C_, dp.TREE, 2),
    "contig-L16-seq": (8, 65536, 4096, 16, C_, dp.SEQ, 1),
}


@pytest.mark.parametrize("name", list(FED_GEMV_LOOP))
def test_gemv_fed_work_groups_loop_over_row_groups(name):
    import math
    import torch
    m, k, C, L, order, comb, parts = FED_GEMV_LOOP[name]
    s = dp.Strategy(seq_len=C, local_size=L, order=order, wg_combine=comb,
                    rows_per_wg=math.gcd(16, m), row_parts=parts, max_grid=2)
    print(f"fed gemv loop {name}: m={m} k={k} C={C} L={L} parts={parts}", flush=True)
    g = np.random.default_rng(m * 7 + L)
    A = (g.standard_normal((m, k)) * 2.0 ** g.uniform(-12, 12, (m, k))).astype(np.float32)
    x = (g.standard_normal(k) * 2.0 ** g.uniform(-12, 12, k)).astype(np.float32)
    y = dp.gemv(cuda(A), cuda(x), s)
    torch.cuda.synchronize()
    assert_same_bits(y.cpu().numpy(), S.gemv(A, x, to_plan(s)), name)
