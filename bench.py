"""Throughput of the strategy-preserving dot + gemv on one MI355X.

One step = one FP32 dot product of N = 2^26 (x, y uniform in [-1, 1]) and
one FP32 gemv y = A x with A 8192 x 8192 row-major, entries N(0, 1), x
uniform in [-1, 1] (seed 1712), each under a fixed DPIA strategy; the dot is
one kernel (its last work-group folds the chunk values), and the gemv reads
three copies of A in turn, so that none is served from the last-level cache.  Inputs are
resident in HBM before timing starts.  Value = algorithmic bytes of the step
(every input element read once, results written once) x steps / wall time,
in GB/s.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

Prints one JSON line.  Besides the whole-job figure it reports the dominant
kernel (the dot) against the HBM roofline, timed with HIP events on the
stream the kernels run on, and the CPU oracle timed on this host's cores on
the same workload (bounded to a few repetitions).

Other workloads (one JSON line per measured item, not the headline):
    --workload small      dot and asum N = 2^20 under split 4096 / 256 / tree /
                          2 passes (cache-resident: time and parity only)
    --workload sweep      dot N = 2^26 and gemv 16384^2 over the 24-strategy
                          sweep each, with the autotuner's pick
    --workload precision  gemv 16384^2 with bf16 and fp8-e4m3 (row-scaled) A,
                          and the compensated dots (Kahan, Sum2) at N = 2^28, with their
                          error against the exact (binary64-correctly-rounded)
                          value
    --workload batch      4096 dot / asum instances (n log-uniform in
                          [2^8, 2^20]) and 512 gemvs (m, k in [64, 4096]),
                          strategies tuned per size class: per-instance
                          launches (eager, graph) against one batched run
                          by each engine, two launches or one (eager, graph)
    --workload scal       scal y = alpha x, N = 2^26, under strided and
                          contiguous strategies, out of place and in place;
                          and the BLAS gemv y := alpha A x + beta y beside
                          y = A x (binary32, 8192^2 and 16384^2)
    --workload vector     dot N = 2^26 under vector (asVector 4) strategies,
                          among them the dot expression of Sec. 6.2 (float4
                          views, 64 work-items folding 2048 vectors each, no
                          work-group combine): chunk kernel and fold timed
                          apart
    --workload generated  the headline dot and gemv strategies compiled from
                          their DPIA expressions by the generator, timed
                          beside the hand-written kernels (same bits)
    --workload kernels    each hot kernel (the dot, f32 / bf16 / fp8
                          gemvs) launched --steps times with the cache evicted
                          in between, beside the read-stream ceiling on the
                          same bytes: a fixed kernel mix for counter runs
Oracle work (parity, exact references) runs only in the CPU-baseline leg,
which --no-cpu-baseline skips.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

import paper_1710_08332_amd as dp
from paper_1710_08332_amd.timing import TimingEvents

METRIC = "HBM GB/s (% of peak) for dot/asum/gemv per strategy; batched vs plain"
PEAK_GBPS = 8000.0   # MI355X HBM3E, published

N_DOT = 1 << 26
M_GEMV = K_GEMV = 8192
SEED = 1712

# split 262144 -> mapWorkgroup (1024 lanes, each folding a strided row of 256
# -> mapLocal reduceSeq) -> tree in local memory; then reduceSeq over the 256
# chunk values, in the last work-group to finish (one kernel)
DOT_STRATEGY = dp.Strategy(seq_len=256, local_size=1024, order=dp.STRIDED, wg_combine=dp.TREE,
                           passes=1)
# rows of 8192 = 256 lanes x 32 strided elements, tree, 4 rows per work-group
GEMV_STRATEGY = dp.Strategy(seq_len=32, local_size=256, order=dp.STRIDED, wg_combine=dp.TREE,
                            rows_per_wg=4)

DOT_BYTES = 2 * 4 * N_DOT + 4                    # x, y read; one result written
G_DOT = N_DOT // (DOT_STRATEGY.seq_len * DOT_STRATEGY.local_size)
# the whole dot in one kernel: x, y read, G chunk values written and read
# back by the last work-group, the result written
DOT_KERNEL_BYTES = 2 * 4 * N_DOT + 2 * 4 * G_DOT + 4
GEMV_BYTES = 4 * M_GEMV * K_GEMV + 4 * K_GEMV + 4 * M_GEMV
A_COPIES = 3


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "dot_f32_2p26_and_gemv_f32_8192_hbm_traffic.md")


def measured_traffic():
    """HBM bytes per launch of the dot kernel from the committed rocprofv3
    counter summary, or None when the kernel sources changed since
    the counters were taken (their hash no longer matches)."""
    import hashlib
    try:
        kv = dict(line.split(": ", 1) for line in open(TRAFFIC_FILE).read().splitlines()
                  if ": " in line and not line.startswith(("|", "-", "#", " ")))
        h = hashlib.sha256()
        root = os.path.dirname(os.path.abspath(__file__))
        for f in kv["sources"].split():
            h.update(open(os.path.join(root, f), "rb").read())
        if h.hexdigest() != kv["source_sha256"].strip():
            return None
        return int(kv["dot_traffic_bytes"])
    except (OSError, KeyError, ValueError):
        return None


def strategy_text(s: dp.Strategy, gemv: bool = False) -> str:
    comb = {dp.TREE: "tree", dp.SEQ: "seq", dp.NONE: "uncombined"}[s.wg_combine]
    return (f"C={s.seq_len} L={s.local_size} {'strided' if s.order == dp.STRIDED else 'contiguous'}"
            f" {comb}" + (f" V={s.vec_width}" if s.vec_width > 1 else "")
            + (f" R={s.rows_per_wg}" if gemv else f" passes={s.passes}"))


def cpu_baseline(x, y, A, xv, gpu_dot_val, gpu_y, budget_s=10.0):
    """The oracle on the same step, timed twice on this host: serially on
    one core, and with its outermost maps (the dot's chunks, the gemv's rows)
    evaluated by worker processes on every core this process may use; each
    repeated until about ``budget_s`` seconds have passed.  Also confirms bit
    parity of the measured GPU results with both."""
    from oracle import parallel as P
    from oracle import strategies as S
    from tests.gpu_util import to_plan
    dplan, gplan = to_plan(DOT_STRATEGY), to_plan(GEMV_STRATEGY)
    step_bytes = DOT_BYTES + GEMV_BYTES

    def timed(run):
        reps, t0 = 0, time.perf_counter()
        while True:
            d, g = run()
            reps += 1
            el = time.perf_counter() - t0
            if el >= budget_s or reps >= 1000:
                return d, g, reps, el

    d1, g1, reps1, el1 = timed(lambda: (S.dot(x, y, dplan), S.gemv(A, xv, gplan)))
    t0 = time.perf_counter()
    with P.Evaluator({"xs": x, "ys": y, "A": A, "x": xv}) as ev:
        setup = time.perf_counter() - t0
        dn, gn, repsn, eln = timed(lambda: (ev.dot(dplan), ev.gemv(gplan)))
        workers = ev.workers

    def same(a, b):
        return bool(np.array_equal(np.asarray(a, np.float32).view(np.uint32),
                                   np.asarray(b, np.float32).view(np.uint32)))
    parity = {"dot_bit_exact": same(d1, gpu_dot_val) and same(dn, gpu_dot_val),
              "gemv_bit_exact": same(g1, gpu_y) and same(gn, gpu_y)}
    one = step_bytes * reps1 / el1 / 1e9
    many = step_bytes * repsn / eln / 1e9
    return {"value": round(many, 3), "unit": "GB/s", "cores": workers, "kind": "oracle",
            "cpu_model": P.cpu_model(), "host_cores_available": P.host_cores(cap=1 << 16),
            "sample": f"the full step (dot 2^26 + gemv 8192^2, same strategies) x {repsn} "
                      f"repetitions in {eln:.1f} s, the dot's chunks and the gemv's rows split "
                      f"over {workers} worker processes (pool set-up {setup:.1f} s, untimed)",
            "single_core": {"value": round(one, 3), "cores": 1,
                            "sample": f"the full step x {reps1} repetitions in {el1:.1f} s, "
                                      "serial"}}, parity


def _line(**kw):
    print(json.dumps(kw), flush=True)


def _gbs(nbytes, us):
    return round(nbytes / us / 1e3, 1)


def workload_small(args):
    import torch
    import synthetic
    from paper_1710_08332_amd.autotune import time_us
    n = 1 << 20
    x, y = synthetic.dot_inputs(n, synthetic.SEEDS["small"])
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    s = dp.Strategy(seq_len=256, local_size=16, order=dp.CONTIGUOUS, wg_combine=dp.TREE, passes=2)
    ws = dp.workspace(s, dp.OP_DOT, dp.F32, 0, n)
    out = torch.empty(1, device="cuda")
    res = {}
    for name, fn, nbytes in (("dot", lambda: dp.dot(xt, yt, s, out=out, ws=ws), 8 * n + 4),
                             ("asum", lambda: dp.asum(xt, s, out=out, ws=ws), 4 * n + 4)):
        med, p10, p90 = time_us(fn, reps=100)
        fn()
        torch.cuda.synchronize()
        res[name] = out.cpu().numpy()[0]
        # the ceiling for these bytes when they are cache-resident: the plain
        # read kernel over a buffer of the same size, back to back (warm),
        # best of five grids
        buf = torch.ones((nbytes - 4) // 4, dtype=torch.int32, device="cuda")   # the inputs
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        sink = torch.empty(cus * 16, dtype=torch.int32, device="cuda")
        ceil_us = min(time_us(lambda g=g: dp.read_stream(buf, g, sink=sink), reps=100)[0]
                      for g in (cus // 4, cus // 2, cus, 2 * cus, 4 * cus))
        one = s.with_(passes=1)
        ws1 = dp.workspace(one, dp.OP_DOT, dp.F32, 0, n)
        run1 = ((lambda: dp.dot(xt, yt, one, out=out, ws=ws1)) if name == "dot"
                else (lambda: dp.asum(xt, one, out=out, ws=ws1)))
        med1 = time_us(run1, reps=100)[0]
        _line(workload="small", op=name, n=n, strategy=strategy_text(s), us=round(med, 2),
              p10=round(p10, 2), p90=round(p90, 2), gbs=_gbs(nbytes, med),
              one_pass_us=round(med1, 2), warm_read_ceiling_us=round(ceil_us, 2),
              pct_of_warm_read_ceiling=round(100 * ceil_us / med, 1),
              note="cache-resident (2^20 elements fit in L2/MALL): no HBM claim; the ceiling is "
                   "the read kernel over the same bytes, warm")
    if not args.no_cpu_baseline:
        from oracle import strategies as S
        from tests.gpu_util import to_plan
        t0 = time.perf_counter()
        d = S.dot(x, y, to_plan(s))
        a = S.asum(x, to_plan(s))
        el = time.perf_counter() - t0
        _line(workload="small", cpu_baseline={"kind": "oracle", "cores": 1, "seconds": round(el, 3)},
              parity={"dot_bit_exact": bool(np.float32(d).view(np.uint32) == np.float32(res["dot"]).view(np.uint32)),
                      "asum_bit_exact": bool(np.float32(a).view(np.uint32) == np.float32(res["asum"]).view(np.uint32))})


def workload_sweep(args):
    import dataclasses
    import torch
    import synthetic
    from paper_1710_08332_amd import autotune as T
    seed = synthetic.SEEDS["sweep"]
    n = 1 << 26
    x, y = synthetic.dot_inputs(n, seed)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    best, table = T.tune_dot(xt, yt, reps=args.steps)
    outs = {}
    for row in table:
        st = dp.Strategy(**row["strategy"])
        _line(workload="sweep", op="dot", n=n, strategy=strategy_text(st), us=round(row["us"], 2),
              p10=round(row["p10"], 2), p90=round(row["p90"], 2), gbs=_gbs(8 * n + 4, row["us"]),
              pct_peak=round(100 * (8 * n + 4) / row["us"] / 1e3 / PEAK_GBPS, 1))
        outs[st] = dp.dot(xt, yt, st).cpu().numpy()[0]
    _line(workload="sweep", op="dot", autotuned=dataclasses.asdict(best), text=strategy_text(best))
    del xt, yt
    m = k = 16384
    A, xv = synthetic.gemv_inputs(m, k, seed)
    At, xvt = torch.from_numpy(A).cuda(), torch.from_numpy(xv).cuda()
    gbest, gtable = T.tune_gemv(At, xvt, reps=args.steps)
    gbytes = 4 * (m * k + m + k)
    gouts = {}
    for row in gtable:
        st = dp.Strategy(**row["strategy"])
        _line(workload="sweep", op="gemv", m=m, k=k, strategy=strategy_text(st, gemv=True)
              + f" parts={st.row_parts}", us=round(row["us"], 2), p10=round(row["p10"], 2),
              p90=round(row["p90"], 2), gbs=_gbs(gbytes, row["us"]),
              pct_peak=round(100 * gbytes / row["us"] / 1e3 / PEAK_GBPS, 1))
        gouts[st] = dp.gemv(At, xvt, st).cpu().numpy()
    _line(workload="sweep", op="gemv", autotuned=dataclasses.asdict(gbest),
          text=strategy_text(gbest, gemv=True))
    if not args.no_cpu_baseline:
        from oracle import strategies as S
        from tests.gpu_util import to_plan
        t0 = time.perf_counter()
        dot_ok = all(np.float32(S.dot(x, y, to_plan(st))).view(np.uint32) == np.float32(v).view(np.uint32)
                     for st, v in outs.items())
        gemv_ok = all(np.array_equal(S.gemv(A, xv, to_plan(st)).view(np.uint32), v.view(np.uint32))
                      for st, v in gouts.items())
        _line(workload="sweep", cpu_baseline={"kind": "oracle", "cores": 1,
                                              "seconds": round(time.perf_counter() - t0, 1)},
              parity={"dot_all_24_bit_exact": bool(dot_ok), "gemv_all_24_bit_exact": bool(gemv_ok)})


KAHAN_DOT = dp.Strategy(seq_len=256, local_size=1024, order=dp.STRIDED, wg_combine=dp.TREE,
                        passes=2, accum=dp.KAHAN, final_f64=1)


PRECISION_CANDIDATES = [(64, 256), (128, 128), (32, 512), (16, 1024), (8, 2048)]


def workload_precision(args):
    import dataclasses
    import torch
    import synthetic
    from paper_1710_08332_amd import autotune as T
    from paper_1710_08332_amd.autotune import time_us
    seed = synthetic.SEEDS["precision"]
    m = k = 16384
    A, xv = synthetic.gemv_inputs(m, k, seed)
    xvt = torch.from_numpy(xv).cuda()
    codes16 = synthetic.quantise_bf16(A)
    codes8, scale = synthetic.quantise_fp8_rows(A)
    results, chosen = {}, {}
    evict = T.cache_evictor()
    cands = [dp.Strategy(seq_len=C, local_size=L, order=dp.STRIDED, wg_combine=dp.TREE)
             for C, L in PRECISION_CANDIDATES]
    for name, codes, dt, sc, nbytes in (
            ("gemv_f32", A, dp.F32, None, 4 * m * k + 4 * k + 4 * m),
            ("gemv_bf16", codes16.view(np.int16), dp.BF16, None, 2 * m * k + 4 * k + 4 * m),
            ("gemv_fp8", codes8, dp.FP8_E4M3, scale, m * k + 4 * k + 8 * m)):
        At = torch.from_numpy(np.ascontiguousarray(codes)).cuda()
        sct = torch.from_numpy(sc).cuda() if sc is not None else None
        y = torch.empty(m, device="cuda")
        # the strategy for this format: autotuned over the candidate tilings
        s, table = T.tune(cands, lambda st: (lambda: dp.gemv(At, xvt, st, y=y, row_scale=sct,
                                                             a_dtype=dt)), reps=10)
        chosen[name] = s
        # timed with the last-level cache evicted before every call (the fp8
        # matrix alone is about the size of the 256 MB cache)
        med, p10, p90 = time_us(lambda: dp.gemv(At, xvt, s, y=y, row_scale=sct, a_dtype=dt),
                                reps=args.steps, between=evict)
        results[name] = y.cpu().numpy()
        # the read-stream ceiling over the matrix's own bytes, timed the same way
        ceil_us, _ = evicted_read_ceiling(At, evict)
        a_bytes = At.numel() * At.element_size()
        _line(workload="precision", op=name, m=m, k=k, strategy=strategy_text(s, gemv=True),
              us=round(med, 2), p10=round(p10, 2), p90=round(p90, 2), gbs=_gbs(nbytes, med),
              pct_peak=round(100 * nbytes / med / 1e3 / PEAK_GBPS, 1), algorithmic_bytes=nbytes,
              read_ceiling_gbs=_gbs(a_bytes, ceil_us),
              pct_of_read_ceiling=round(100 * (nbytes / med) / (a_bytes / ceil_us), 1),
              tuned_over=[f"C={r['strategy']['seq_len']} L={r['strategy']['local_size']}: "
                          f"{r['us']:.1f} us" for r in table])
        del At
    n = 1 << 28
    x, y = synthetic.kahan_dot_inputs(n, seed)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    ws = dp.workspace(KAHAN_DOT, dp.OP_DOT, dp.F32, 0, n)
    plain = KAHAN_DOT.with_(accum=dp.PLAIN, final_f64=0)
    sum2 = KAHAN_DOT.with_(accum=dp.SUM2)
    out32 = torch.empty(1, device="cuda")
    out2 = torch.empty(1, dtype=torch.float64, device="cuda")
    for name, fn, o in (("dot_kahan", lambda: dp.dot(xt, yt, KAHAN_DOT, out=out, ws=ws), out),
                        ("dot_sum2", lambda: dp.dot(xt, yt, sum2, out=out2, ws=ws), out2),
                        ("dot_plain", lambda: dp.dot(xt, yt, plain, out=out32, ws=ws), out32)):
        med, p10, p90 = time_us(fn, reps=args.steps)
        fn()
        torch.cuda.synchronize()
        results[name] = o.cpu().numpy()[0]
        _line(workload="precision", op=name, n=n, strategy=strategy_text(KAHAN_DOT), us=round(med, 2),
              p10=round(p10, 2), p90=round(p90, 2), gbs=_gbs(8 * n + 8, med),
              pct_peak=round(100 * (8 * n + 8) / med / 1e3 / PEAK_GBPS, 1))
    if not args.no_cpu_baseline:
        import math
        from oracle import exact
        from oracle import strategies as S
        from tests.gpu_util import to_plan
        t0 = time.perf_counter()
        ex = exact.gemv_exact(A, xv)
        absx = np.abs(A.astype(np.float64)) @ np.abs(xv.astype(np.float64))
        ref = {"gemv_f32": S.gemv(A, xv, to_plan(chosen["gemv_f32"])),
               "gemv_bf16": S.gemv(codes16, xv, to_plan(chosen["gemv_bf16"]), a_format="bf16"),
               "gemv_fp8": S.gemv(codes8, xv, to_plan(chosen["gemv_fp8"]), a_format="fp8",
                                  scale=scale)}
        for name in ("gemv_f32", "gemv_bf16", "gemv_fp8"):
            got = results[name].astype(np.float64)
            _line(workload="precision", op=name, bit_exact_vs_oracle=bool(np.array_equal(
                      results[name].view(np.uint32), ref[name].view(np.uint32))),
                  max_rel_err_vs_exact_f32_A=float(np.max(np.abs(got - ex) / absx)),
                  note="error normalised by sum |A_rk x_k| per row; includes quantisation for bf16/fp8")
        prod = x.astype(np.float64) * y.astype(np.float64)
        sx = math.fsum(prod)
        sabs = math.fsum(np.abs(prod))
        # exact sum of the binary32-rounded products: what a perfect
        # accumulator of the kernel's products would return
        s32 = math.fsum((x * y).astype(np.float64))
        kref = S.dot(x, y, to_plan(KAHAN_DOT))
        sref = S.dot(x, y, to_plan(sum2))
        pref = S.dot(x, y, to_plan(plain))
        _line(workload="precision", op="dot_kahan",
              bit_exact_vs_oracle=bool(np.float64(kref).view(np.uint64) == np.float64(results["dot_kahan"]).view(np.uint64)),
              rel_err_vs_exact=abs(float(results["dot_kahan"]) - sx) / sabs,
              plain_rel_err_vs_exact=abs(float(results["dot_plain"]) - sx) / sabs,
              accumulation_err=abs(float(results["dot_kahan"]) - s32) / sabs,
              plain_accumulation_err=abs(float(results["dot_plain"]) - s32) / sabs,
              plain_bit_exact_vs_oracle=bool(np.float32(pref).view(np.uint32) == np.float32(results["dot_plain"]).view(np.uint32)),
              sum2_bit_exact_vs_oracle=bool(np.float64(sref).view(np.uint64) == np.float64(results["dot_sum2"]).view(np.uint64)),
              sum2_rel_err_vs_exact=abs(float(results["dot_sum2"]) - sx) / sabs,
              sum2_accumulation_err=abs(float(results["dot_sum2"]) - s32) / sabs,
              cpu_seconds=round(time.perf_counter() - t0, 1),
              note="normwise: |computed - exact| / sum |x_i y_i|; exact = math.fsum of binary64 "
                   "products; accumulation_err uses the exact sum of the binary32-rounded "
                   "products instead (rounding of the accumulation alone)")


def batch_instances(seed: int, n_red: int = 4096, n_gemv: int = 512):
    """Config 5: n_red dot / asum instances (seeded coin) with n = floor(2^U(8, 20))
    and n_gemv gemvs with m, k uniform in {64..4096}; all data uniform in
    [-1, 1].  Returns (instances, host copies, algorithmic bytes)."""
    import torch
    import synthetic
    g = synthetic.rng(seed)
    insts, host, nbytes = [], [], 0
    for _ in range(n_red):
        op = dp.OP_DOT if g.random() < 0.5 else dp.OP_ASUM
        n = int(2 ** g.uniform(8, 20))
        x = synthetic.uniform_pm1(g, n)
        d = {"op": op, "x": torch.from_numpy(x).cuda(), "out": torch.empty(1, device="cuda")}
        y = None
        if op == dp.OP_DOT:
            y = synthetic.uniform_pm1(g, n)
            d["y"] = torch.from_numpy(y).cuda()
            nbytes += 8 * n + 4
        else:
            nbytes += 4 * n + 4
        insts.append(d)
        host.append((op, x, y))
    for _ in range(n_gemv):
        m, k = int(g.integers(64, 4097)), int(g.integers(64, 4097))
        lda = -(-k // 4) * 4
        A = torch.empty((m, lda), dtype=torch.float32, device="cuda")
        Ah = synthetic.uniform_pm1(g, (m, k))
        A[:, :k].copy_(torch.from_numpy(Ah))
        x = synthetic.uniform_pm1(g, k)
        insts.append({"op": dp.OP_GEMV, "A": A[:, :k], "x": torch.from_numpy(x).cuda(),
                      "out": torch.empty(m, device="cuda")})
        host.append((dp.OP_GEMV, Ah, x))
        nbytes += 4 * (m * k + k + m)
    return insts, host, nbytes


def workload_batch(args):
    import torch
    import synthetic
    from paper_1710_08332_amd import autotune as T
    from paper_1710_08332_amd.autotune import time_us
    t0 = time.perf_counter()
    insts, host, nbytes = batch_instances(synthetic.SEEDS["batch"])
    gen_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    strategies, assign, table = T.tune_batch(insts, reps=5)
    tune_s = time.perf_counter() - t0
    for i, d in enumerate(insts):
        d["strategy"] = assign[i]
    plan = dp.BatchPlan(insts, strategies)
    ws = plan.workspace()
    plan.upload(ws)

    # per-instance calls, each with its class's strategy (2 passes), one
    # shared workspace (calls are ordered on the stream)
    big = max(dp.strategy_check(strategies[assign[i]], d["op"], dp.F32, 0, d["x"].numel())
              for i, d in enumerate(insts) if d["op"] != dp.OP_GEMV)
    ws1 = torch.zeros(big, dtype=torch.uint8, device="cuda")

    def per_instance():
        for i, d in enumerate(insts):
            s = strategies[assign[i]]
            if d["op"] == dp.OP_DOT:
                dp.dot(d["x"], d["y"], s, out=d["out"], ws=ws1)
            elif d["op"] == dp.OP_ASUM:
                dp.asum(d["x"], s, out=d["out"], ws=ws1)
            else:
                dp.gemv(d["A"], d["x"], s, y=d["out"])

    def graphed(fn):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            fn()
            torch.cuda.synchronize()
            with torch.cuda.graph(gr, stream=side):
                fn()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        return gr

    reps = max(3, min(args.steps, 20))
    rows = {}
    per_us, _, _ = time_us(per_instance, reps=3, warmup=1)
    per_out = [d["out"].clone() for d in insts]
    rows["per_instance_eager"] = per_us
    g1 = graphed(per_instance)
    rows["per_instance_graph"] = time_us(g1.replay, reps=reps, warmup=1)[0]
    same = True
    for one in (False, True):
        name = "one_launch" if one else "two_launches"
        rows[f"batched_{name}_eager"] = time_us(lambda: plan.run(ws, one_launch=one), reps=reps,
                                                warmup=1)[0]
        g2 = graphed(lambda: plan.run(ws, one_launch=one))
        rows[f"batched_{name}_graph"] = time_us(g2.replay, reps=reps, warmup=1)[0]
        del g2
        for d in insts:
            d["out"].fill_(float("nan"))
        plan.run(ws, one_launch=one)
        torch.cuda.synchronize()
        same = same and all(np.array_equal(d["out"].cpu().numpy().view(np.uint32),
                                           p.cpu().numpy().view(np.uint32))
                            for d, p in zip(insts, per_out))
    for name, us in rows.items():
        _line(workload="batch", mode=name, instances=len(insts), us=round(us, 1),
              gbs=_gbs(nbytes, us), pct_peak=round(100 * nbytes / us / 1e3 / PEAK_GBPS, 1),
              speedup_vs_per_instance_graph=round(rows["per_instance_graph"] / us, 2))
    _line(workload="batch", algorithmic_bytes=nbytes, batched_equals_per_instance_bitwise=bool(same),
          strategies=[strategy_text(s) for s in strategies],
          size_classes=len({row["class"] for row in table}), tuning_runs=len(table),
          tune_seconds=round(tune_s, 1), generate_seconds=round(gen_s, 1),
          note="batched: two launches (tiles, then folds) or one persistent launch (per-instance "
               "arrival counters, the last tile folds); per-instance = one call per instance "
               "(2 kernels per reduction); the same strategies throughout")
    if not args.no_cpu_baseline:
        from oracle import strategies as S
        from tests.gpu_util import to_plan
        g = np.random.default_rng(5)
        sample = sorted(g.choice(len(insts), size=64, replace=False).tolist())
        ok = True
        t0 = time.perf_counter()
        for i in sample:
            op, a, b = host[i]
            p = to_plan(strategies[assign[i]])
            got = insts[i]["out"].cpu().numpy()
            if op == dp.OP_GEMV:
                want = S.gemv(a, b, p)
            elif op == dp.OP_DOT:
                want = np.atleast_1d(S.dot(a, b, p))
            else:
                want = np.atleast_1d(S.asum(a, p))
            ok = ok and np.array_equal(got.view(np.uint32), np.asarray(want, np.float32).view(np.uint32))
        _line(workload="batch", cpu_baseline={"kind": "oracle", "cores": 1, "sample": "64 random instances",
                                              "seconds": round(time.perf_counter() - t0, 1)},
              parity={"sample_bit_exact": bool(ok)})


def workload_scal(args):
    import torch
    import synthetic
    from paper_1710_08332_amd.autotune import time_us
    n = 1 << 26
    x, _ = synthetic.dot_inputs(n, synthetic.SEEDS["scale"])
    alpha = np.float32(-1.3)
    xt = torch.from_numpy(x).cuda()
    yt = torch.empty_like(xt)
    # in place, x is 256 MiB: evict the last-level cache before every timed call
    from paper_1710_08332_amd.autotune import cache_evictor
    evict = cache_evictor()
    strategies = [dp.Strategy(seq_len=C, local_size=L, order=o)
                  for C, L, o in ((16, 1024, dp.STRIDED), (64, 1024, dp.STRIDED),
                                  (256, 1024, dp.STRIDED), (16, 256, dp.CONTIGUOUS),
                                  (64, 256, dp.CONTIGUOUS))]
    # the copy ceiling: the runtime's device-to-device copy of the same bytes
    # (read 256 MiB, write 256 MiB), timed the same way
    cp_us = time_us(lambda: yt.copy_(xt), reps=40, between=evict)[0]
    _line(workload="scal", op="copy_ceiling", n=n, us=round(cp_us, 2), gbs=_gbs(8 * n, cp_us),
          pct_peak=round(100 * 8 * n / cp_us / 1e3 / PEAK_GBPS, 1))
    for s in strategies:
        for place in ("out", "in"):
            dst = yt if place == "out" else xt
            med, p10, p90 = time_us(lambda: dp.scal(float(alpha), xt, s, y=dst), reps=40,
                                    between=evict)
            _line(workload="scal", n=n, strategy=strategy_text(s), place=place,
                  us=round(med, 2), p10=round(p10, 2), p90=round(p90, 2),
                  gbs=_gbs(8 * n, med), pct_peak=round(100 * 8 * n / med / 1e3 / PEAK_GBPS, 1),
                  pct_of_copy=round(100 * cp_us / med, 1))
    xt.copy_(torch.from_numpy(x))
    dp.scal(float(alpha), xt, strategies[0], y=yt)
    torch.cuda.synchronize()
    # the BLAS gemv y := alpha A x + beta y beside the plain y = A x, binary32
    # 8192^2 (the headline strategy) and 16384^2, cache evicted before each call
    blas_out = {}
    for mk, gs in ((8192, GEMV_STRATEGY),
                   (16384, dp.Strategy(seq_len=32, local_size=512, order=dp.STRIDED,
                                       wg_combine=dp.TREE))):
        A, xv = synthetic.gemv_inputs(mk, mk, synthetic.SEEDS["scale"])
        At, xvt = torch.from_numpy(A).cuda(), torch.from_numpy(xv).cuda()
        y0 = torch.from_numpy(synthetic.dot_inputs(mk, synthetic.SEEDS["scale"] + 1)[0]).cuda()
        yb = torch.empty_like(y0)
        # the read-stream ceiling on A itself, timed the same way (cache evicted)
        ceil_us, ceil_grid = evicted_read_ceiling(At, evict)
        a_bytes = 4 * mk * mk
        _line(workload="scal", op="read_ceiling", bytes=a_bytes, grid=ceil_grid,
              us=round(ceil_us, 2), gbs=_gbs(a_bytes, ceil_us),
              pct_peak=round(100 * a_bytes / ceil_us / 1e3 / PEAK_GBPS, 1))
        for form, a_, b_, nbytes in (("y = A x", 1.0, 0.0, 4 * (mk * mk + 2 * mk)),
                                     ("y := 1.3 A x - 2.1 y", 1.3, -2.1, 4 * (mk * mk + 3 * mk))):
            def run():
                if b_ == 0.0:
                    dp.gemv(At, xvt, gs, y=yb)
                else:      # in place: y grows by about 2.1x per call, far from overflow
                    dp.gemv_blas(a_, At, xvt, b_, yb, gs)
            yb.copy_(y0)
            med, p10, p90 = time_us(run, reps=20, between=evict)
            _line(workload="scal", op="gemv_blas" if b_ else "gemv", m=mk, k=mk, form=form,
                  strategy=strategy_text(gs, gemv=True), us=round(med, 2), p10=round(p10, 2),
                  p90=round(p90, 2), gbs=_gbs(nbytes, med),
                  pct_peak=round(100 * nbytes / med / 1e3 / PEAK_GBPS, 1),
                  pct_of_read_ceiling=round(100 * (nbytes / med) / (a_bytes / ceil_us), 1))
            if mk == 8192:
                yb.copy_(y0)
                run()
                blas_out[form] = yb.cpu().numpy()
        if mk == 8192:
            blas_in = (A, xv, y0.cpu().numpy(), gs)
        del At
    if not args.no_cpu_baseline:
        from oracle import strategies as S
        from tests.gpu_util import to_plan
        A, xv, y0h, gs = blas_in
        t0 = time.perf_counter()
        want = S.gemv_blas(np.float32(1.3), A, xv, np.float32(-2.1), y0h, to_plan(gs))
        el = time.perf_counter() - t0
        _line(workload="scal", op="gemv_blas", cpu_baseline={"kind": "oracle", "cores": 1,
                                                             "sample": "8192^2, one call",
                                                             "seconds": round(el, 2)},
              parity={"bit_exact": bool(np.array_equal(
                  blas_out["y := 1.3 A x - 2.1 y"].view(np.uint32),
                  np.asarray(want, np.float32).view(np.uint32)))})
    if not args.no_cpu_baseline:
        from oracle import strategies as S
        m = 1 << 22                                  # a 4 Mi-element prefix: ~1 s of oracle work
        t0 = time.perf_counter()
        want = S.scal(alpha, x[:m])
        el = time.perf_counter() - t0
        got = yt[:m].cpu().numpy()
        _line(workload="scal", cpu_baseline={"kind": "oracle", "cores": 1, "sample": f"first {m} elements",
                                             "gbs": _gbs(8 * m, el * 1e6)},
              parity={"bit_exact_prefix": bool(np.array_equal(got.view(np.uint32),
                                                              np.asarray(want, np.float32).view(np.uint32)))})


VECTOR_STRATEGIES = [
    ("sec6.2", dp.Strategy(seq_len=2048, local_size=64, order=dp.CONTIGUOUS, wg_combine=dp.NONE,
                           vec_width=4)),
    ("contig-v4-tree", dp.Strategy(seq_len=64, local_size=256, order=dp.CONTIGUOUS,
                                   wg_combine=dp.TREE, vec_width=4)),
    ("strided-v4-tree", dp.Strategy(seq_len=64, local_size=256, order=dp.STRIDED,
                                    wg_combine=dp.TREE, vec_width=4)),
    ("strided-v4-tree-c256", dp.Strategy(seq_len=256, local_size=256, order=dp.STRIDED,
                                         wg_combine=dp.TREE, vec_width=4)),
    ("scalar-headline", DOT_STRATEGY),
]


def workload_vector(args):
    import torch
    import synthetic
    from paper_1710_08332_amd.autotune import time_us
    n = N_DOT
    x, y = synthetic.dot_inputs(n, SEED)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    res = {}
    for name, s in VECTOR_STRATEGIES:
        s = s.with_(passes=2)
        cbuf = torch.empty(dp.num_chunks(s, n) * dp.values_per_chunk(s) * 4, dtype=torch.uint8,
                           device="cuda")
        out = torch.empty(1, device="cuda")
        c_us = time_us(lambda: dp.chunks(dp.OP_DOT, s, xt, yt, out=cbuf), reps=40)[0]
        f_us = time_us(lambda: dp.fold(dp.OP_DOT, s, cbuf, n, dp.F32, out=out), reps=40)[0]
        ws = dp.workspace(s, dp.OP_DOT, dp.F32, 0, n)
        t_us = time_us(lambda: dp.dot(xt, yt, s, out=out, ws=ws), reps=40)[0]
        torch.cuda.synchronize()
        res[name] = (s, out.cpu().numpy()[0])
        # the same strategy in one pass (one launch; with many chunk values
        # the fold runs beside the chunk values still being computed)
        s1 = s.with_(passes=1)
        ws1 = dp.workspace(s1, dp.OP_DOT, dp.F32, 0, n)
        out1 = torch.empty(1, device="cuda")
        t1_us = time_us(lambda: dp.dot(xt, yt, s1, out=out1, ws=ws1), reps=40)[0]
        torch.cuda.synchronize()
        res[name + " 1-pass"] = (s1, out1.cpu().numpy()[0])
        nval = dp.num_chunks(s, n) * dp.values_per_chunk(s)
        _line(workload="vector", name=name, n=n, strategy=strategy_text(s), chunk_values=nval,
              chunks_us=round(c_us, 2), fold_us=round(f_us, 2), dot_us=round(t_us, 2),
              chunks_gbs=_gbs(8 * n + 4 * nval, c_us),
              chunks_pct_peak=round(100 * (8 * n + 4 * nval) / c_us / 1e3 / PEAK_GBPS, 1),
              dot_gbs=_gbs(8 * n + 4, t_us), dot_1pass_us=round(t1_us, 2),
              dot_1pass_gbs=_gbs(8 * n + 4, t1_us))
    if not args.no_cpu_baseline:
        from oracle import strategies as S
        from tests.gpu_util import to_plan
        parity = {}
        t0 = time.perf_counter()
        for name, (s, got) in res.items():
            want = np.float32(S.dot(x, y, to_plan(s)))
            parity[name] = bool(want.view(np.uint32) == np.float32(got).view(np.uint32))
        el = time.perf_counter() - t0
        _line(workload="vector", cpu_baseline={"kind": "oracle", "cores": 1,
                                               "seconds_all_strategies": round(el, 2)},
              parity_bit_exact=parity)


def workload_generated(args):
    import torch
    import synthetic
    from paper_1710_08332_amd.autotune import time_us
    from paper_1710_08332_amd.generator import catalog, runtime
    x, y = synthetic.dot_inputs(N_DOT, SEED)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    A, xv = synthetic.gemv_inputs(M_GEMV, K_GEMV, SEED)
    At, xvt = torch.from_numpy(A).cuda(), torch.from_numpy(xv).cuda()
    gd = runtime.Generated(catalog.path("dot_headline_2p26"))
    gg = runtime.Generated(catalog.path("gemv_headline_8192"))
    dout, gout = gd.outputs(), gg.outputs()
    ws = dp.workspace(DOT_STRATEGY, dp.OP_DOT, dp.F32, 0, N_DOT)
    out = torch.empty(1, device="cuda")
    yg = torch.empty(M_GEMV, device="cuda")
    rows = [
        ("dot", "generated", lambda: gd.run({"xs": xt, "ys": yt}, dout), DOT_BYTES),
        ("dot", "library", lambda: dp.dot(xt, yt, DOT_STRATEGY, out=out, ws=ws), DOT_BYTES),
        ("gemv", "generated", lambda: gg.run({"A": At, "x": xvt}, gout), GEMV_BYTES),
        ("gemv", "library", lambda: dp.gemv(At, xvt, GEMV_STRATEGY, y=yg), GEMV_BYTES),
    ]
    # low-precision gemv 16384 x 16384, C=16 L=1024 strided tree, 2 rows per work-group
    big = dp.Strategy(seq_len=16, local_size=1024, order=dp.STRIDED, wg_combine=dp.TREE,
                      rows_per_wg=2)
    A16, xv16 = synthetic.gemv_inputs(16384, 16384, synthetic.SEEDS["precision"])
    xv16t = torch.from_numpy(xv16).cuda()
    c16 = torch.from_numpy(synthetic.quantise_bf16(A16).view(np.int16)).cuda()
    c8n, sc8n = synthetic.quantise_fp8_rows(A16)
    c8, sc8 = torch.from_numpy(c8n).cuda(), torch.from_numpy(sc8n).cuda()
    del A16
    gb, gf = (runtime.Generated(catalog.path("gemv_bf16_16384")),
              runtime.Generated(catalog.path("gemv_fp8_16384")))
    bout, fout = gb.outputs(), gf.outputs()
    yb, yf = torch.empty(16384, device="cuda"), torch.empty(16384, device="cuda")
    nb16 = 2 * 16384 * 16384 + 8 * 16384
    nb8 = 16384 * 16384 + 12 * 16384
    rows += [
        ("gemv_bf16_16384", "generated", lambda: gb.run({"A": c16, "x": xv16t}, bout), nb16),
        ("gemv_bf16_16384", "library",
         lambda: dp.gemv(c16, xv16t, big, y=yb, a_dtype=dp.BF16), nb16),
        ("gemv_fp8_16384", "generated",
         lambda: gf.run({"A": c8, "x": xv16t, "scale": sc8}, fout), nb8),
        ("gemv_fp8_16384", "library",
         lambda: dp.gemv(c8, xv16t, big, y=yf, row_scale=sc8, a_dtype=dp.FP8_E4M3), nb8),
    ]
    for op, kind, fn, nbytes in rows:
        med, p10, p90 = time_us(fn, reps=30)
        _line(workload="generated", op=op, kind=kind, us=round(med, 2), p10=round(p10, 2),
              p90=round(p90, 2), gbs=_gbs(nbytes, med),
              pct_peak=round(100 * nbytes / med / 1e3 / PEAK_GBPS, 1))
    torch.cuda.synchronize()
    same_dot = bool(dout["out"].cpu().numpy()[:1].view(np.uint32)[0]
                    == out.cpu().numpy().view(np.uint32)[0])
    same_gemv = bool(np.array_equal(gout["out"].cpu().numpy().view(np.uint32),
                                    yg.cpu().numpy().view(np.uint32)))
    same_lp = {name: bool(np.array_equal(a["out"].cpu().numpy().view(np.uint32),
                                         b.cpu().numpy().view(np.uint32)))
               for name, a, b in (("gemv_bf16", bout, yb), ("gemv_fp8", fout, yf))}
    _line(workload="generated", generated_equals_library_bitwise=dict(
        dot=same_dot, gemv=same_gemv, **same_lp))
    for g in (gd, gg, gb, gf):
        g.close()


KERNEL_CASES = (
    # (name, format, m = k, strategy)
    ("gemv_f32_8192", "f32", 8192, GEMV_STRATEGY),
    ("gemv_f32_16384_C32_L512", "f32", 16384,
     dp.Strategy(seq_len=32, local_size=512, order=dp.STRIDED, wg_combine=dp.TREE)),
    ("gemv_f32_16384_C64_L256_R4", "f32", 16384,
     dp.Strategy(seq_len=64, local_size=256, order=dp.STRIDED, wg_combine=dp.TREE, rows_per_wg=4)),
    ("gemv_f32_16384_C16_L1024", "f32", 16384,
     dp.Strategy(seq_len=16, local_size=1024, order=dp.STRIDED, wg_combine=dp.TREE)),
    ("gemv_bf16_16384_C32_L512", "bf16", 16384,
     dp.Strategy(seq_len=32, local_size=512, order=dp.STRIDED, wg_combine=dp.TREE)),
    ("gemv_fp8_16384_C64_L256", "fp8", 16384,
     dp.Strategy(seq_len=64, local_size=256, order=dp.STRIDED, wg_combine=dp.TREE)),
)


def workload_kernels(args):
    """Each hot kernel of the headline and precision configurations, launched
    ``--steps`` times with the last-level cache evicted before every launch:
    the dot (2^26, headline strategy, one kernel), the gemvs above, and the
    read-stream ceiling on each matrix's bytes.  A small, fixed kernel mix for
    rocprofv3 counter runs; each line gives the evicted median."""
    import torch
    import synthetic
    from paper_1710_08332_amd.autotune import cache_evictor, time_us
    evict = cache_evictor()
    reps = max(3, args.steps)
    x, y = synthetic.dot_inputs(N_DOT, SEED)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    out = torch.empty(1, device="cuda")
    ws = dp.workspace(DOT_STRATEGY, dp.OP_DOT, dp.F32, 0, N_DOT)
    med = time_us(lambda: dp.dot(xt, yt, DOT_STRATEGY, out=out, ws=ws), reps=reps,
                  between=evict)[0]
    _line(workload="kernels", op="dot_2p26", strategy=strategy_text(DOT_STRATEGY),
          us=round(med, 2), gbs=_gbs(DOT_KERNEL_BYTES, med),
          pct_peak=round(100 * DOT_KERNEL_BYTES / med / 1e3 / PEAK_GBPS, 1))
    del xt, yt
    mats = {}
    for name, fmt, mk, s in KERNEL_CASES:
        if (fmt, mk) not in mats:
            A, xv = synthetic.gemv_inputs(mk, mk, synthetic.SEEDS["precision"])
            if fmt == "bf16":
                At, sc = torch.from_numpy(synthetic.quantise_bf16(A).view(np.int16)).cuda(), None
            elif fmt == "fp8":
                codes, scale = synthetic.quantise_fp8_rows(A)
                At, sc = torch.from_numpy(codes).cuda(), torch.from_numpy(scale).cuda()
            else:
                At, sc = torch.from_numpy(A).cuda(), None
            mats = {(fmt, mk): (At, sc, torch.from_numpy(xv).cuda())}
        At, sc, xvt = mats[(fmt, mk)]
        dt = {"f32": dp.F32, "bf16": dp.BF16, "fp8": dp.FP8_E4M3}[fmt]
        yv = torch.empty(mk, device="cuda")
        med = time_us(lambda: dp.gemv(At, xvt, s, y=yv, row_scale=sc, a_dtype=dt), reps=reps,
                      between=evict)[0]
        a_bytes = At.numel() * At.element_size()
        nbytes = a_bytes + 4 * mk + 4 * mk + (4 * mk if sc is not None else 0)
        ceil_us, grid = evicted_read_ceiling(At, evict, reps=reps)
        _line(workload="kernels", op=name, strategy=strategy_text(s, gemv=True), us=round(med, 2),
              gbs=_gbs(nbytes, med), pct_peak=round(100 * nbytes / med / 1e3 / PEAK_GBPS, 1),
              read_ceiling_us=round(ceil_us, 2), read_ceiling_grid=grid,
              pct_of_read_ceiling=round(100 * (nbytes / med) / (a_bytes / ceil_us), 1))


def read_ceiling(dev, nbytes):
    """The measured read-stream ceiling: the best bandwidth of the plain read
    kernel (every byte loaded once, 16-byte non-temporal loads) over a few
    grid sizes, on a buffer as large as the dot's inputs, timed as the dot's
    kernel is (graph_us)."""
    import torch
    buf = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    sink = torch.empty(cus * 16, dtype=torch.int32, device=dev)
    best = None
    for per_cu in (1, 2, 4, 8, 16):
        grid = cus * per_cu
        us = graph_us(lambda: dp.read_stream(buf, grid, sink=sink))
        if best is None or us < best[0]:
            best = (us, grid)
    del buf
    return {"kernel": "read_stream_kernel<8> (16-byte non-temporal loads, XOR of every word)",
            "bytes_per_launch": nbytes, "gbs": round(nbytes / best[0] / 1e3, 3),
            "avg_kernel_us": round(best[0], 3), "grid": best[1]}


def graph_steps(dot, gemv, steps, outputs):
    """K steps captured in one HIP graph, replayed once untimed (the graph's
    upload), then once timed: host clock around the replay, synchronized on
    both sides.  The dot and the gemv of a step read and write disjoint
    buffers, so the graph holds them as two branches: the K dots in order on
    one stream and the K gemvs in order (``gemv(j)`` for step j) on a second
    one, forked at the start and joined at the end; the dot's tail (its last
    work-group folding the chunk values) and each launch's ramp run beside the
    other branch's loads.  The ``outputs`` are compared bit for bit with their
    eager values after each replay.  Returns (seconds for the K steps, equal)."""
    import torch
    eager = [o.clone() for o in outputs]
    main = torch.cuda.Stream()
    branch = torch.cuda.Stream()
    main.wait_stream(torch.cuda.current_stream())
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.stream(main):
        dot()
        gemv(0)
        torch.cuda.synchronize()
        with torch.cuda.graph(gr, stream=main):
            branch.wait_stream(main)
            for _ in range(steps):
                dot()
            with torch.cuda.stream(branch):
                for j in range(steps):
                    gemv(j)
            main.wait_stream(branch)
    torch.cuda.current_stream().wait_stream(main)
    torch.cuda.synchronize()
    same = True
    for timed in (False, True):
        for o in outputs:
            o.fill_(0)                  # eager work between replays
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gr.replay()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        same &= all(torch.equal(o.view(torch.int32), e.view(torch.int32))
                    for o, e in zip(outputs, eager))
    del gr
    return el, bool(same)


def graph_us(launch, count=20, replays=5):
    """A kernel's average duration: ``count`` back-to-back launches captured
    in one HIP graph, one untimed replay, then ``replays`` replays each
    bracketed by events on torch's current stream (the replay's stream).
    Median replay / count: the GPU-side gaps between the launches are
    included, the host's launch latency is not."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        launch()
        torch.cuda.synchronize()
        with torch.cuda.graph(gr, stream=side):
            for _ in range(count):
                launch()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    gr.replay()
    torch.cuda.synchronize()
    ev = TimingEvents(replays)
    for i in range(replays):
        ev.record(i, 0)
        gr.replay()
        ev.record(i, 1)
        torch.cuda.synchronize()
    per = sorted(ev.elapsed_ms(i) * 1e3 / count for i in range(replays))
    ev.close()
    del gr
    return per[len(per) // 2]


def evicted_read_ceiling(t, evict, reps=20):
    """(median µs, grid) of the best grid of the read-stream kernel over the
    bytes of device tensor t, with ``evict`` run before every timed call."""
    import torch
    from paper_1710_08332_amd.autotune import time_us
    cus = torch.cuda.get_device_properties(t.device).multi_processor_count
    sink = torch.empty(cus * 16, dtype=torch.int32, device=t.device)
    return min((time_us(lambda: dp.read_stream(t, g, sink=sink), reps=reps, between=evict)[0], g)
               for g in (cus, 2 * cus, 4 * cus, 8 * cus, 16 * cus))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="scale",
                    choices=["scale", "small", "sweep", "precision", "batch", "scal", "vector",
                             "generated", "kernels"])
    ap.add_argument("--profile-copy", action="store_true",
                    help="also launch one plain 256 MiB device-to-device copy (a kernel of "
                         "known traffic, to calibrate hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synthetic

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload != "scale":
        {"small": workload_small, "sweep": workload_sweep, "precision": workload_precision,
         "batch": workload_batch, "scal": workload_scal,
         "vector": workload_vector, "generated": workload_generated,
         "kernels": workload_kernels}[args.workload](args)
        return
    from paper_1710_08332_amd.autotune import cache_evictor, time_us
    dev = torch.device("cuda:0")
    x, y = synthetic.dot_inputs(N_DOT, SEED)
    A, xv = synthetic.gemv_inputs(M_GEMV, K_GEMV, SEED)
    xt, yt = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    # A_COPIES copies of A, read in turn: between two reads of one copy the
    # step streams the dot's 512 MiB and the other copies' 512 MiB, so the
    # gemv never finds its matrix in the 256 MB last-level cache
    Ats = [torch.from_numpy(A).to(dev) for _ in range(A_COPIES)]
    xvt = torch.from_numpy(xv).to(dev)
    out = torch.empty(1, dtype=torch.float32, device=dev)
    yg = torch.empty(M_GEMV, dtype=torch.float32, device=dev)
    ws_dot = dp.workspace(DOT_STRATEGY, dp.OP_DOT, dp.F32, 0, N_DOT, dev)

    # one step: the dot (one kernel: chunk values, then their ordered fold in
    # the last work-group) and the gemv, on torch's current stream; `first`
    # optionally times the dot alone (roofline), `parts` each part of the step
    def step(i, first=None, parts=None):
        if first is not None:
            first.record(i, 0)
        if parts is not None:
            parts[0].record(i, 0)
        dp.dot(xt, yt, DOT_STRATEGY, out=out, ws=ws_dot)
        if first is not None:
            first.record(i, 1)
        if parts is not None:
            parts[0].record(i, 1)
            parts[1].record(i, 0)
        dp.gemv(Ats[i % A_COPIES], xvt, GEMV_STRATEGY, y=yg)
        if parts is not None:
            parts[1].record(i, 1)

    if args.profile_copy:
        src = torch.empty(1 << 26, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)            # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        del src, dst

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    # K eager steps back to back, only the dot bracketed (the roofline's
    # kernel time; the eager figure beside the headline)
    timer = TimingEvents(args.steps)
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i, first=timer)
    torch.cuda.synchronize()
    el_eager = time.perf_counter() - t0
    dot_ms = [timer.elapsed_ms(i) for i in range(args.steps)]
    dot_avg_s = float(np.mean(dot_ms)) / 1e3
    timer_kind = timer.kind
    timer.close()

    # the same steps again, each part of the step bracketed (not the headline:
    # the extra events add their own small gaps)
    parts = (TimingEvents(args.steps), TimingEvents(args.steps))
    for i in range(args.steps):
        step(i, parts=parts)
    torch.cuda.synchronize()
    dot_e2e_us = float(np.median([parts[0].elapsed_ms(i) for i in range(args.steps)])) * 1e3
    gemv_step_us = float(np.median([parts[1].elapsed_ms(i) for i in range(args.steps)])) * 1e3
    for t in parts:
        t.close()
    # the gemv alone with the last-level cache evicted before every call
    evict = cache_evictor()
    gemv_cold_us = time_us(lambda: dp.gemv(Ats[0], xvt, GEMV_STRATEGY, y=yg), reps=20,
                           between=evict)[0]
    del evict

    # the headline: the same K steps replayed from one HIP graph (no host
    # launch between kernels), the dots and the gemvs on two branches
    el, graph_same = graph_steps(lambda: dp.dot(xt, yt, DOT_STRATEGY, out=out, ws=ws_dot),
                                 lambda j: dp.gemv(Ats[j % A_COPIES], xvt, GEMV_STRATEGY, y=yg),
                                 args.steps, [out, yg])
    if not graph_same:
        print("bench.py: the graph-replayed step's outputs differ from the eager step's",
              file=sys.stderr)
        sys.exit(1)
    total_bytes = (DOT_BYTES + GEMV_BYTES) * args.steps
    value = total_bytes / el / 1e9
    value_eager = total_bytes / el_eager / 1e9
    # the roofline's kernel time: back-to-back dots replayed from a graph
    dot_kernel_us = graph_us(lambda: dp.dot(xt, yt, DOT_STRATEGY, out=out, ws=ws_dot))
    achieved = DOT_KERNEL_BYTES / dot_kernel_us / 1e3
    ceiling = read_ceiling(dev, 2 * N_DOT * 4)
    ceiling["frac"] = round(achieved / ceiling["gbs"], 4)
    rec = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "FP32 dot N=2^26 + FP32 gemv 8192x8192 (one step = one of each; the "
                        f"gemv reads {A_COPIES} copies of A in turn, none cache-resident)",
            "dot_strategy": strategy_text(DOT_STRATEGY),
            "gemv_strategy": strategy_text(GEMV_STRATEGY, gemv=True),
            "percent_of_hbm_peak": round(100 * value / PEAK_GBPS, 2),
            "parallelism": "single GPU",
        },
        "step_parts": {
            "dot_end_to_end": {"us": round(dot_e2e_us, 2), "bytes": DOT_BYTES,
                               "gbs": _gbs(DOT_BYTES, dot_e2e_us),
                               "frac": round(DOT_BYTES / dot_e2e_us / 1e3 / PEAK_GBPS, 4),
                               "what": "the whole dot: chunk values and their ordered fold"},
            "gemv_in_step": {"us": round(gemv_step_us, 2), "bytes": GEMV_BYTES,
                             "gbs": _gbs(GEMV_BYTES, gemv_step_us),
                             "frac": round(GEMV_BYTES / gemv_step_us / 1e3 / PEAK_GBPS, 4)},
            "gemv_cache_evicted": {"us": round(gemv_cold_us, 2), "bytes": GEMV_BYTES,
                                   "gbs": _gbs(GEMV_BYTES, gemv_cold_us),
                                   "frac": round(GEMV_BYTES / gemv_cold_us / 1e3 / PEAK_GBPS, 4),
                                   "what": "the gemv alone, 512 MiB written before every call"},
            "timed_with": timer_kind + " (medians)",
        },
        "timed_as": f"the {args.steps} steps captured in one HIP graph and replayed once "
                    "(host clock around the replay; one untimed replay before it): the dots "
                    "in order on one branch, the gemvs in order on a second, joined at the "
                    "end; outputs equal to the eager step's after each replay",
        "graph_outputs_bit_exact_vs_eager": graph_same,
        "eager": {"value": round(value_eager, 3), "ms_per_step": round(el_eager / args.steps * 1e3, 4),
                  "percent_of_hbm_peak": round(100 * value_eager / PEAK_GBPS, 2),
                  "what": "the same steps launched one by one from the host"},
        "roofline": {
            "bound": "hbm",
            "kernel": "reduce_kernel<DotF32, strided, 4, tree> (the whole dot, 1 pass)",
            "bytes_per_launch": DOT_KERNEL_BYTES,
            "achieved": round(achieved, 3),
            "peak": PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_GBPS, 4),
            "traffic": measured_traffic(),
            "avg_kernel_us": round(dot_kernel_us, 3),
            "timed_with": timer_kind + " around replays of 20 back-to-back dots captured in "
                          "one HIP graph (median replay / 20; the gaps between launches included)",
            "per_launch_events_us": round(dot_avg_s * 1e6, 3),
            "read_ceiling": ceiling,
        },
    }
    if not args.no_cpu_baseline:
        torch.cuda.synchronize()
        base, parity = cpu_baseline(x, y, A, xv, out.cpu().numpy()[0], yg.cpu().numpy())
        rec["cpu_baseline"] = base
        rec["parity"] = parity
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
