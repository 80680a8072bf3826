"""Throughput of the strategy-preserving dot + gemv on one MI355X.

One step = one FP32 dot product of N = 2^26 (x, y uniform in [-1, 1]) and
one FP32 gemv y = A x with A 8192 x 8192 row-major, entries N(0, 1), x
uniform in [-1, 1] (seed 1712), each under a fixed DPIA strategy.  Inputs are
resident in HBM before timing starts.  Value = algorithmic bytes of the step
(every input element read once, results written once) x steps / wall time,
in GB/s.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

Prints one JSON line.  Besides the whole-job figure it reports the dominant
kernel (the dot) against the HBM roofline, timed with HIP events on the
stream the kernels run on, and the CPU oracle timed on this host's cores on
the same workload (bounded to a few repetitions).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

import paper_1710_08332_amd as dp

METRIC = "HBM GB/s (% of peak) for dot/asum/gemv per strategy; batched vs plain"
PEAK_GBPS = 8000.0   # MI355X HBM3E, published

N_DOT = 1 << 26
M_GEMV = K_GEMV = 8192
SEED = 1712

# split 262144 -> mapWorkgroup (1024 lanes, each folding a strided row of 256
# -> mapLocal reduceSeq) -> tree in local memory; then reduceSeq over the 256
# chunk values in a second pass
DOT_STRATEGY = dp.Strategy(seq_len=256, local_size=1024, order=dp.STRIDED, wg_combine=dp.TREE,
                           passes=2)
# rows of 8192 = 256 lanes x 32 strided elements, tree, 4 rows per work-group
GEMV_STRATEGY = dp.Strategy(seq_len=32, local_size=256, order=dp.STRIDED, wg_combine=dp.TREE,
                            rows_per_wg=4)

DOT_BYTES = 2 * 4 * N_DOT + 4                    # x, y read; one result written
G_DOT = N_DOT // (DOT_STRATEGY.seq_len * DOT_STRATEGY.local_size)
CHUNK_KERNEL_BYTES = 2 * 4 * N_DOT + 4 * G_DOT   # first pass: x, y read; G values written
GEMV_BYTES = 4 * M_GEMV * K_GEMV + 4 * K_GEMV + 4 * M_GEMV


def strategy_text(s: dp.Strategy, gemv: bool = False) -> str:
    return (f"C={s.seq_len} L={s.local_size} {'strided' if s.order == dp.STRIDED else 'contiguous'}"
            f" {'tree' if s.wg_combine == dp.TREE else 'seq'}"
            + (f" R={s.rows_per_wg}" if gemv else f" passes={s.passes}"))


def cpu_baseline(x, y, A, xv, gpu_dot_val, gpu_y, budget_s=12.0):
    """The oracle (numpy, one thread) on the same step, repeated until about
    ``budget_s`` seconds have passed; also confirms bit parity of the
    measured GPU results."""
    from oracle import strategies as S
    from tests.gpu_util import to_plan
    dplan, gplan = to_plan(DOT_STRATEGY), to_plan(GEMV_STRATEGY)
    reps, t0 = 0, time.perf_counter()
    while True:
        d = S.dot(x, y, dplan)
        g = S.gemv(A, xv, gplan)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 100:
            break
    parity = {
        "dot_bit_exact": bool(np.asarray(d).view(np.uint32) == np.float32(gpu_dot_val).view(np.uint32)),
        "gemv_bit_exact": bool(np.array_equal(np.asarray(g).view(np.uint32), gpu_y.view(np.uint32))),
    }
    value = (DOT_BYTES + GEMV_BYTES) * reps / el / 1e9
    return {"value": round(value, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"the full step (dot 2^26 + gemv 8192^2, same strategies) x {reps} "
                      f"repetitions, {el:.1f} s, numpy single thread"}, parity


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-copy", action="store_true",
                    help="also launch one plain 256 MiB device-to-device copy (a kernel of "
                         "known traffic, to calibrate hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synthetic

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    x, y = synthetic.dot_inputs(N_DOT, SEED)
    A, xv = synthetic.gemv_inputs(M_GEMV, K_GEMV, SEED)
    xt, yt = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    At, xvt = torch.from_numpy(A).to(dev), torch.from_numpy(xv).to(dev)
    out = torch.empty(1, dtype=torch.float32, device=dev)
    yg = torch.empty(M_GEMV, dtype=torch.float32, device=dev)
    chunk_vals = torch.empty(G_DOT * 4, dtype=torch.uint8, device=dev)

    # one step: the dot's two passes (chunk values, then their ordered fold)
    # and the gemv, all on torch's current stream
    def step(ev=None):
        if ev is not None:
            ev[0].record()
        dp.chunks(dp.OP_DOT, DOT_STRATEGY, xt, yt, out=chunk_vals)
        if ev is not None:
            ev[1].record()
        dp.fold(dp.OP_DOT, DOT_STRATEGY, chunk_vals, N_DOT, dp.F32, out=out)
        dp.gemv(At, xvt, GEMV_STRATEGY, y=yg)

    if args.profile_copy:
        src = torch.empty(1 << 26, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)            # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    dot_ms = [a.elapsed_time(b) for a, b in evs]
    dot_avg_s = float(np.mean(dot_ms)) / 1e3

    total_bytes = (DOT_BYTES + GEMV_BYTES) * args.steps
    value = total_bytes / el / 1e9
    achieved = CHUNK_KERNEL_BYTES / dot_avg_s / 1e9
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
            "workload": "FP32 dot N=2^26 + FP32 gemv 8192x8192 (one step = one of each)",
            "dot_strategy": strategy_text(DOT_STRATEGY),
            "gemv_strategy": strategy_text(GEMV_STRATEGY, gemv=True),
            "percent_of_hbm_peak": round(100 * value / PEAK_GBPS, 2),
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "reduce_kernel<DotF32, strided, 4, tree> (dot first pass)",
            "bytes_per_launch": CHUNK_KERNEL_BYTES,
            "achieved": round(achieved, 3),
            "peak": PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_GBPS, 4),
            "traffic": None,
            "avg_kernel_us": round(dot_avg_s * 1e6, 3),
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
