"""Strategy enumeration and autotuning.

The paper's premise is that a strategy is chosen by exploring semantically
equivalent expressions (Sec. 1; the stochastic search of Steuwer et al. 2015
that it builds on).  Here the space is the strategy descriptor: every
candidate is a valid DPIA strategy for the problem, each gives its own
(fixed) rounding, and the tuner times them on the device and keeps the
fastest per operation, element type and size class.  The bits each candidate
produces are checked against the CPU oracle by the test suite, not here: this
module only measures.

Cache: a JSON file (``DPIA_TUNE_CACHE``, default ``~/.cache/dpia/tune.json``)
mapping "device|runtime|op|dtype|shape" to the chosen descriptor, where device
is the GPU's name and architecture (``device_name``) and runtime the HIP
version and the library's ABI version (``runtime_tag``).
"""

from __future__ import annotations

import dataclasses
import json
import os
import statistics
from typing import Callable, Dict, List, Sequence, Tuple

from . import (CONTIGUOUS, F32, OP_ASUM, OP_DOT, OP_GEMV, STRIDED, TREE, Strategy,
               strategy_check)
from ._lib import DpiaError

SEQ_LENS = (64, 128, 256, 512, 1024, 8192)
ORDERS = (CONTIGUOUS, STRIDED)


def sweep_dot(n: int, local_size: int = 256) -> List[Strategy]:
    """The 24 dot / asum strategies of the sweep: C in SEQ_LENS x {contiguous,
    strided} x {1 pass, 2 passes}, L lanes, tree combine; candidates whose
    chunk does not divide n are dropped."""
    out = []
    for C in SEQ_LENS:
        for order in ORDERS:
            for passes in (1, 2):
                s = Strategy(seq_len=C, local_size=local_size, order=order, wg_combine=TREE,
                             passes=passes)
                if n % (C * local_size) == 0:
                    out.append(s)
    return out


def sweep_gemv(m: int, k: int, max_lanes: int = 256) -> List[Strategy]:
    """The 24 gemv strategies: C in SEQ_LENS x {contiguous, strided} x {1, 2
    row parts}; L = min(max_lanes, k / (C * parts)) lanes per row part, tree
    combine, R = max(1, 256 / team threads) rows per work-group (whole rows
    of y per work-group; R never changes a result)."""
    out = []
    for C in SEQ_LENS:
        for order in ORDERS:
            for parts in (1, 2):
                if k % (C * parts):
                    continue
                L = min(max_lanes, k // (C * parts))
                if L < 1 or C * L * parts != k or (L & (L - 1)):
                    continue
                team = L // 4 if order == STRIDED and L % 4 == 0 else L
                R = max(1, 256 // max(1, team))
                while m % R:
                    R //= 2
                s = Strategy(seq_len=C, local_size=L, order=order, wg_combine=TREE,
                             rows_per_wg=R, row_parts=parts)
                out.append(s)
    return out


def cache_evictor(device=None, mib: int = 512):
    """A callable that reads ``mib`` MiB of scratch memory: more than the
    MI355X's 256 MB last-level (Infinity) cache, so inputs timed after it
    come from HBM.  It reads rather than writes, so no dirty lines are left
    to be written back while the timed kernel runs."""
    import torch
    buf = torch.zeros(mib << 18, dtype=torch.float32, device=device or "cuda")
    return lambda: buf.sum()


def valid(s: Strategy, op: int, dtype: int, m: int, n: int) -> bool:
    try:
        strategy_check(s, op, dtype, m, n)
        return True
    except DpiaError:
        return False


def time_us(fn: Callable[[], object], reps: int = 20, warmup: int = 3,
            between: Callable[[], object] = None) -> Tuple[float, float, float]:
    """(median, p10, p90) in microseconds of ``fn`` on torch's current stream,
    with timing-only HIP events around each call (see ``timing``).
    ``between`` (untimed) runs before every timed call, e.g. to evict the
    last-level cache."""
    import torch
    from .timing import TimingEvents
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = TimingEvents(reps)
    for i in range(reps):
        if between is not None:
            between()
        ev.record(i, 0)
        fn()
        ev.record(i, 1)
    torch.cuda.synchronize()
    ts = sorted(ev.elapsed_ms(i) * 1e3 for i in range(reps))
    ev.close()
    q = statistics.quantiles(ts, n=10) if len(ts) >= 2 else [ts[0]] * 9
    return statistics.median(ts), q[0], q[-1]


def tune(candidates: Sequence[Strategy], run: Callable[[Strategy], Callable[[], object]],
         reps: int = 20) -> Tuple[Strategy, List[Dict]]:
    """Times ``run(s)`` for every candidate; returns the fastest and the table."""
    table = []
    for s in candidates:
        med, p10, p90 = time_us(run(s), reps=reps)
        table.append({"strategy": dataclasses.asdict(s), "us": med, "p10": p10, "p90": p90})
    best = min(range(len(table)), key=lambda i: table[i]["us"])
    return candidates[best], table


# ------------------------------------------------------------ cache

def cache_path() -> str:
    return os.environ.get("DPIA_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "dpia", "tune.json"))


def runtime_tag() -> str:
    """The software a tuned choice was measured with: the HIP runtime torch
    was built against and the library's ABI version."""
    try:
        import torch
        hip = torch.version.hip or "none"
    except ImportError:
        hip = "none"
    from ._lib import ABI_VERSION
    return f"hip-{hip}|dpia-abi-{ABI_VERSION}"


def device_name(device=None) -> str:
    """Name and architecture of a GPU (e.g. 'AMD Instinct MI355X gfx950')."""
    import torch
    p = torch.cuda.get_device_properties(device if device is not None else 0)
    return f"{p.name} {getattr(p, 'gcnArchName', '')}".strip()


def _key(device: str, op: int, dtype: int, shape: Tuple[int, ...]) -> str:
    # a choice is only reused on the same device under the same software
    return f"{device}|{runtime_tag()}|{op}|{dtype}|{'x'.join(str(v) for v in shape)}"


def load_cache() -> Dict[str, Dict]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def store(device: str, op: int, dtype: int, shape: Tuple[int, ...], s: Strategy) -> None:
    c = load_cache()
    c[_key(device, op, dtype, shape)] = dataclasses.asdict(s)
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(device: str, op: int, dtype: int, shape: Tuple[int, ...]):
    d = load_cache().get(_key(device, op, dtype, shape))
    return Strategy(**d) if d else None


# ------------------------------------------------------------ convenience

def tune_dot(x, y, candidates=None, reps: int = 20, op: int = OP_DOT):
    """Tunes a dot (or asum, op=OP_ASUM, y ignored) on the given device tensors."""
    from . import asum, dot, workspace
    n = x.numel()
    cands = [s for s in (candidates or sweep_dot(n)) if valid(s, op, F32, 0, n)]
    out = __import__("torch").empty(1, device=x.device)

    def run(s):
        ws = workspace(s, op, F32, 0, n, x.device)
        if op == OP_ASUM:
            return lambda: asum(x, s, out=out, ws=ws)
        return lambda: dot(x, y, s, out=out, ws=ws)
    return tune(cands, run, reps)


def tune_gemv(A, x, candidates=None, reps: int = 20, a_dtype: int = None):
    from . import gemv
    m, k = A.shape
    dt = F32 if a_dtype is None else a_dtype
    cands = [s for s in (candidates or sweep_gemv(m, k)) if valid(s, OP_GEMV, dt, m, k)]
    y = __import__("torch").empty(m, device=A.device)

    def run(s):
        return lambda: gemv(A, x, s, y=y, a_dtype=a_dtype)
    return tune(cands, run, reps)


# ------------------------------------------------------------ batched

def size_class(inst) -> Tuple[str, int]:
    """Reductions are classed by floor(log2 n), gemvs by floor(log2 k)."""
    import math
    if inst["op"] == OP_GEMV:
        return ("gemv", int(math.floor(math.log2(max(1, inst["A"].shape[1])))))
    return ("red", int(math.floor(math.log2(max(1, inst["x"].numel())))))


def batch_candidates(cls: Tuple[str, int]) -> List[Strategy]:
    """Batch-eligible strategies (16-byte loads, threads per chunk dividing
    256) for a size class."""
    kind, c = cls
    out = []
    if kind == "red":
        for L in (64, 256, 1024):
            for C in (4, 16, 64, 256):
                if C * L <= 4 * (2 ** (c + 1)):        # at most 4x zero extension
                    out.append(Strategy(seq_len=C, local_size=L, order=STRIDED, wg_combine=TREE))
        if not out:
            out.append(Strategy(seq_len=4, local_size=64, order=STRIDED, wg_combine=TREE))
    else:
        kmax = 2 ** (c + 1)                           # every k of the class fits
        for L in (16, 64, 256):
            C = max(1, -(-kmax // L))
            out.append(Strategy(seq_len=C, local_size=L, order=STRIDED, wg_combine=TREE))
    return out


def tune_batch(instances, reps: int = 5):
    """Picks a strategy per size class by timing batched runs of that class's
    instances under each candidate.  Returns (strategies, assignment) where
    assignment[i] indexes strategies for instance i, and the timing table."""
    from . import BatchPlan
    classes: Dict[Tuple[str, int], List[int]] = {}
    for i, d in enumerate(instances):
        classes.setdefault(size_class(d), []).append(i)
    strategies: List[Strategy] = []
    assignment = [0] * len(instances)
    table = []
    for cls in sorted(classes):
        members = classes[cls]
        sub = [dict(instances[i], strategy=0) for i in members]
        best, best_us = None, float("inf")
        for cand in batch_candidates(cls):
            plan = BatchPlan(sub, [cand])
            ws = plan.workspace()
            plan.upload(ws)
            med, _, _ = time_us(lambda: plan.run(ws), reps=reps, warmup=1)
            table.append({"class": f"{cls[0]}:{cls[1]}", "members": len(members),
                          "strategy": dataclasses.asdict(cand), "us": med})
            plan.close()
            if med < best_us:
                best, best_us = cand, med
        if best not in strategies:
            strategies.append(best)
        for i in members:
            assignment[i] = strategies.index(best)
    return strategies, assignment, table
