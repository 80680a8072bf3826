"""The oracle's expressions evaluated with their outermost map split over
host cores.

TEST INFRASTRUCTURE ONLY, like the rest of this package: it is used by the
tests and by the CPU-baseline leg of the benchmark, never by the library.

Stage II of the translation (Sec. 4.2) gives every map the meaning of a
parallel loop whose iterations are independent, and the hierarchy variants
of Sec. 6.1 (mapWorkgroup, mapGlobal) mean the same.  So the mapWorkgroup
level of a dot or asum strategy (one iteration per chunk of W elements) and
the map over gemv rows may be evaluated for disjoint, consecutive ranges of
iterations at the same time, each range by the same expression over its own
slice of the input.  The chunk values (or rows of y) are joined in iteration
order, and a dot's or asum's outer reduceSeq then runs once, sequentially,
over all of them, exactly as in the whole expression.  The result is
therefore the same, bit for bit, as strategies.dot / asum / gemv; only the
host cores that evaluate the map differ.

The ranges run in worker processes (the evaluator interprets the
expression in Python between numpy array operations, so threads would
queue on the interpreter lock).  The inputs are placed once in shared
memory, and the pool is kept for as many evaluations as the caller makes.
"""

from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor
from multiprocessing import shared_memory
from typing import Dict, List, Tuple

import numpy as np

from . import strategies as S
from .eval_numpy import evaluate


def host_cores(cap: int = 15) -> int:
    """Cores this process may run on (its affinity mask), at most ``cap``."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def ranges(items: int, unit: int, parts: int) -> List[Tuple[int, int]]:
    """Iterations [0, items) in at most ``parts`` consecutive ranges whose
    bounds are multiples of ``unit`` (the last one ends at ``items``)."""
    units = -(-items // unit)
    per = -(-units // max(1, parts))
    return [(u * unit, min(items, (u + per) * unit)) for u in range(0, units, per)]


def fold(values: np.ndarray, plan: S.Plan):
    """The outer reduceSeq of the strategy over the joined chunk values."""
    return evaluate(S._final("p", plan), {"p": values}, "f32")


# ------------------------------------------------------------ worker side
_ARRAYS: Dict[str, np.ndarray] = {}
_SHM: List[shared_memory.SharedMemory] = []


def _attach(specs):
    for name, (shm_name, shape, dtype) in specs.items():
        shm = shared_memory.SharedMemory(name=shm_name)
        _SHM.append(shm)
        _ARRAYS[name] = np.ndarray(shape, np.dtype(dtype), buffer=shm.buf)


def _chunk_values_of(task):
    op, plan, a, b, xs, ys = task
    if op == "dot":
        return np.asarray(evaluate(S.dot_chunks_expr(b - a, plan),
                                   {"xs": _ARRAYS[xs][a:b], "ys": _ARRAYS[ys][a:b]}, "f32"))
    expr = S._partials(b - a, S._vectors("xs", plan), plan, S.ABS_ADD)
    return np.asarray(evaluate(expr, {"xs": _ARRAYS[xs][a:b]}, "f32"))


def _rows_of(task):
    plan, a, b, A, x = task
    return np.asarray(S.gemv(_ARRAYS[A][a:b], _ARRAYS[x], plan))


# ------------------------------------------------------------ caller side
class Evaluator:
    """A pool of ``workers`` processes holding the named host arrays.

    Arrays for dot / asum must already be zero-extended to a multiple of the
    strategy's chunk (strategies.extended_length).  Use as a context manager,
    or call close()."""

    def __init__(self, arrays: Dict[str, np.ndarray], workers: int = None):
        self.workers = workers or host_cores()
        self._shm = []
        specs = {}
        for name, arr in arrays.items():
            arr = np.ascontiguousarray(arr)
            shm = shared_memory.SharedMemory(create=True, size=max(1, arr.nbytes))
            np.ndarray(arr.shape, arr.dtype, buffer=shm.buf)[...] = arr
            self._shm.append(shm)
            specs[name] = (shm.name, arr.shape, arr.dtype.str)
        self.shapes = {name: arr.shape for name, arr in arrays.items()}
        self._pool = ProcessPoolExecutor(max_workers=self.workers,
                                         mp_context=mp.get_context("spawn"),
                                         initializer=_attach, initargs=(specs,))
        # start every worker now, so that no evaluation pays for it
        list(self._pool.map(abs, range(self.workers)))

    def _reduction(self, op, plan: S.Plan, xs: str, ys: str = None):
        if plan.accum != "plain":
            raise ValueError("the parallel evaluation covers plain accumulation")
        n = self.shapes[xs][0]
        if n % plan.chunk:
            raise ValueError("the inputs must be zero-extended to a multiple of the chunk")
        tasks = [(op, plan, a, b, xs, ys) for a, b in ranges(n, plan.chunk, self.workers)]
        parts = list(self._pool.map(_chunk_values_of, tasks))
        return fold(np.concatenate(parts), plan)

    def dot(self, plan: S.Plan, xs: str = "xs", ys: str = "ys"):
        return self._reduction("dot", plan, xs, ys)

    def asum(self, plan: S.Plan, xs: str = "xs"):
        return self._reduction("asum", plan, xs)

    def gemv(self, plan: S.Plan, A: str = "A", x: str = "x"):
        m = self.shapes[A][0]
        tasks = [(plan, a, b, A, x) for a, b in ranges(m, plan.rows, self.workers)]
        return np.concatenate(list(self._pool.map(_rows_of, tasks)))

    def close(self):
        if self._pool is not None:
            self._pool.shutdown(wait=True)
            self._pool = None
        for shm in self._shm:
            shm.close()
            shm.unlink()
        self._shm = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
