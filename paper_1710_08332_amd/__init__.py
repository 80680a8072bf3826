"""MI355X strategy-preserving dot / asum / gemv (DPIA strategies on gfx950).

Thin Python binding of include/dpia.h: argument marshalling only.  Every
step of the computation runs in the HIP kernels of libdpia.so; PyTorch
supplies device memory and the current stream.  See the header for the
semantics of a strategy and of each entry point.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass, replace

from . import _lib
from ._lib import (BF16, CONTIGUOUS, F32, F64, FP8_E4M3, I32, KAHAN, NONE, OP_ASUM,  # noqa: F401
                   OP_DOT, OP_GEMV, OP_SCAL, PLAIN, SEQ, STRIDED, SUM2, TREE, DpiaError,
                   last_error_detail)


@dataclass(frozen=True)
class Strategy:
    """Mirror of dpia_strategy (include/dpia.h)."""
    seq_len: int                  # C: elements folded sequentially per lane
    local_size: int               # L: lanes per chunk
    order: int = CONTIGUOUS       # CONTIGUOUS | STRIDED
    wg_combine: int = TREE        # TREE | SEQ
    passes: int = 2               # 1 | 2
    accum: int = PLAIN            # PLAIN | KAHAN | SUM2
    final_f64: int = 0
    rows_per_wg: int = 1
    row_parts: int = 1
    max_grid: int = 0
    vec_width: int = 1            # V: dot / asum over asVector V views (1: scalar)

    def c(self) -> _lib.CStrategy:
        return _lib.CStrategy(_lib.ABI_VERSION, self.seq_len, self.local_size, self.order,
                              self.wg_combine, self.passes, self.accum, self.final_f64,
                              self.rows_per_wg, self.row_parts, self.max_grid, self.vec_width)

    def with_(self, **kw) -> "Strategy":
        return replace(self, **kw)


def strategy_check(s: Strategy, op: int, dtype: int, m: int, n: int) -> int:
    """Validates ``s`` for the problem; returns the workspace size in bytes."""
    cs = s.c()
    ws = ctypes.c_size_t(0)
    _lib.check(_lib.lib().dpia_strategy_check(ctypes.byref(cs), op, dtype, m, n,
                                              ctypes.byref(ws)), "dpia_strategy_check")
    return ws.value


# ------------------------------------------------------------ torch glue

def _torch():
    import torch
    return torch


_DT = {}


def _dtype_code(t) -> int:
    torch = _torch()
    if not _DT:
        _DT.update({torch.float32: F32, torch.float64: F64, torch.int32: I32,
                    torch.uint32: I32, torch.bfloat16: BF16, torch.uint16: BF16,
                    torch.float8_e4m3fn: FP8_E4M3, torch.uint8: FP8_E4M3})
    if t.dtype not in _DT:
        raise TypeError(f"unsupported tensor dtype {t.dtype}")
    return _DT[t.dtype]


def _dev(t):
    if not t.is_cuda:
        raise ValueError("tensors must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def workspace(s: Strategy, op: int, dtype: int, m: int, n: int, device="cuda"):
    """A zeroed workspace tensor of the size the strategy needs (or None)."""
    nbytes = strategy_check(s, op, dtype, m, n)
    if nbytes == 0:
        return None
    return _torch().zeros(nbytes, dtype=_torch().uint8, device=device)


def _ws(ws):
    if ws is None:
        return ctypes.c_void_p(0), 0
    return _dev(ws), ws.numel() * ws.element_size()


def dot(x, y, s: Strategy, out=None, ws=None, out_dtype=None, stream=None):
    torch = _torch()
    dt = _dtype_code(x)
    if _dtype_code(y) != dt:
        raise TypeError("x and y must have the same dtype")
    n = x.numel()
    if out is None:
        od = out_dtype or (torch.float64 if (s.accum != PLAIN and s.final_f64) else x.dtype)
        out = torch.empty(1, dtype=od, device=x.device)
    if ws is None:
        ws = workspace(s, OP_DOT, dt, 0, n, x.device)
    cs = s.c()
    w, wb = _ws(ws)
    _lib.check(_lib.lib().dpia_dot(ctypes.byref(cs), dt, n, _dev(x), _dev(y), _dev(out),
                                   _dtype_code(out), w, wb, _stream(stream)), "dpia_dot")
    return out


def dot_noalloc(x, y, s: Strategy, out, stream=None):
    """dpia_dot_noalloc: the dot with the library's own per-device scratch in
    place of a workspace (no allocation in the call; ``out`` is required)."""
    dt = _dtype_code(x)
    if _dtype_code(y) != dt:
        raise TypeError("x and y must have the same dtype")
    cs = s.c()
    _lib.check(_lib.lib().dpia_dot_noalloc(ctypes.byref(cs), dt, x.numel(), _dev(x), _dev(y),
                                           _dev(out), _dtype_code(out), _stream(stream)),
               "dpia_dot_noalloc")
    return out


def asum(x, s: Strategy, out=None, ws=None, stream=None):
    torch = _torch()
    n = x.numel()
    if out is None:
        out = torch.empty(1, dtype=torch.float32, device=x.device)
    if ws is None:
        ws = workspace(s, OP_ASUM, F32, 0, n, x.device)
    cs = s.c()
    w, wb = _ws(ws)
    _lib.check(_lib.lib().dpia_asum(ctypes.byref(cs), _dtype_code(x), n, _dev(x), _dev(out),
                                    _dtype_code(out), w, wb, _stream(stream)), "dpia_asum")
    return out


def gemv(A, x, s: Strategy, y=None, row_scale=None, a_dtype=None, stream=None):
    """y = A x.  ``A`` is a 2-D row-major tensor (float32, bfloat16 / uint16
    codes, float8_e4m3fn / uint8 codes, or int32); ``a_dtype`` overrides the
    element type read from A's dtype."""
    torch = _torch()
    m, k = A.shape
    adt = a_dtype if a_dtype is not None else _dtype_code(A)
    lda = A.stride(0)
    if A.stride(1) != 1:
        raise ValueError("A must be row-major")
    if y is None:
        y = torch.empty(m, dtype=torch.int32 if adt == I32 else torch.float32, device=A.device)
    cs = s.c()
    sc = _dev(row_scale) if row_scale is not None else ctypes.c_void_p(0)
    _lib.check(_lib.lib().dpia_gemv(ctypes.byref(cs), adt, m, k, lda,
                                    ctypes.c_void_p(A.data_ptr()), sc, _dev(x), _dev(y),
                                    ctypes.c_void_p(0), 0, _stream(stream)), "dpia_gemv")
    return y


def gemv_blas(alpha: float, A, x, beta: float, y, s: Strategy, row_scale=None, a_dtype=None,
              stream=None):
    """y := alpha * (A x) + beta * y in place (y is not read when beta == 0).
    ``A`` as for ``gemv`` (float32, bf16 or fp8 codes)."""
    m, k = A.shape
    adt = a_dtype if a_dtype is not None else _dtype_code(A)
    if A.stride(1) != 1:
        raise ValueError("A must be row-major")
    cs = s.c()
    sc = _dev(row_scale) if row_scale is not None else ctypes.c_void_p(0)
    _lib.check(_lib.lib().dpia_gemv_blas(ctypes.byref(cs), adt, m, k, A.stride(0), float(alpha),
                                         ctypes.c_void_p(A.data_ptr()), sc, _dev(x), float(beta),
                                         _dev(y), _stream(stream)), "dpia_gemv_blas")
    return y


def scal(alpha: float, x, s: Strategy, y=None, stream=None):
    """y = alpha * x (y may be x: in place)."""
    if y is None:
        y = _torch().empty_like(x)
    cs = s.c()
    _lib.check(_lib.lib().dpia_scal(ctypes.byref(cs), _dtype_code(x), x.numel(), float(alpha),
                                    _dev(x), _dev(y), _stream(stream)), "dpia_scal")
    return y


def read_stream(x, grid: int, sink=None, stream=None):
    """Reads every byte of the device tensor x once (the read-bandwidth
    ceiling kernel) with ``grid`` work-groups; work-group b stores the XOR of
    the 32-bit words it read in sink[b] (``grid`` int32 values on the
    device).  Returns sink."""
    if sink is None:
        sink = _torch().empty(grid, dtype=_torch().int32, device=x.device)
    if sink.numel() < grid:
        raise ValueError("sink needs one int32 per work-group")
    _lib.check(_lib.lib().dpia_read_stream(_dev(x), x.numel() * x.element_size(), int(grid),
                                           _dev(sink), _stream(stream)), "dpia_read_stream")
    return sink


def num_chunks(s: Strategy, n: int) -> int:
    """G: chunks of a length-n dot / asum (the last one may be partial)."""
    w = s.seq_len * s.local_size * max(1, s.vec_width)
    return -(-n // w)


def values_per_chunk(s: Strategy) -> int:
    """Chunk values per chunk: the vector width, times L when uncombined."""
    return max(1, s.vec_width) * (s.local_size if s.wg_combine == NONE else 1)


def chunks(op: int, s: Strategy, x, y=None, out=None, stream=None):
    """The mapWorkgroup level of a dot (op=OP_DOT) or asum (OP_ASUM): the
    chunks' values (``values_per_chunk`` each; 4 bytes, or 8 for a Kahan
    pair)."""
    torch = _torch()
    n = x.numel()
    dt = _dtype_code(x)
    vb = 8 if s.accum != PLAIN else 4
    if out is None:
        out = torch.empty(max(1, num_chunks(s, n) * values_per_chunk(s)) * vb, dtype=torch.uint8,
                          device=x.device)
    cs = s.c()
    yp = _dev(y) if y is not None else ctypes.c_void_p(0)
    _lib.check(_lib.lib().dpia_chunks(ctypes.byref(cs), op, dt, n, _dev(x), yp, _dev(out),
                                      out.numel() * out.element_size(), _stream(stream)),
               "dpia_chunks")
    return out


def fold(op: int, s: Strategy, chunk_values, n: int, dtype: int, out=None, out_dtype=None,
         stream=None):
    """The outer reduceSeq of the strategy over chunk values from ``chunks``."""
    torch = _torch()
    if out is None:
        od = out_dtype or (torch.float64 if (s.accum != PLAIN and s.final_f64) else
                           (torch.int32 if dtype == I32 else torch.float32))
        out = torch.empty(1, dtype=od, device=chunk_values.device)
    cs = s.c()
    _lib.check(_lib.lib().dpia_fold(ctypes.byref(cs), op, dtype, n, _dev(chunk_values),
                                    _dev(out), _dtype_code(out), _stream(stream)), "dpia_fold")
    return out


# ------------------------------------------------------------ batched

class BatchPlan:
    """Many dot / asum / gemv instances, each with its own strategy, run by
    one of two engines (see dpia_batch_* in include/dpia.h).

    ``instances``: list of dicts with keys ``op`` (OP_DOT / OP_ASUM /
    OP_GEMV), ``strategy`` (index into ``strategies``), and tensors ``x``,
    ``y`` (dot), ``A``, ``x`` (gemv), ``out`` (a 1-element float32 tensor for
    dot / asum, the m-element y for gemv).  The tensors must stay alive while
    the plan is used.
    """

    def __init__(self, instances, strategies):
        L = _lib.lib()
        n = len(instances)
        arr = (_lib.CInstance * max(1, n))()
        for i, d in enumerate(instances):
            c = arr[i]
            c.op, c.dtype, c.strategy, c.reserved = d["op"], F32, d["strategy"], 0
            if d["op"] == OP_GEMV:
                A = d["A"]
                if A.stride(1) != 1:
                    raise ValueError("A must be row-major")
                c.m, c.n, c.lda = A.shape[0], A.shape[1], A.stride(0)
                c.a, c.b = A.data_ptr(), _dev(d["x"]).value
            else:
                c.m, c.n, c.lda = 0, d["x"].numel(), 0
                c.a = _dev(d["x"]).value
                c.b = _dev(d["y"]).value if d["op"] == OP_DOT else None
            c.out = _dev(d["out"]).value
        cs = (_lib.CStrategy * max(1, len(strategies)))(*[s.c() for s in strategies])
        h = ctypes.c_void_p(0)
        _lib.check(L.dpia_batch_plan_create(arr, n, cs, len(strategies), ctypes.byref(h)),
                   "dpia_batch_plan_create")
        self._h = h
        self._uploaded = False
        self.workspace_bytes = L.dpia_batch_workspace_bytes(h)

    def workspace(self, device="cuda"):
        return _torch().zeros(max(256, self.workspace_bytes), dtype=_torch().uint8, device=device)

    def upload(self, ws, stream=None):
        _lib.check(_lib.lib().dpia_batch_upload(self._h, _dev(ws), ws.numel(), _stream(stream)),
                   "dpia_batch_upload")
        self._uploaded = True

    def run(self, ws, stream=None, one_launch=False):
        """Runs every instance: two launches (dpia_batch_run), or one
        persistent launch with per-instance arrival counters
        (dpia_batch_run_one_launch); the same bits either way."""
        f = _lib.lib().dpia_batch_run_one_launch if one_launch else _lib.lib().dpia_batch_run
        _lib.check(f(self._h, _dev(ws), ws.numel(), _stream(stream)),
                   "dpia_batch_run_one_launch" if one_launch else "dpia_batch_run")

    def close(self):
        if self._h:
            if self._uploaded:
                _torch().cuda.synchronize()   # the upload copies from the plan's tables
            _lib.lib().dpia_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
