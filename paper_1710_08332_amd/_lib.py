"""ctypes declarations of the C ABI in include/dpia.h (libdpia.so).

Loading fails loudly: there is no fallback implementation of any entry point.
"""

from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdpia.so")

ABI_VERSION = 2

# dpia_status
OK, ERR_NULL, ERR_SHAPE, ERR_STRATEGY, ERR_DTYPE, ERR_WORKSPACE, ERR_HIP, ERR_ABI = range(8)
# dpia_dtype
F32, F64, I32, BF16, FP8_E4M3 = range(5)
# dpia_op
OP_DOT, OP_ASUM, OP_GEMV, OP_SCAL = range(4)
# dpia_order, dpia_combine, dpia_accum
CONTIGUOUS, STRIDED = 0, 1
TREE, SEQ, NONE = 0, 1, 2
PLAIN, KAHAN, SUM2 = 0, 1, 2

EXPORTS = ("dpia_strategy_check", "dpia_dot", "dpia_dot_noalloc", "dpia_asum", "dpia_gemv",
           "dpia_gemv_blas", "dpia_scal", "dpia_chunks", "dpia_module_load", "dpia_module_launch",
           "dpia_module_unload", "dpia_read_stream",
           "dpia_fold", "dpia_batch_plan_create", "dpia_batch_workspace_bytes",
           "dpia_batch_upload", "dpia_batch_run", "dpia_batch_run_one_launch",
           "dpia_batch_plan_destroy", "dpia_status_str",
           "dpia_last_error_detail", "dpia_abi_version")


class CStrategy(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint32) for name in (
        "abi_version", "seq_len", "local_size", "order", "wg_combine", "passes", "accum",
        "final_f64", "rows_per_wg", "row_parts", "max_grid", "vec_width")]


class CInstance(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint32), ("dtype", ctypes.c_uint32), ("strategy", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("a", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("out", ctypes.c_void_p)]


class DpiaError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {status_str(status)} ({detail})")


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1710_08332_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        i64, u64, vp = ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p
        sp = ctypes.POINTER(CStrategy)
        L.dpia_strategy_check.argtypes = [sp, ctypes.c_int, ctypes.c_int, i64, i64,
                                          ctypes.POINTER(u64)]
        L.dpia_dot.argtypes = [sp, ctypes.c_int, i64, vp, vp, vp, ctypes.c_int, vp, u64, vp]
        L.dpia_dot_noalloc.argtypes = [sp, ctypes.c_int, i64, vp, vp, vp, ctypes.c_int, vp]
        L.dpia_asum.argtypes = [sp, ctypes.c_int, i64, vp, vp, ctypes.c_int, vp, u64, vp]
        L.dpia_gemv.argtypes = [sp, ctypes.c_int, i64, i64, i64, vp, vp, vp, vp, vp, u64, vp]
        L.dpia_scal.argtypes = [sp, ctypes.c_int, i64, ctypes.c_float, vp, vp, vp]
        L.dpia_module_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
        L.dpia_module_launch.argtypes = [vp, ctypes.c_char_p, ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.POINTER(vp), ctypes.c_int32, vp]
        L.dpia_module_unload.argtypes = [vp]
        L.dpia_read_stream.argtypes = [vp, i64, ctypes.c_int32, vp, vp]
        L.dpia_gemv_blas.argtypes = [sp, ctypes.c_int, i64, i64, i64, ctypes.c_float, vp, vp, vp,
                                     ctypes.c_float, vp, vp]
        L.dpia_chunks.argtypes = [sp, ctypes.c_int, ctypes.c_int, i64, vp, vp, vp, u64, vp]
        L.dpia_fold.argtypes = [sp, ctypes.c_int, ctypes.c_int, i64, vp, vp, ctypes.c_int, vp]
        pp = ctypes.POINTER(ctypes.c_void_p)
        L.dpia_batch_plan_create.argtypes = [ctypes.POINTER(CInstance), ctypes.c_int32, sp,
                                             ctypes.c_int32, pp]
        L.dpia_batch_workspace_bytes.argtypes = [vp]
        L.dpia_batch_workspace_bytes.restype = u64
        L.dpia_batch_upload.argtypes = [vp, vp, u64, vp]
        L.dpia_batch_run.argtypes = [vp, vp, u64, vp]
        L.dpia_batch_run_one_launch.argtypes = [vp, vp, u64, vp]
        L.dpia_batch_plan_destroy.argtypes = [vp]
        L.dpia_batch_plan_destroy.restype = None
        for f in ("dpia_strategy_check", "dpia_dot", "dpia_dot_noalloc", "dpia_asum",
                  "dpia_gemv", "dpia_gemv_blas", "dpia_scal", "dpia_chunks", "dpia_fold", "dpia_batch_plan_create",
                  "dpia_batch_upload", "dpia_batch_run", "dpia_batch_run_one_launch",
                  "dpia_module_load",
                  "dpia_module_launch", "dpia_module_unload", "dpia_read_stream"):
            getattr(L, f).restype = ctypes.c_int
        L.dpia_status_str.argtypes = [ctypes.c_int]
        L.dpia_status_str.restype = ctypes.c_char_p
        L.dpia_last_error_detail.argtypes = []
        L.dpia_last_error_detail.restype = ctypes.c_char_p
        L.dpia_abi_version.argtypes = []
        L.dpia_abi_version.restype = ctypes.c_uint32
        if L.dpia_abi_version() != ABI_VERSION:
            raise ImportError("libdpia.so ABI version mismatch")
        _lib = L
    return _lib


def status_str(st: int) -> str:
    return lib().dpia_status_str(st).decode()


def last_error_detail() -> str:
    return lib().dpia_last_error_detail().decode()


def check(st: int, where: str):
    if st != OK:
        raise DpiaError(st, where, last_error_detail())
