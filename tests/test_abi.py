"""C-ABI checks that need no GPU: the library loads, exports every function
include/dpia.h declares, and validates descriptors and arguments before any
launch (so these calls never reach HIP)."""

import ctypes
import os
import re

import pytest

import paper_1710_08332_amd as dp
from paper_1710_08332_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# fake, 256-byte aligned device addresses: validation must reject the call
# before anything dereferences them
P = ctypes.c_void_p(0x7000_0000)
P2 = ctypes.c_void_p(0x7100_0000)


def header_functions():
    text = open(os.path.join(ROOT, "include", "dpia.h")).read()
    # declarations: a return type at the start of a line, then the name
    return sorted(set(re.findall(r"^(?:const\s+)?\w+\s*\**\s*(dpia_[a-z0-9_]+)\s*\(",
                                 text, re.M)))


def test_library_exports_every_declared_function():
    L = _lib.lib()
    names = header_functions()
    assert set(names) == set(_lib.EXPORTS)
    for name in names:
        assert hasattr(L, name), name
    assert L.dpia_abi_version() == _lib.ABI_VERSION


def test_descriptor_layout_matches_header():
    text = open(os.path.join(ROOT, "include", "dpia.h")).read()
    body = re.search(r"typedef struct \{(.*?)\} dpia_strategy;", text, re.S).group(1)
    fields = re.findall(r"uint32_t\s+(\w+);", body)
    assert fields == [f for f, _ in _lib.CStrategy._fields_]
    assert ctypes.sizeof(_lib.CStrategy) == 4 * len(fields)


def check(s, op, dt, m, n):
    cs = s.c() if isinstance(s, dp.Strategy) else s
    ws = ctypes.c_size_t(0)
    st = _lib.lib().dpia_strategy_check(ctypes.byref(cs), op, dt, m, n, ctypes.byref(ws))
    return st, ws.value


BASE = dp.Strategy(seq_len=256, local_size=16)


def test_ragged_lengths_are_zero_extended():
    # plain strategies accept any n (G = ceil(n / W)) and gemv rows up to W
    st, ws = check(BASE, dp.OP_DOT, dp.F32, 0, (1 << 20) + 1)
    assert st == _lib.OK and ws == 257 * 4 + 256 + (256 - 257 * 4 % 256) % 256
    assert check(BASE, dp.OP_GEMV, dp.F32, 10, 4000)[0] == _lib.OK
    assert check(BASE.with_(row_parts=2), dp.OP_GEMV, dp.F32, 10, 4097)[0] == _lib.OK


def test_vector_and_uncombined_workspace():
    # a chunk of V*L*C elements gives V values, or L*V uncombined
    s = dp.Strategy(seq_len=2048, local_size=64, vec_width=4, wg_combine=dp.NONE)
    st, ws = check(s, dp.OP_DOT, dp.F32, 0, 1 << 26)
    assert st == _lib.OK and ws == 128 * 64 * 4 * 4 + 256
    assert dp.num_chunks(s, 1 << 26) == 128 and dp.values_per_chunk(s) == 256
    st, ws = check(s.with_(wg_combine=dp.TREE), dp.OP_ASUM, dp.F32, 0, (1 << 26) + 1)
    assert st == _lib.OK and ws == 256 + 4 * 129 * 4 + (256 - 4 * 129 * 4 % 256) % 256 * 1
    st, ws = check(dp.Strategy(seq_len=64, local_size=1, wg_combine=dp.NONE), dp.OP_DOT, dp.I32,
                   0, 640)
    assert st == _lib.OK and ws == 256 + 256


def test_valid_strategy_reports_workspace():
    st, ws = check(BASE, dp.OP_DOT, dp.F32, 0, 1 << 20)
    assert st == _lib.OK
    # 256 chunk results of 4 bytes, then one 256-byte counter section
    assert ws == 256 * 4 + 256
    st, ws = check(BASE.with_(accum=dp.KAHAN), dp.OP_DOT, dp.F32, 0, 1 << 20)
    assert st == _lib.OK and ws == 2048 + 256
    st, ws = check(dp.Strategy(seq_len=64, local_size=128, order=dp.STRIDED, rows_per_wg=2),
                   dp.OP_GEMV, dp.BF16, 8192, 8192)
    assert st == _lib.OK and ws == 0


@pytest.mark.parametrize("s,op,dt,m,n,want", [
    (BASE.with_(accum=dp.KAHAN), dp.OP_DOT, dp.F32, 0, (1 << 20) + 5, _lib.ERR_SHAPE),  # n % W, Kahan
    (BASE.with_(local_size=12), dp.OP_DOT, dp.F32, 0, 12 * 256, _lib.ERR_STRATEGY),  # tree, L not 2^k
    (BASE.with_(seq_len=0), dp.OP_DOT, dp.F32, 0, 4096, _lib.ERR_STRATEGY),
    (BASE.with_(passes=3), dp.OP_DOT, dp.F32, 0, 4096, _lib.ERR_STRATEGY),
    (BASE.with_(order=2), dp.OP_DOT, dp.F32, 0, 4096, _lib.ERR_STRATEGY),
    (BASE.with_(final_f64=1), dp.OP_DOT, dp.F32, 0, 4096, _lib.ERR_STRATEGY),  # needs Kahan
    (BASE.with_(accum=dp.KAHAN), dp.OP_ASUM, dp.F32, 0, 4096, _lib.ERR_STRATEGY),
    (BASE.with_(accum=dp.KAHAN), dp.OP_DOT, dp.I32, 0, 4096, _lib.ERR_DTYPE),
    (BASE, dp.OP_DOT, dp.BF16, 0, 4096, _lib.ERR_DTYPE),
    (BASE, dp.OP_ASUM, dp.I32, 0, 4096, _lib.ERR_DTYPE),
    (BASE.with_(rows_per_wg=2), dp.OP_DOT, dp.F32, 0, 4096, _lib.ERR_STRATEGY),
    (BASE.with_(local_size=2048, seq_len=1, wg_combine=dp.SEQ), dp.OP_DOT, dp.F32, 0, 2048,
     _lib.ERR_STRATEGY),   # 2048 contiguous lanes > 1024 threads
    (BASE, dp.OP_GEMV, dp.F32, 10, 4097, _lib.ERR_SHAPE),           # k > L*C
    (BASE.with_(rows_per_wg=3), dp.OP_GEMV, dp.F32, 10, 4096, _lib.ERR_SHAPE),  # m % R
    (BASE.with_(rows_per_wg=0), dp.OP_GEMV, dp.F32, 10, 4096, _lib.ERR_STRATEGY),
    (BASE.with_(row_parts=3), dp.OP_GEMV, dp.F32, 10, 4096, _lib.ERR_STRATEGY),
    (BASE, dp.OP_DOT, dp.F32, 0, -4096, _lib.ERR_SHAPE),
    (BASE.with_(vec_width=3), dp.OP_DOT, dp.F32, 0, 4096, _lib.ERR_STRATEGY),
    (BASE.with_(vec_width=8), dp.OP_DOT, dp.F32, 0, 1 << 15, _lib.ERR_STRATEGY),
    (BASE.with_(vec_width=4), dp.OP_GEMV, dp.F32, 16, 1024, _lib.ERR_STRATEGY),
    (BASE.with_(wg_combine=dp.NONE), dp.OP_GEMV, dp.F32, 16, 1024, _lib.ERR_STRATEGY),
    (BASE.with_(vec_width=4, accum=dp.KAHAN), dp.OP_DOT, dp.F32, 0, 1 << 14, _lib.ERR_STRATEGY),
    (BASE.with_(wg_combine=3), dp.OP_DOT, dp.F32, 0, 4096, _lib.ERR_STRATEGY),
])
def test_invalid_descriptors_are_rejected(s, op, dt, m, n, want):
    st, _ = check(s, op, dt, m, n)
    assert st == want, (st, _lib.last_error_detail())
    assert _lib.last_error_detail() != ""


def test_abi_version_mismatch_and_null_descriptor():
    cs = BASE.c()
    cs.abi_version = 99
    assert check(cs, dp.OP_DOT, dp.F32, 0, 4096)[0] == _lib.ERR_ABI
    ws = ctypes.c_size_t(0)
    assert _lib.lib().dpia_strategy_check(None, dp.OP_DOT, dp.F32, 0, 4096,
                                          ctypes.byref(ws)) == _lib.ERR_NULL


def test_status_strings():
    for st in range(8):
        assert _lib.status_str(st)
    assert _lib.status_str(0) == "ok"


def _dot(s, n, x=P, y=P, out=P2, out_dt=dp.F32, ws=P2, wsb=1 << 20, dt=dp.F32):
    cs = s.c()
    return _lib.lib().dpia_dot(ctypes.byref(cs), dt, n, x, y, out, out_dt, ws, wsb, None)


def test_entry_points_validate_before_launching():
    n = 1 << 20
    assert _dot(BASE.with_(accum=dp.KAHAN), n + 1) == _lib.ERR_SHAPE
    assert _dot(BASE, n, out=ctypes.c_void_p(0)) == _lib.ERR_NULL
    assert _dot(BASE, n, x=ctypes.c_void_p(0)) == _lib.ERR_NULL
    assert _dot(BASE, n, x=ctypes.c_void_p(0x7000_0004)) == _lib.ERR_SHAPE   # misaligned
    assert _dot(BASE, n, wsb=100) == _lib.ERR_WORKSPACE
    assert _dot(BASE, n, ws=ctypes.c_void_p(0)) == _lib.ERR_WORKSPACE
    assert _dot(BASE, n, ws=ctypes.c_void_p(0x7100_0010)) == _lib.ERR_SHAPE  # ws alignment
    assert _dot(BASE, n, out_dt=dp.F64) == _lib.ERR_DTYPE
    assert _dot(BASE, n, dt=dp.I32, out_dt=dp.F32) == _lib.ERR_DTYPE
    cs = BASE.c()
    L = _lib.lib()
    assert L.dpia_asum(ctypes.byref(cs), dp.F32, n, P, P2, dp.F64, P2, 1 << 20, None) == _lib.ERR_DTYPE
    gs = dp.Strategy(seq_len=64, local_size=64).c()
    # FP8 without row scales; scales with a non-FP8 matrix; lda < k
    assert L.dpia_gemv(ctypes.byref(gs), dp.FP8_E4M3, 64, 4096, 4096, P, None, P, P2, None, 0,
                       None) == _lib.ERR_NULL
    assert L.dpia_gemv(ctypes.byref(gs), dp.F32, 64, 4096, 4096, P, P, P, P2, None, 0,
                       None) == _lib.ERR_DTYPE
    assert L.dpia_gemv(ctypes.byref(gs), dp.F32, 64, 4096, 4095, P, None, P, P2, None, 0,
                       None) == _lib.ERR_SHAPE
    # m = 0 is a valid empty problem: nothing is launched
    assert L.dpia_gemv(ctypes.byref(gs), dp.F32, 0, 4096, 4096, P, None, P, P2, None, 0,
                       None) == _lib.OK


def _dot_noalloc(s, n, x=P, y=P, out=P2, out_dt=dp.F32, dt=dp.F32):
    cs = s.c()
    return _lib.lib().dpia_dot_noalloc(ctypes.byref(cs), dt, n, x, y, out, out_dt, None)


def test_noalloc_dot_validates_before_any_hip_call():
    n = 1 << 20
    assert _dot_noalloc(BASE.with_(accum=dp.KAHAN), n + 1) == _lib.ERR_SHAPE
    assert _dot_noalloc(BASE, n, out=ctypes.c_void_p(0)) == _lib.ERR_NULL
    assert _dot_noalloc(BASE, n, y=ctypes.c_void_p(0)) == _lib.ERR_NULL
    assert _dot_noalloc(BASE, n, y=ctypes.c_void_p(0x7000_0008)) == _lib.ERR_SHAPE
    assert _dot_noalloc(BASE, n, out_dt=dp.F64) == _lib.ERR_DTYPE
    assert _dot_noalloc(BASE, n, dt=dp.BF16) == _lib.ERR_DTYPE
    # chunk values beyond the 1 MiB scratch (less its 256-byte counter
    # section): 2^18 - 64 binary32 values fit, 2^18 do not
    one = dp.Strategy(seq_len=1, local_size=1, wg_combine=dp.NONE)
    assert _dot_noalloc(one, 1 << 18) == _lib.ERR_WORKSPACE
    assert "scratch" in _lib.last_error_detail()
    kahan = dp.Strategy(seq_len=1, local_size=1, accum=dp.KAHAN)
    assert _dot_noalloc(kahan, 1 << 17) == _lib.ERR_WORKSPACE   # 8-byte pairs


def test_python_strategy_check_raises_with_detail():
    with pytest.raises(dp.DpiaError) as ei:
        dp.strategy_check(BASE.with_(accum=dp.KAHAN), dp.OP_DOT, dp.F32, 0, 1000)
    assert "multiple of the chunk" in str(ei.value)


def test_stage_entry_points_validate_before_launching():
    L = _lib.lib()
    cs = BASE.c()
    n = 1 << 20                      # G = 256 chunk values of 4 bytes
    assert L.dpia_chunks(ctypes.byref(cs), dp.OP_DOT, dp.F32, n, P, P, P2, 1023, None) == _lib.ERR_WORKSPACE
    assert L.dpia_chunks(ctypes.byref(cs), dp.OP_DOT, dp.F32, n, P, None, P2, 1024, None) == _lib.ERR_NULL
    assert L.dpia_chunks(ctypes.byref(cs), dp.OP_GEMV, dp.F32, n, P, P, P2, 1024, None) == _lib.ERR_STRATEGY
    assert L.dpia_chunks(ctypes.byref(cs), dp.OP_DOT, dp.F32, -1, P, P, P2, 1 << 20, None) == _lib.ERR_SHAPE
    ks = BASE.with_(accum=dp.KAHAN).c()
    assert L.dpia_chunks(ctypes.byref(ks), dp.OP_DOT, dp.F32, n, P, P, P2, 2047, None) == _lib.ERR_WORKSPACE
    assert L.dpia_fold(ctypes.byref(cs), dp.OP_DOT, dp.F32, n, P, P2, dp.F64, None) == _lib.ERR_DTYPE
    assert L.dpia_fold(ctypes.byref(cs), dp.OP_DOT, dp.F32, n, None, P2, dp.F32, None) == _lib.ERR_NULL
    assert L.dpia_fold(ctypes.byref(cs), dp.OP_ASUM, dp.I32, n, P, P2, dp.I32, None) == _lib.ERR_DTYPE


def _inst(op, n, strategy=0, a=P, b=P, out=P2, m=0, lda=0, dtype=dp.F32, reserved=0):
    c = _lib.CInstance()
    c.op, c.dtype, c.strategy, c.reserved = op, dtype, strategy, reserved
    c.m, c.n, c.lda = m, n, lda
    c.a, c.b, c.out = a.value, (b.value if b is not None else None), out.value
    return c


def _plan(insts, strategies):
    arr = (_lib.CInstance * len(insts))(*insts)
    cs = (_lib.CStrategy * len(strategies))(*[s.c() for s in strategies])
    h = ctypes.c_void_p(0)
    st = _lib.lib().dpia_batch_plan_create(arr, len(insts), cs, len(strategies), ctypes.byref(h))
    return st, h


def test_batch_plan_validation_is_host_only():
    L = _lib.lib()
    good = dp.Strategy(seq_len=16, local_size=256, order=dp.STRIDED)
    st, h = _plan([_inst(dp.OP_DOT, 100000), _inst(dp.OP_ASUM, 300, b=None),
                   _inst(dp.OP_GEMV, 4000, m=10, lda=4000)], [good])
    assert st == _lib.OK, _lib.last_error_detail()
    # tables: 3 instances (256 B), tiles, 2 reduction indices, chunk values
    assert L.dpia_batch_workspace_bytes(h) > 0
    L.dpia_batch_plan_destroy(h)
    bad_cases = [
        ([_inst(dp.OP_DOT, 1000, strategy=1)], [good], _lib.ERR_STRATEGY),        # index
        ([_inst(dp.OP_DOT, 1000, dtype=dp.I32)], [good], _lib.ERR_DTYPE),
        ([_inst(dp.OP_DOT, 1000)], [good.with_(accum=dp.KAHAN)], _lib.ERR_STRATEGY),
        ([_inst(dp.OP_DOT, 1000)], [good.with_(local_size=254, wg_combine=dp.SEQ)],
         _lib.ERR_STRATEGY),                                                      # 16-byte loads
        ([_inst(dp.OP_DOT, 1000)], [good.with_(local_size=4096)], _lib.ERR_STRATEGY),  # > 256 threads
        ([_inst(dp.OP_DOT, 1000)], [good.with_(local_size=12, wg_combine=dp.SEQ)],
         _lib.ERR_STRATEGY),                                                      # 3 threads
        ([_inst(dp.OP_DOT, 1000, b=None)], [good], _lib.ERR_NULL),
        ([_inst(dp.OP_DOT, 1000, a=ctypes.c_void_p(0x7000_0008))], [good], _lib.ERR_SHAPE),
        ([_inst(dp.OP_GEMV, 4000, m=10, lda=4002)], [good], _lib.ERR_SHAPE),      # lda % 4
        ([_inst(dp.OP_GEMV, 5000, m=10, lda=5000)], [good], _lib.ERR_SHAPE),      # k > W
        ([_inst(dp.OP_DOT, 0)], [good], _lib.ERR_SHAPE),
        ([_inst(dp.OP_SCAL, 1000)], [good], _lib.ERR_STRATEGY),                 # not batched
        ([_inst(7, 1000)], [good], _lib.ERR_STRATEGY),                          # unknown op
        ([_inst(dp.OP_DOT, 1000, reserved=1)], [good], _lib.ERR_STRATEGY),
    ]
    for insts, strats, want in bad_cases:
        st, h = _plan(insts, strats)
        assert st == want, (st, _lib.last_error_detail())
        assert not h.value
    # workspace checks happen before any copy or launch
    st, h = _plan([_inst(dp.OP_DOT, 100000)], [good])
    assert L.dpia_batch_upload(h, P2, 10, None) == _lib.ERR_WORKSPACE
    assert L.dpia_batch_run(h, P2, 10, None) == _lib.ERR_WORKSPACE
    assert L.dpia_batch_run(None, P2, 1 << 20, None) == _lib.ERR_NULL
    L.dpia_batch_plan_destroy(h)


def test_scal_validates_before_launching():
    L = _lib.lib()
    cs = dp.Strategy(seq_len=16, local_size=256, order=dp.STRIDED).c()
    assert L.dpia_scal(ctypes.byref(cs), dp.I32, 4096, 2.0, P, P2, None) == _lib.ERR_DTYPE
    assert L.dpia_scal(ctypes.byref(cs), dp.F32, 4096, 2.0, None, P2, None) == _lib.ERR_NULL
    assert L.dpia_scal(ctypes.byref(cs), dp.F32, 4096, 2.0, ctypes.c_void_p(0x7000_0004), P2,
                       None) == _lib.ERR_SHAPE
    assert L.dpia_scal(ctypes.byref(cs), dp.F32, 0, 2.0, None, None, None) == _lib.OK
    ks = dp.Strategy(seq_len=16, local_size=256, accum=dp.KAHAN).c()
    assert L.dpia_scal(ctypes.byref(ks), dp.F32, 4096, 2.0, P, P2, None) == _lib.ERR_STRATEGY


def test_read_stream_validates_before_launching():
    L = _lib.lib()
    assert L.dpia_read_stream(P, 4100, 8, P2, None) == _lib.ERR_SHAPE        # not 16-byte units
    assert L.dpia_read_stream(P, -16, 8, P2, None) == _lib.ERR_SHAPE
    assert L.dpia_read_stream(ctypes.c_void_p(0x7000_0008), 4096, 8, P2, None) == _lib.ERR_SHAPE
    assert L.dpia_read_stream(P, 4096, 0, P2, None) == _lib.ERR_SHAPE
    assert L.dpia_read_stream(P, 4096, 65537, P2, None) == _lib.ERR_SHAPE
    assert L.dpia_read_stream(P, 4096, 8, None, None) == _lib.ERR_NULL
    assert L.dpia_read_stream(None, 4096, 8, P2, None) == _lib.ERR_NULL
    assert L.dpia_read_stream(None, 0, 8, P2, None) == _lib.OK                # nothing to read


def test_gemv_blas_validates_before_launching():
    L = _lib.lib()
    cs = dp.Strategy(seq_len=16, local_size=16).c()
    args = (256, 256, 1.0, P, None, P2, 0.5, P2, None)
    assert L.dpia_gemv_blas(ctypes.byref(cs), dp.I32, 4, *args) == _lib.ERR_DTYPE
    assert L.dpia_gemv_blas(ctypes.byref(cs), dp.FP8_E4M3, 4, *args) == _lib.ERR_NULL
    assert L.dpia_gemv_blas(ctypes.byref(cs), dp.F32, 4, 256, 255, 1.0, P, None, P2, 0.5, P2,
                            None) == _lib.ERR_SHAPE
    assert L.dpia_gemv_blas(ctypes.byref(cs), dp.F32, 0, *args) == _lib.OK


def test_module_entry_points_validate_before_any_hip_call():
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.dpia_module_load(None, ctypes.byref(h)) == _lib.ERR_NULL
    assert L.dpia_module_load(b"/nonexistent.hsaco", None) == _lib.ERR_NULL
    args = (ctypes.c_void_p * 1)(0x7000_0000)
    assert L.dpia_module_launch(None, b"k", 1, 64, args, 1, None) == _lib.ERR_NULL
    assert L.dpia_module_unload(None) == _lib.OK


def test_a_missing_library_fails_loudly(monkeypatch, tmp_path):
    # no fallback path: without libdpia.so every entry point raises
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.lib()
    with pytest.raises(ImportError):
        dp.strategy_check(dp.Strategy(seq_len=4, local_size=4), dp.OP_DOT, dp.F32, 0, 16)


@pytest.mark.parametrize("s,dt,n,want", [
    (dp.Strategy(seq_len=16, local_size=16, accum=dp.SUM2), dp.F32, 256 * 3 + 1, _lib.ERR_SHAPE),
    (dp.Strategy(seq_len=16, local_size=16, accum=dp.SUM2), dp.I32, 256 * 3, _lib.ERR_DTYPE),
    (dp.Strategy(seq_len=16, local_size=16, accum=3), dp.F32, 256 * 3, _lib.ERR_STRATEGY),
    (dp.Strategy(seq_len=16, local_size=16, accum=dp.SUM2, final_f64=1), dp.F32, 256 * 3, _lib.OK),
])
def test_sum2_descriptor_rules(s, dt, n, want):
    assert check(s, dp.OP_DOT, dt, 0, n)[0] == want
