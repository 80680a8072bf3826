"""dpia_dot_noalloc (the dot without a workspace argument, its chunk values
and arrival counter in the library's per-device scratch) against dpia_dot
with a caller workspace: same strategy, same inputs, the same bits.  Every
case makes two calls in a row, the second on a smaller input, so the second
call reads a scratch that still holds the first call's values."""

import numpy as np
import pytest

import paper_1710_08332_amd as dp
import synthetic
from oracle import strategies as S
from tests.gpu_util import assert_same_bits, to_plan

pytestmark = pytest.mark.gpu

C_, T_ = dp.CONTIGUOUS, dp.STRIDED

CASES = [
    # (strategy, n of the first call, n of the second call)
    (dp.Strategy(seq_len=256, local_size=16, order=C_, passes=2), 1 << 20, 3 * 4096 + 17),
    (dp.Strategy(seq_len=256, local_size=16, order=C_, passes=1), 1 << 20, 3 * 4096 + 17),
    (dp.Strategy(seq_len=64, local_size=256, order=T_, passes=1), (1 << 22) + 5, 16384 * 2),
    (dp.Strategy(seq_len=256, local_size=1024, order=T_, passes=2), 1 << 26, 1 << 18),
    (dp.Strategy(seq_len=16, local_size=64, order=C_, wg_combine=dp.SEQ, passes=1), 1 << 18, 999),
    (dp.Strategy(seq_len=2048, local_size=64, vec_width=4, wg_combine=dp.NONE, passes=1),
     1 << 24, 1 << 20),
]


def _ids(c):
    s, n1, n2 = c
    return f"C{s.seq_len}-L{s.local_size}-o{s.order}-c{s.wg_combine}-p{s.passes}-V{s.vec_width}"


def _pair(x, y, s, out_dtype=None):
    import torch
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    ref = dp.dot(xt, yt, s, out_dtype=out_dtype)
    out = torch.empty_like(ref).fill_(float("nan"))
    dp.dot_noalloc(xt, yt, s, out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_noalloc_dot_equals_workspace_dot_twice(case):
    s, n1, n2 = case
    for call, n in enumerate((n1, n2)):
        print(f"noalloc dot call {call}: {_ids(case)} n={n}", flush=True)
        x, y = synthetic.dot_inputs(n, synthetic.SEEDS["small"] + call)
        ref, got = _pair(x, y, s)
        assert_same_bits(got, ref, f"call {call}, n={n}")
        if n <= (1 << 20):
            assert_same_bits(got, np.atleast_1d(S.dot(x, y, to_plan(s))), f"oracle, call {call}")


@pytest.mark.parametrize("accum", [dp.KAHAN, dp.SUM2], ids=["kahan", "sum2"])
def test_noalloc_compensated_binary64_twice(accum):
    import torch
    s = dp.Strategy(seq_len=64, local_size=256, order=T_, accum=accum, final_f64=1, passes=1)
    for call, n in enumerate((64 * 256 * 40, 64 * 256 * 3)):
        print(f"noalloc compensated call {call}: accum={accum} n={n}", flush=True)
        x, y = synthetic.kahan_dot_inputs(n, synthetic.SEEDS["precision"] + call)
        ref, got = _pair(x, y, s, out_dtype=torch.float64)
        assert_same_bits(got, ref, f"binary64, call {call}")
        ref32, got32 = _pair(x, y, s, out_dtype=torch.float32)
        assert_same_bits(got32, ref32, f"binary32, call {call}")


def test_noalloc_one_pass_after_a_larger_two_pass_call():
    # the 2-pass call writes chunk values over bytes a 1-pass call of fewer
    # chunks would find right after its own values; the counter sits apart
    big = dp.Strategy(seq_len=16, local_size=64, order=T_, passes=2)
    small = big.with_(passes=1)
    for call, (s, n) in enumerate(((big, 1 << 22), (small, 1 << 14), (small, 1 << 12))):
        print(f"noalloc mixed call {call}: passes={s.passes} n={n}", flush=True)
        x, y = synthetic.dot_inputs(n, synthetic.SEEDS["small"] + 7 + call)
        ref, got = _pair(x, y, s)
        assert_same_bits(got, ref, f"call {call}")


def test_noalloc_integer_dot_twice():
    import torch
    s = dp.Strategy(seq_len=32, local_size=128, order=C_, passes=1)
    rng = np.random.default_rng(5)
    for call, n in enumerate((1 << 20, 4096 * 3 + 1)):
        x = rng.integers(0, 2**32, n, dtype=np.uint32).view(np.int32)
        y = rng.integers(0, 2**32, n, dtype=np.uint32).view(np.int32)
        xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
        ref = dp.dot(xt, yt, s)
        out = torch.zeros_like(ref)
        dp.dot_noalloc(xt, yt, s, out)
        torch.cuda.synchronize()
        assert_same_bits(out.cpu().numpy(), ref.cpu().numpy(), f"call {call}")
        want = np.uint32((x.astype(np.uint64) * y.astype(np.uint64)).sum() % (1 << 32))
        assert out.cpu().numpy().view(np.uint32)[0] == want


def test_noalloc_rejects_strategies_beyond_the_scratch():
    import torch
    s = dp.Strategy(seq_len=1, local_size=1, wg_combine=dp.NONE)
    x = torch.ones(1 << 18, dtype=torch.float32, device="cuda")   # 2^18 values: 1 MiB
    out = torch.full((1,), 7.0, device="cuda")
    with pytest.raises(dp.DpiaError) as e:
        dp.dot_noalloc(x, x, s, out)
    assert e.value.status == dp._lib.ERR_WORKSPACE
    torch.cuda.synchronize()
    assert out.item() == 7.0                  # nothing launched, out untouched
