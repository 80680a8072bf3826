"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
the oracle on the same seeded inputs, compare bits."""

import numpy as np

import paper_1710_08332_amd as dp
from oracle import strategies as S


def to_plan(s: dp.Strategy) -> S.Plan:
    """The oracle's reading of a descriptor (field for field)."""
    return S.Plan(seq=s.seq_len, lanes=s.local_size,
                  order="strided" if s.order == dp.STRIDED else "contiguous",
                  combine={dp.SEQ: "seq", dp.TREE: "tree", dp.NONE: "none"}[s.wg_combine],
                  accum={dp.PLAIN: "plain", dp.KAHAN: "kahan", dp.SUM2: "sum2"}[s.accum],
                  final_f64=bool(s.final_f64), rows=s.rows_per_wg, row_parts=s.row_parts,
                  vec=max(1, s.vec_width))


def bits(a):
    a = np.asarray(a)
    if a.dtype == np.float32:
        return a.view(np.uint32)
    if a.dtype == np.float64:
        return a.view(np.uint64)
    if a.dtype == np.int32:
        return a.view(np.uint32)
    return a


def assert_same_bits(got, want, what=""):
    g, w = bits(got), bits(want)
    if not np.array_equal(g, w):
        diff = np.nonzero(np.atleast_1d(g != w))[0]
        raise AssertionError(f"{what}: {len(diff)} mismatching elements, first at {diff[:5]}: "
                             f"got {np.atleast_1d(got)[diff[:5]]} want {np.atleast_1d(want)[diff[:5]]}")


def cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_dot(x, y, s, out_dtype=None):
    import torch
    xt, yt = cuda(x.view(np.int32) if x.dtype == np.uint32 else x), \
        cuda(y.view(np.int32) if y.dtype == np.uint32 else y)
    r = dp.dot(xt, yt, s, out_dtype=out_dtype)
    torch.cuda.synchronize()
    out = r.cpu().numpy()
    if out.dtype == np.int32:
        out = out.view(np.uint32)
    return out[0]


def gpu_asum(x, s):
    import torch
    r = dp.asum(cuda(x), s)
    torch.cuda.synchronize()
    return r.cpu().numpy()[0]


def gpu_gemv(A, x, s, a_dtype=None, scale=None):
    import torch
    At = cuda(A.view(np.int32) if A.dtype == np.uint32 else
              (A.view(np.int16) if A.dtype == np.uint16 else A))
    xt = cuda(x.view(np.int32) if x.dtype == np.uint32 else x)
    st = cuda(scale) if scale is not None else None
    y = dp.gemv(At, xt, s, row_scale=st, a_dtype=a_dtype)
    torch.cuda.synchronize()
    out = y.cpu().numpy()
    return out.view(np.uint32) if out.dtype == np.int32 else out


def discriminating(seed, n):
    """Cancelling products (exact dot 0): the result is pure rounding error,
    which identifies the association."""
    g = np.random.default_rng(seed)
    v = (np.where(g.random(n // 2) < 0.5, -1, 1) * 2.0 ** g.uniform(-20, 20, n // 2)).astype(np.float32)
    w = 2 * g.random(n // 2, dtype=np.float32) - 1
    pad = [np.zeros(n % 2, np.float32)]       # odd n: one zero product
    perm = g.permutation(n)
    return (np.concatenate([v, v] + pad)[perm], np.concatenate([w, -w] + pad)[perm])
