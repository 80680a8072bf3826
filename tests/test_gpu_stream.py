"""The read-bandwidth ceiling kernel reads every word it is given: the XOR of
its per-work-group values equals the host's XOR of all 32-bit words, for
ragged sizes and any grid."""

import numpy as np
import pytest
import torch

import paper_1710_08332_amd as dp
from tests.gpu_util import cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("words", [4, 12, 4 * 2047, 4 * 2048 * 3 + 8, 1 << 24])
@pytest.mark.parametrize("grid", [1, 3, 256, 65536])
def test_read_stream_xor_of_all_words(words, grid):
    rng = np.random.default_rng(1716 + words)
    host = rng.integers(0, 1 << 32, size=words, dtype=np.uint64).astype(np.uint32)
    x = cuda(host.view(np.int32))
    sink = torch.full((grid,), -1, dtype=torch.int32, device="cuda")   # every value is written
    dp.read_stream(x, grid, sink=sink)
    torch.cuda.synchronize()
    got = np.bitwise_xor.reduce(sink.cpu().numpy().view(np.uint32))
    assert int(got) == int(np.bitwise_xor.reduce(host))


def test_read_stream_empty_leaves_sink():
    sink = torch.full((4,), 7, dtype=torch.int32, device="cuda")
    dp.read_stream(torch.empty(0, dtype=torch.int32, device="cuda"), 4, sink=sink)
    torch.cuda.synchronize()
    assert sink.cpu().tolist() == [7, 7, 7, 7]
