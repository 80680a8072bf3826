"""The tune cache keys a choice by device, runtime and problem (CPU only)."""

import paper_1710_08332_amd as dp
from paper_1710_08332_amd import autotune as T


def test_cache_keys_carry_device_runtime_and_shape(tmp_path, monkeypatch):
    monkeypatch.setenv("DPIA_TUNE_CACHE", str(tmp_path / "tune.json"))
    s = dp.Strategy(seq_len=64, local_size=256, order=dp.STRIDED)
    T.store("GPU-A gfx950", dp.OP_DOT, dp.F32, (1 << 26,), s)
    assert T.lookup("GPU-A gfx950", dp.OP_DOT, dp.F32, (1 << 26,)) == s
    # another device, dtype or shape finds nothing
    assert T.lookup("GPU-B gfx942", dp.OP_DOT, dp.F32, (1 << 26,)) is None
    assert T.lookup("GPU-A gfx950", dp.OP_DOT, dp.I32, (1 << 26,)) is None
    assert T.lookup("GPU-A gfx950", dp.OP_DOT, dp.F32, (1 << 25,)) is None
    key = next(iter(T.load_cache()))
    assert "hip-" in key and "dpia-abi-" in key and key.startswith("GPU-A gfx950|")
    # the same device under other software finds nothing
    monkeypatch.setattr(T, "runtime_tag", lambda: "hip-0.0|dpia-abi-0")
    assert T.lookup("GPU-A gfx950", dp.OP_DOT, dp.F32, (1 << 26,)) is None
