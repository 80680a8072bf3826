"""Timing events for measurements on the GPU.

HIP events created with ``hipEventDisableSystemFence``: recording a default
event performs a system-scope cache write-back and invalidate, which costs a
few microseconds per record and perturbs the work after it.  Events used
only to time work do not need it.  The events come from the HIP runtime that
torch has loaded, so they share its streams; where that library cannot be
found, torch's events are used.
"""

from __future__ import annotations


class TimingEvents:
    """``n`` pairs of timing events: ``record(i, 0)`` / ``record(i, 1)`` on
    torch's current stream, ``elapsed_ms(i)`` after a synchronisation."""

    DISABLE_SYSTEM_FENCE = 0x20000000

    def __init__(self, n):
        import ctypes
        import torch
        self._ct = ctypes
        self.hip = None
        try:
            with open("/proc/self/maps") as f:
                paths = [ln.split()[-1] for ln in f if "libamdhip64" in ln]
            self.hip = ctypes.CDLL(paths[0]) if paths else None
        except OSError:
            self.hip = None
        self.pairs = []
        for _ in range(n):
            if self.hip is None:
                self.pairs.append((torch.cuda.Event(enable_timing=True),
                                   torch.cuda.Event(enable_timing=True)))
                continue
            pair = []
            for _ in range(2):
                e = ctypes.c_void_p()
                if self.hip.hipEventCreateWithFlags(ctypes.byref(e), ctypes.c_uint(
                        self.DISABLE_SYSTEM_FENCE)) != 0:
                    raise RuntimeError("hipEventCreateWithFlags failed")
                pair.append(e)
            self.pairs.append(tuple(pair))
        self.kind = "hip events without system fence" if self.hip else "torch events"

    def record(self, i, which):
        import torch
        e = self.pairs[i][which]
        if self.hip is None:
            e.record()
        elif self.hip.hipEventRecord(e, self._ct.c_void_p(
                torch.cuda.current_stream().cuda_stream)) != 0:
            raise RuntimeError("hipEventRecord failed")

    def elapsed_ms(self, i):
        a, b = self.pairs[i]
        if self.hip is None:
            return a.elapsed_time(b)
        ms = self._ct.c_float()
        if self.hip.hipEventElapsedTime(self._ct.byref(ms), a, b) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return ms.value

    def close(self):
        if self.hip is not None:
            for a, b in self.pairs:
                self.hip.hipEventDestroy(a)
                self.hip.hipEventDestroy(b)
            self.pairs = []
