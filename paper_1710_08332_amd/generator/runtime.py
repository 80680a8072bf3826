"""Compiling and running generated programs.

``compile_program`` writes the HIP source of a translated expression, builds
a gfx950 code object with hipcc (the same flags as the library: no
contraction, no fast math, packed binary32 arithmetic off) and a JSON
description of its kernels and buffers.  ``Generated`` loads that code object
through the library's module entry points and runs the kernels in order on a
stream; workspace buffers are allocated once per ``Generated`` object.
Compiling needs hipcc; running needs only the code object.
"""

from __future__ import annotations

import ctypes
import dataclasses
import json
import os
import shutil
import subprocess
from typing import Dict, Optional

from .. import _lib
from .translate import Program, block_size, grid_size, translate

HIPCC_FLAGS = ["--genco", "--offload-arch=gfx950", "-O3", "-ffp-contract=off", "-fno-fast-math",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return shutil.which("hipcc") or os.path.join(rocm, "bin", "hipcc")


def describe(prog: Program, name: str, text: str, inputs, num: str) -> Dict:
    return {
        "name": name, "expression": text, "num": num,
        "inputs": {k: [v[0], list(v[1])] for k, v in inputs.items()},
        "kernels": [{"name": k.name, "kind": k.kind, "block": block_size(k),
                     "iterations": k.iterations, "local_width": k.local_width}
                    for k in prog.kernels],
        "buffers": [dataclasses.asdict(b) for b in prog.buffers],
    }


def compile_program(text: str, inputs: Dict, path_base: str, num: str = "f32",
                    name: Optional[str] = None) -> str:
    """Translates ``text`` and builds ``path_base``.hsaco / .hip / .json.
    Returns the JSON path."""
    name = name or os.path.basename(path_base)
    prog = translate(text, inputs, num=num, name=name.replace("-", "_"))
    os.makedirs(os.path.dirname(os.path.abspath(path_base)), exist_ok=True)
    src = path_base + ".hip"
    with open(src, "w") as f:
        f.write(prog.source)
    tmp = path_base + ".hsaco.tmp"
    r = subprocess.run([hipcc()] + HIPCC_FLAGS + ["-o", tmp, src], capture_output=True,
                       text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, path_base + ".hsaco")
    meta = describe(prog, name, text, inputs, num)
    with open(path_base + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    return path_base + ".json"


_TORCH_DTYPES = {"float": "float32", "double": "float64", "unsigned": "int32"}


class Generated:
    """A compiled program, loaded on the current device."""

    def __init__(self, json_path: str, device=None):
        import torch
        with open(json_path) as f:
            self.meta = json.load(f)
        hsaco = json_path[:-len(".json")] + ".hsaco"
        if not os.path.exists(hsaco):
            raise FileNotFoundError(f"{hsaco} is missing: build the program first")
        L = _lib.lib()
        h = ctypes.c_void_p()
        _lib.check(L.dpia_module_load(hsaco.encode(), ctypes.byref(h)), "dpia_module_load")
        self._h = h
        self.device = torch.device(device or "cuda")
        self.ws = {b["name"]: torch.zeros(b["elems"],
                                          dtype=getattr(torch, _TORCH_DTYPES[b["ctype"]]),
                                          device=self.device)
                   for b in self.meta["buffers"] if b["kind"] == "ws"}
        cus = torch.cuda.get_device_properties(self.device).multi_processor_count
        self.launches = []
        for k in self.meta["kernels"]:
            if k["kind"] == "single":
                grid = 1
            elif k["kind"] == "global":
                grid = max(1, min(-(-k["iterations"] // 256), cus * 8))
            else:
                grid = max(1, min(k["iterations"], cus * max(1, 2048 // k["block"])))
            self.launches.append((k["name"].encode(), grid, k["block"]))

    def outputs(self):
        """Freshly allocated output buffers, by name."""
        import torch
        return {b["name"]: torch.empty(b["elems"],
                                       dtype=getattr(torch, _TORCH_DTYPES[b["ctype"]]),
                                       device=self.device)
                for b in self.meta["buffers"] if b["kind"] == "out"}

    def run(self, inputs: Dict, outs: Optional[Dict] = None, stream=None):
        """inputs: name -> device tensor (contiguous, of the declared element
        type and size).  Returns the output tensors by name."""
        import torch
        outs = outs if outs is not None else self.outputs()
        ptrs = []
        for b in self.meta["buffers"]:
            if b["kind"] == "in":
                t = inputs[b["name"]]
                if not t.is_contiguous() or t.numel() < b["elems"] or t.device.type != "cuda":
                    raise ValueError(f"input {b['name']} must be a contiguous device tensor of "
                                     f"{b['elems']} elements")
                if t.data_ptr() % 16:
                    # the generated kernels read adjacent lanes' elements with
                    # 16-byte loads
                    raise ValueError(f"input {b['name']} must be 16-byte aligned")
            elif b["kind"] == "out":
                t = outs[b["name"]]
                if t.numel() < b["elems"]:
                    raise ValueError(f"output {b['name']} needs {b['elems']} elements")
            else:
                t = self.ws[b["name"]]
            ptrs.append(t.data_ptr())
        args = (ctypes.c_void_p * len(ptrs))(*ptrs)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        sp = ctypes.c_void_p(s.cuda_stream)
        L = _lib.lib()
        for name, grid, block in self.launches:
            _lib.check(L.dpia_module_launch(self._h, name, grid, block, args, len(ptrs), sp),
                       "dpia_module_launch")
        return outs

    def close(self):
        if self._h:
            _lib.lib().dpia_module_unload(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
