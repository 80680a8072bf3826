"""Runs a generated program's imperative form on the CPU (test helper).

Executes the commands the generator emits (after its optimisation passes:
hoisted loads, 16-byte loads, blocked loops, coarsened lanes), kernel by
kernel, with numpy scalars of the program's C types: parallel loops run their
iterations one after another (their iterations are independent, Stage II),
and code at
work-group level runs once per work-group (every work-item would compute the
same private values and make the same writes).  Each numeric node is one
numpy operation on binary32 / binary64 / 32-bit unsigned scalars, so the
rounding is the IEEE-754 operation the HIP code performs.  Used by the tests
to check the translation on the CPU; the product never runs it.
"""

from __future__ import annotations

import numpy as np

from oracle import formats
from paper_1710_08332_amd.generator import ir

NP = {"float": np.float32, "double": np.float64, "unsigned": np.uint32,
      "unsigned short": np.uint16, "unsigned char": np.uint8}


def _ix(e, env):
    if isinstance(e, ir.IConst):
        return e.v
    if isinstance(e, ir.IVar):
        return env[e.name]
    a, b = _ix(e.a, env), _ix(e.b, env)
    if e.op == "+":
        return a + b
    if e.op == "*":
        return a * b
    if e.op == "/":
        return a // b
    return a % b


def _ex(e, env, mem, types):
    if isinstance(e, ir.Lit):
        return NP[e.ctype](e.value)
    if isinstance(e, ir.Ref):
        return mem[e.name][0 if e.idx is None else _ix(e.idx, env)]
    if isinstance(e, ir.Bin):
        a, b = _ex(e.a, env, mem, types), _ex(e.b, env, mem, types)
        if e.op == "+":
            r = a + b
        elif e.op == "-":
            r = a - b
        elif e.op == "*":
            r = a * b
        else:
            r = a / b
        return type(a)(r)
    if isinstance(e, ir.Un):
        a = _ex(e.a, env, mem, types)
        return type(a)(-a if e.op == "neg" else abs(a))
    if isinstance(e, ir.Cast):
        return NP[e.ctype](_ex(e.a, env, mem, types))
    if isinstance(e, ir.Decode):
        c = _ex(e.a, env, mem, types)
        dec = formats.bf16_decode if e.fmt == "bf16" else formats.fp8_decode
        return np.float32(dec(np.asarray([c]))[0])
    return _ex(e.options[_ix(e.sel, env)], env, mem, types)


def _run(cmds, env, mem, types):
    for c in cmds:
        if isinstance(c, ir.Decl):
            mem[c.name] = np.zeros(max(1, c.size), NP[c.ctype])
        elif isinstance(c, ir.Assign):
            mem[c.name][0 if c.idx is None else _ix(c.idx, env)] = _ex(c.rhs, env, mem, types)
        elif isinstance(c, ir.Load):
            mem[c.name] = np.array([mem[c.buf][_ix(c.idx, env)]])
        elif isinstance(c, ir.VLoad):
            i, w = _ix(c.idx, env), c.width
            assert i % w == 0, "a vector load at an index that is not a multiple of its width"
            assert w * mem[c.buf].itemsize <= 16, "a vector load of more than 16 bytes"
            mem[c.name] = np.array(mem[c.buf][i:i + w])
            assert mem[c.name].size == w, "a vector load past the end of its array"
        elif isinstance(c, ir.SchedBarrier):
            pass
        elif isinstance(c, ir.Blocked):
            k = 0
            while k + c.step <= c.n:
                env[c.var] = k
                _run(c.main, env, mem, types)
                k += c.step
            while k < c.n:
                env[c.var] = k
                _run(c.tail, env, mem, types)
                k += 1
        elif isinstance(c, ir.Lanes):
            for base in range(0, c.n, c.lanes):
                env[c.var] = base
                _run(c.body, env, mem, types)
        else:
            for i in range(c.n):
                env[c.var] = i
                _run(c.body, env, mem, types)


def run(prog, inputs):
    """inputs: name -> ndarray.  Returns the output buffers by name."""
    mem = {}
    for b in prog.buffers:
        if b.kind == "in":
            a = np.ascontiguousarray(inputs[b.name], NP[b.ctype]).reshape(-1)
            if a.size == 0:
                a = np.zeros(1, NP[b.ctype])
            mem[b.name] = a
        else:
            mem[b.name] = np.zeros(b.elems, NP[b.ctype])
    with np.errstate(over="ignore", under="ignore", invalid="ignore", divide="ignore"):
        for k in prog.kernels:
            _run(k.body, {}, mem, prog.types)
    return {b.name: mem[b.name] for b in prog.buffers if b.kind == "out"}
