"""Optimisations of the imperative program, as program-to-program passes.

Each pass keeps every arithmetic operation and, for each accumulator, the
order of its updates: it only changes when reads happen and which work-item
runs which independent iteration.  The passes run before emission, so the
test suite executes their output on the CPU (against the oracle) exactly as
the GPU runs it.

1. ``extract_loads``: in a sequential loop of straight-line code, every read
   of an array at a loop-dependent position, of an input or of an array the
   loop does not write, becomes a private constant (``Load``) at the start of
   the body.
2. ``coarsen``: a mapLocal loop whose lanes are straight-line code around
   such loops runs F adjacent lanes per work-item (``Lanes``; F = 16 bytes
   of the narrowest loaded element: 4 binary32, 8 bf16 or 16 fp8 lanes, and
   at least 64 work-items): the lanes' commands are copied with their
   private names renamed and their loops fused, each lane's steps in its own
   order (lanes are independent iterations, Stage II).  Where w lanes read w
   consecutive elements from an index that is a multiple of w, one load of
   up to 16 bytes (``VLoad``) serves them.
3. ``batch``: such a loop runs B iterations per round (``Blocked``): the
   loads of all B iterations first, then the B steps in increasing order, so
   B iterations' loads (128 bytes per work-item) are in flight together.

Before these, ``pair_rows`` runs two iterations of a work-group's
sequential loop at once where they share operand reads (a gemv's rows
reading the same x with A in a 1- or 2-byte format): the two iterations'
commands are copied with their names renamed, and their parallel and
sequential loops fused position by position, so that ``extract_loads``
finds each shared read once.  The two iterations are independent (the
loop is a ``map``), and each keeps its own operations in its own order.
"""

from __future__ import annotations

from typing import Dict, List, Set

from . import ir
from .ir import (Assign, Blocked, Decl, For, IConst, IVar, Lanes, Load, ParFor, Ref,
                 SchedBarrier, VLoad, iadd)

LANES = 4
BATCH_BYTES = 128         # bytes of loads per work-item issued per round


# ------------------------------------------------------------------ helpers

def ix_uses(e, var: str) -> bool:
    if isinstance(e, IVar):
        return e.name == var
    if isinstance(e, ir.IBin):
        return ix_uses(e.a, var) or ix_uses(e.b, var)
    return False


def ix_replace(e, var: str, by):
    if isinstance(e, IVar) and e.name == var:
        return by
    if isinstance(e, ir.IBin):
        return ir.IBin(e.op, ix_replace(e.a, var, by), ix_replace(e.b, var, by))
    return e


def ex_ix(e, g):
    """e with g applied to every index expression (positions and selectors)."""
    if isinstance(e, Ref):
        return e if e.idx is None else Ref(e.name, g(e.idx))
    if isinstance(e, ir.Bin):
        return ir.Bin(e.op, ex_ix(e.a, g), ex_ix(e.b, g))
    if isinstance(e, ir.Un):
        return ir.Un(e.op, ex_ix(e.a, g))
    if isinstance(e, ir.Cast):
        return ir.Cast(e.ctype, ex_ix(e.a, g))
    if isinstance(e, ir.Select):
        return ir.Select(g(e.sel), tuple(ex_ix(o, g) for o in e.options))
    if isinstance(e, ir.Decode):
        return ir.Decode(e.fmt, ex_ix(e.a, g))
    return e


def ex_refs(e, f):
    """e with f applied to every Ref."""
    if isinstance(e, Ref):
        return f(e)
    if isinstance(e, ir.Bin):
        return ir.Bin(e.op, ex_refs(e.a, f), ex_refs(e.b, f))
    if isinstance(e, ir.Un):
        return ir.Un(e.op, ex_refs(e.a, f))
    if isinstance(e, ir.Cast):
        return ir.Cast(e.ctype, ex_refs(e.a, f))
    if isinstance(e, ir.Select):
        return ir.Select(e.sel, tuple(ex_refs(o, f) for o in e.options))
    if isinstance(e, ir.Decode):
        return ir.Decode(e.fmt, ex_refs(e.a, f))
    return e


def _straight(body) -> bool:
    return all(isinstance(b, (Assign, Load, VLoad)) or
               (isinstance(b, Decl) and b.space == "private") for b in body)


def _rewrite(cmd, g_ix, ren: Dict[str, str]):
    """A straight-line command with index map g_ix and private names renamed."""
    def rn(r):
        return Ref(ren.get(r.name, r.name), r.idx)
    if isinstance(cmd, Decl):
        return Decl(ren.get(cmd.name, cmd.name), cmd.ctype, cmd.size, cmd.space)
    if isinstance(cmd, Assign):
        return Assign(ren.get(cmd.name, cmd.name), None if cmd.idx is None else g_ix(cmd.idx),
                      ex_refs(ex_ix(cmd.rhs, g_ix), rn), cmd.space, cmd.ctx)
    if isinstance(cmd, Load):
        return Load(ren.get(cmd.name, cmd.name), cmd.ctype, cmd.buf, g_ix(cmd.idx), cmd.nt)
    if isinstance(cmd, VLoad):
        return VLoad(ren.get(cmd.name, cmd.name), cmd.ctype, cmd.buf, g_ix(cmd.idx), cmd.nt,
                     cmd.width)
    raise TypeError(f"not straight-line: {cmd!r}")


def _defined(body) -> Set[str]:
    out = set()
    for b in body:
        if isinstance(b, (Decl, Load, VLoad)):
            out.add(b.name)
        elif isinstance(b, (For, Blocked)):
            out |= _defined(b.body if isinstance(b, For) else b.main + b.tail)
    return out


# ------------------------------------------------------------------ 0. rows

def _deep_defined(body) -> Set[str]:
    out = set()
    for b in body:
        if isinstance(b, Decl):
            out.add(b.name)
        elif isinstance(b, (For, ParFor)):
            out |= _deep_defined(b.body)
    return out


def _deep_rewrite(cmd, g_ix, ren: Dict[str, str]):
    """cmd (declarations, assignments and loops) with index map g_ix and the
    names in ren renamed."""
    if isinstance(cmd, For):
        return For(cmd.var, cmd.n, [_deep_rewrite(b, g_ix, ren) for b in cmd.body])
    if isinstance(cmd, ParFor):
        return ParFor(cmd.level, cmd.var, cmd.n, [_deep_rewrite(b, g_ix, ren) for b in cmd.body])
    return _rewrite(cmd, g_ix, ren)


def _jam(b0, b1):
    """Two copies of one command list, run together: loops at the same
    position fused (copy 0's commands, then copy 1's, per iteration), other
    commands one after the other."""
    out = []
    for x0, x1 in zip(b0, b1):
        if isinstance(x0, ParFor) and x0.level == "local":
            out.append(ParFor(x0.level, x0.var, x0.n, _jam(x0.body, x1.body)))
        elif isinstance(x0, For):
            out.append(For(x0.var, x0.n, _jam(x0.body, x1.body)))
        else:
            out += [x0, x1]
    return out


def _shared_narrow_reads(loop: For, inputs: Set[str], types) -> bool:
    """The loop's lane folds read an input at positions that do not depend
    on the loop variable (shared by its iterations) beside an input of 1 or
    2 bytes per element that they do depend on."""
    shared, narrow = False, False

    def refs(e, acc):
        if isinstance(e, Ref):
            acc.append(e)
        elif isinstance(e, (ir.Bin,)):
            refs(e.a, acc)
            refs(e.b, acc)
        elif isinstance(e, (ir.Un, ir.Cast, ir.Decode)):
            refs(e.a, acc)
        elif isinstance(e, ir.Select):
            for o in e.options:
                refs(o, acc)
        return acc

    def walk(body, in_lanes):
        nonlocal shared, narrow
        for b in body:
            if isinstance(b, ParFor):
                walk(b.body, in_lanes or b.level == "local")
            elif isinstance(b, For):
                walk(b.body, in_lanes)
            elif isinstance(b, Assign) and in_lanes:
                for r in refs(b.rhs, []):
                    if r.idx is None or r.name not in inputs:
                        continue
                    if ix_uses(r.idx, loop.var):
                        narrow = narrow or _ESIZE.get(types[r.name], 4) <= 2
                    else:
                        shared = True
    walk(loop.body, False)
    return shared and narrow


def _independent(loop: For) -> bool:
    """No iteration of the loop reads what another writes: every assignment
    targets a name declared in the body or a global array at a position
    that depends on the loop variable (a map's output, not a reduction's
    accumulator)."""
    local = _deep_defined(loop.body)

    def ok(body):
        for b in body:
            if isinstance(b, (For, ParFor)):
                if not ok(b.body):
                    return False
            elif isinstance(b, Assign) and b.name not in local:
                if b.space != "global" or b.idx is None or not ix_uses(b.idx, loop.var):
                    return False
        return True
    return ok(loop.body)


def pair_rows(cmds, inputs: Set[str], types: Dict[str, str], in_group: bool = False):
    out = []
    for c in cmds:
        if isinstance(c, ParFor):
            out.append(ParFor(c.level, c.var, c.n,
                              pair_rows(c.body, inputs, types, c.level == "workgroup")))
        elif (isinstance(c, For) and in_group and c.n >= 2 and c.n % 2 == 0 and
              any(isinstance(b, ParFor) for b in c.body) and _independent(c) and
              _shared_narrow_reads(c, inputs, types)):
            names = _deep_defined(c.body)
            copies = []
            for j in range(2):
                ren = {nm: f"{nm}_r{j}" for nm in names}
                for nm in names:
                    if nm in types:
                        types[ren[nm]] = types[nm]
                row = iadd(ir.imul(IVar(c.var), 2), j)
                copies.append([_deep_rewrite(b, lambda e, row=row: ix_replace(e, c.var, row), ren)
                               for b in c.body])
            out.append(For(c.var, c.n // 2, _jam(copies[0], copies[1])))
        else:
            out.append(c)
    return out


# ------------------------------------------------------------------ 1. loads

def extract_loads(cmds, inputs: Set[str], streamed: Set[str], types: Dict[str, str], fresh):
    out = []
    for c in cmds:
        if isinstance(c, For) and _straight(c.body):
            out.append(For(c.var, c.n, _loads_first(c.body, c.var, inputs, streamed, types, fresh)))
        elif isinstance(c, For):
            out.append(For(c.var, c.n, extract_loads(c.body, inputs, streamed, types, fresh)))
        elif isinstance(c, ParFor):
            out.append(ParFor(c.level, c.var, c.n,
                              extract_loads(c.body, inputs, streamed, types, fresh)))
        else:
            out.append(c)
    return out


def _loads_first(body, var, inputs, streamed, types, fresh):
    written = {b.name for b in body if isinstance(b, Assign)}
    regs: Dict[Ref, str] = {}
    loads: List[Load] = []

    def take(r):
        if r.idx is None or not ix_uses(r.idx, var):
            return r
        if r.name not in inputs and r.name in written:
            return r
        if r not in regs:
            regs[r] = fresh("ld")
            loads.append(Load(regs[r], types[r.name], r.name, r.idx, r.name in streamed))
        return Ref(regs[r], None)
    rest = []
    for b in body:
        if isinstance(b, Assign):
            rest.append(Assign(b.name, b.idx, ex_refs(b.rhs, take), b.space, b.ctx))
        else:
            rest.append(b)
    return loads + rest


# ------------------------------------------------------------------ 2. coarsen

_ESIZE = {"float": 4, "unsigned": 4, "double": 8, "unsigned short": 2, "unsigned char": 1}


def _lanes_for(c: ParFor, types) -> int:
    """Lanes per work-item for a mapLocal loop, or 0 to leave it alone: 16
    bytes of the narrowest element its fold loops load (4 lanes of binary32,
    8 of bf16, 16 of fp8), fewer if the loop is too short to keep 64
    work-items busy."""
    if c.level != "local":
        return 0
    loops = [b for b in c.body if isinstance(b, For)]
    if not loops or not all(_straight(b.body) for b in loops):
        return 0
    loads = [x for b in loops for x in b.body if isinstance(x, Load)]
    if not loads:
        return 0
    if not all(isinstance(b, (For, Assign)) or (isinstance(b, Decl) and b.space == "private")
               for b in c.body):
        return 0
    F = min(16, 16 // min(_ESIZE.get(types[x.buf], 4) for x in loads))
    while F >= LANES:
        if c.n % F == 0 and c.n >= 64 * F:
            return F
        F //= 2
    return 0


def _additive_once(e, var: str) -> int:
    """How often var occurs, if only as a summand (else -1)."""
    if isinstance(e, IVar):
        return 1 if e.name == var else 0
    if isinstance(e, IConst):
        return 0
    if e.op == "+":
        a, b = _additive_once(e.a, var), _additive_once(e.b, var)
        return -1 if a < 0 or b < 0 else a + b
    return -1 if ix_uses(e, var) else 0


def _aligned(e, base: str, w: int) -> bool:
    """e is a multiple of w for all values (base is one by construction)."""
    if isinstance(e, IConst):
        return e.v % w == 0
    if isinstance(e, IVar):
        return e.name == base
    if e.op == "+":
        return _aligned(e.a, base, w) and _aligned(e.b, base, w)
    if e.op == "*":
        return _aligned(e.a, base, w) or _aligned(e.b, base, w)
    return False


def coarsen(cmds, types: Dict[str, str], fresh):
    out = []
    for c in cmds:
        if isinstance(c, ParFor) and _lanes_for(c, types):
            out.append(_coarsened(c, _lanes_for(c, types), types, fresh))
        elif isinstance(c, ParFor):
            out.append(ParFor(c.level, c.var, c.n, coarsen(c.body, types, fresh)))
        elif isinstance(c, For):
            out.append(For(c.var, c.n, coarsen(c.body, types, fresh)))
        else:
            out.append(c)
    return out


def _coarsened(c: ParFor, F: int, types, fresh) -> Lanes:
    base = fresh(c.var + "q")
    names = _defined(c.body)
    ren = [{nm: f"{nm}_{j}" for nm in names} for j in range(F)]

    def lane_ix(j):
        by = iadd(IVar(base), j)
        return lambda e: ix_replace(e, c.var, by)
    body = []
    for b in c.body:
        if not isinstance(b, For):
            body += [_rewrite(b, lane_ix(j), ren[j]) for j in range(F)]
            continue
        # the F lanes' loads of consecutive elements: groups of w lanes (w
        # elements, at most 16 bytes) from an index that is a multiple of w
        vec_of: Dict[tuple, tuple] = {}              # (load name, lane) -> (vector, component)
        vloads = []
        for ld in (x for x in b.body if isinstance(x, Load)):
            w = min(F, 16 // _ESIZE.get(types[ld.buf], 4))
            if w < 2 or _additive_once(ld.idx, c.var) != 1 or \
                    not _aligned(ix_replace(ld.idx, c.var, IVar(base)), base, w):
                continue
            for g in range(F // w):
                q = fresh("vq")
                vloads.append(VLoad(q, ld.ctype, ld.buf,
                                    ix_replace(ld.idx, c.var, iadd(IVar(base), g * w)), ld.nt, w))
                for i in range(w):
                    vec_of[(ld.name, g * w + i)] = (q, i)
        fused = list(vloads)
        for j in range(F):
            alias = {f"{nm}_{j}": vec_of[(nm, jj)] for (nm, jj) in vec_of if jj == j}

            def comp(r, alias=alias):
                if r.name in alias:
                    q, i = alias[r.name]
                    return Ref(q, IConst(i))
                return r
            for x in b.body:
                if isinstance(x, Load) and (x.name, j) in vec_of:
                    continue                          # served by a vector load
                y = _rewrite(x, lane_ix(j), ren[j])
                if isinstance(y, Assign):
                    y = Assign(y.name, y.idx, ex_refs(y.rhs, comp), y.space, y.ctx)
                fused.append(y)
        body.append(For(b.var, b.n, fused))
    return Lanes(base, c.n, F, body)


# ------------------------------------------------------------------ 3. batch

def batch(cmds, fresh):
    out = []
    for c in cmds:
        if isinstance(c, For) and _straight(c.body):
            out.append(_batched(c) or c)
        elif isinstance(c, For):
            out.append(For(c.var, c.n, batch(c.body, fresh)))
        elif isinstance(c, ParFor):
            out.append(ParFor(c.level, c.var, c.n, batch(c.body, fresh)))
        elif isinstance(c, Lanes):
            out.append(Lanes(c.var, c.n, c.lanes, batch(c.body, fresh)))
        else:
            out.append(c)
    return out


def _batched(c: For):
    loads = [b for b in c.body if isinstance(b, (Load, VLoad)) and ix_uses(b.idx, c.var)]
    if not loads:
        return None
    nbytes = sum((b.width if isinstance(b, VLoad) else 1) * _ESIZE.get(b.ctype, 4) for b in loads)
    B = max(1, BATCH_BYTES // nbytes)
    if c.n < 2 * B:
        return None
    names = _defined(c.body)
    first, rest = [], []
    for u in range(B):
        ren = {nm: f"{nm}_u{u}" for nm in names}

        def shift(e, u=u):
            return ix_replace(e, c.var, iadd(IVar(c.var), u))
        for b in c.body:
            y = _rewrite(b, shift, ren)
            (first if isinstance(b, (Load, VLoad)) else rest).append(y)
    return Blocked(c.var, c.n, B, first + [SchedBarrier()] + rest, c.body)


def optimise(cmds, inputs: Set[str], streamed: Set[str], types: Dict[str, str], fresh):
    cmds = pair_rows(cmds, inputs, types)
    cmds = extract_loads(cmds, inputs, streamed, types, fresh)
    cmds = coarsen(cmds, types, fresh)
    return batch(cmds, fresh)
