"""Strategy-preserving generation of HIP kernels from DPIA expressions.

The paper's compiler (Secs. 4 and 6) turns a functional DPIA expression whose
parallel maps carry an explicit strategy (mapWorkgroup, mapLocal, mapGlobal,
mapSeq, reduceSeq, toLocal / toPrivate / toGlobal) into imperative code
without changing what the strategy fixes: which work-group and work-item
computes each value, and the order of every sequential fold.  This package
does the same for gfx950:

* ``lang``      parses the expression text, infers types and sizes, and
                checks that the parallel levels nest legally (Sec. 6.1);
* ``translate`` the acceptor- and continuation-passing translations of
                Stage I with the Stage II meanings of mapI and reduceI
                (Sec. 4), layout primitives resolved to index arithmetic
                (Fig. 7), temporaries hoisted (Sec. 6.3), then HIP source
                (Stage III): one kernel per top-level parallel loop;
* ``runtime``   compiles the source for gfx950 with hipcc and runs the
                kernels through the library's module entry points.
"""

from .lang import CheckError, ParseError, parse, check  # noqa: F401
