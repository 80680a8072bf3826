"""CPU oracle for the DPIA dot / asum / gemv strategies.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP library (``paper_1710_08332_amd``) and imports nothing from it.

What it computes: the value of a functional DPIA expression (Atkey, Steuwer,
Lindley, Dubach, "Strategy Preserving Compilation for Parallel Functional
Code"), built from the functional primitives of Fig. 5a plus the OpenCL
strategy primitives of Sec. 6.1, under the set-theoretic data semantics of
Sec. 5.1 (arrays are functions from indices to values) and the Stage II
meanings of map (a parallel loop over indices) and reduce (a new accumulator,
then a sequential loop in increasing index order).  A strategy therefore fixes
the exact floating-point association, and the oracle reproduces it.

Modules:
  dpia_lang   -- abstract syntax, parser and printer of the expression text
  strategies  -- expressions for the dot / asum / gemv strategy families
  eval_numpy  -- evaluator used at every size (parallel maps become numpy
                 array operations; every sequential reduce is a Python loop)
  eval_scalar -- element-by-element evaluator for tiny inputs, arithmetic by
                 rounding Python doubles to binary32 after each operation
  formats     -- bf16 and fp8-e4m3 decoding from the format definitions
  exact       -- correctly rounded reference sums (math.fsum) and bounds
  parallel    -- the same expressions with the outermost map (chunks, gemv
                 rows) split over worker processes and one fold at the end:
                 the serial result's bits on every core of the host

Parity status: every function here is pinned by the tests in
``tests/test_oracle_*.py`` (closed forms, laws of Sec. 5.3, integer brute
force, error bounds, library decoders); none is "parity unpinned".
"""

from .dpia_lang import parse, to_text  # noqa: F401
from .strategies import Plan, dot_expr, asum_expr, gemv_expr  # noqa: F401
from .eval_numpy import evaluate  # noqa: F401
