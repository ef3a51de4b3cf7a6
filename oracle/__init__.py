"""Plain CPU oracle for run-time generated elementwise and map-reduce kernels.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the
package entry point and the benchmark's CPU-baseline leg may import or run
anything in this package; the GPU library never does.  It shares no code,
headers, tables or helpers with the GPU library.

What it computes, from the paper (Kloeckner et al., "GPU Scripting and Code
Generation with PyCUDA"):

* ``elementwise``: the elementwise facility -- a C statement list run for
  every value of the formal index ``i`` over same-length arrays (section
  "Efficient Evaluation of Element-wise Expressions");
* ``reduce``: the map-reduce facility -- a C map expression at every ``i``,
  folded by a reduce expression in ``a`` and ``b`` from a neutral element, the
  result being a single value of the dtype named first (section
  "Map-Reduce");
* ``scan``: the parallel prefix sums the paper lists among the further
  facilities -- every prefix of the map values folded from the neutral
  element, inclusive or exclusive (section "Further Facilities");
* ``laplace5`` and ``cg``: the conjugate-gradient solver the paper lists
  among the further facilities, on the five-point model problem;
* decoders for the 16- and 8-bit float formats used by the precision
  extension, an exact sum and a norm.

Floating point is evaluated in float64 with a running error bound per value
(see ``interp``); integers exactly.  Parity is pinned by tests against closed
forms, the paper's worked listings, brute force with exact rationals, library
special cases and invariants.  Nothing here is "parity unpinned".
"""

from .api import CSyntaxError, Lanes, OracleError, elementwise, map_chunks, map_values
from .ctype import parse_signature, round_fraction, f32_literal
from .formats import decode_bf16, decode_e4m3fn, decode_f16
from .reduce import ReduceResult, canonical_op, eval_neutral, exact_sum, norm2, reduce
from .scan import ScanResult, scan
from .cg import cg, laplace5

__all__ = ["elementwise", "map_values", "map_chunks", "reduce", "ReduceResult", "scan", "ScanResult",
           "cg", "laplace5",
           "canonical_op", "eval_neutral", "exact_sum", "norm2", "parse_signature",
           "round_fraction", "f32_literal", "decode_bf16", "decode_f16", "decode_e4m3fn",
           "Lanes", "OracleError", "CSyntaxError"]
