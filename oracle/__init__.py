"""CPU oracle for delegate-centric top-k / k-selection (Dr. Top-k, SC'21).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` use it.  It shares no code with the HIP library and never
reads a value produced by it.

What it computes
----------------
The paper (Section 1) defines top-k as the k largest elements of an input
vector V and k-selection as the k-th largest.  The delegate method is exact:
Rules 1-3 (Section 4) only discard elements that cannot be in the answer, so
the oracle for the final answer is that plain definition written out:

* ``order``  -- the ranking order on keys (unsigned 32-bit ints as the paper
  evaluates them; float32 under IEEE 754 totalOrder, this project's reading),
  with equal keys ranked by ascending position (this project's tie rule).
* ``topk``   -- brute-force ranks, sort-and-choose, selection-then-extract, a
  textbook min-heap, and selection split over host threads then merged: five
  routes to the same answer.
* ``stages`` -- the method's own steps in the paper's order (delegate vector,
  threshold from the k-th delegate, qualifying subranges, filtered
  concatenation, second top-k), used to check the GPU path stage by stage.

Parity pins for all of these live in ``tests/test_oracle_*.py``.
"""
from .order import rank_key, INVALID_INDEX
from .topk import (topk_bruteforce, topk_sort, topk_select, topk_heap, topk_threaded, kth_value,
                   topk as topk_reference)
from . import stages

__all__ = ["rank_key", "INVALID_INDEX", "topk_bruteforce", "topk_sort", "topk_select",
           "topk_heap", "topk_threaded", "kth_value", "topk_reference", "stages"]
