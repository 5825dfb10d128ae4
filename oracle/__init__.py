"""CPU oracle for exact batch MIPS.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library and does not
import it.

* :mod:`oracle.topk`      -- the result: FP64 keys summed left to right, top-K
                              by (key desc, index asc) (C, OpenMP).
* :mod:`oracle.maximus`   -- the pruning index of Section III (k-means, angle
                              bound, sorted lists, the bounded walk), float64
                              numpy, for its invariants.
* :mod:`oracle.backward`  -- gradients of a loss on the top-K scores with the
                              top-K indices held fixed.
"""
