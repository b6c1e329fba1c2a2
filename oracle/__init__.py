"""FP64 CPU oracle for the IPFP matching sweep -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously correct reference against which the
HIP implementation is checked. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does, and
it imports nothing from the product package.

Contents (each function cites the passage of the paper it follows):

* ``oracle.ipfp``    -- batch IPFP on an explicit kernel matrix (Sec. 3.2,
  eq. 6-7, Alg. 1), the mini-batch form built from factors (Sec. 3.3,
  eq. 8-10, Alg. 2), residuals, matching masses, the stable-factor export.
* ``oracle.brute``   -- an IPFP-free solution of the primal program (eq. 2-3)
  by damped Newton, and of its Lagrange dual, used to pin ``oracle.ipfp``.
* ``oracle.closed``  -- closed forms (uniform and 1x1 markets) and the exact
  O(N+M) replay of the iteration for a separable surplus.
* ``oracle.quant``   -- BF16 and FP8-e4m3 rounding written from the formats'
  definitions, so the oracle can be fed the same quantised factor values the
  GPU path computes with.

Parity status of every function is recorded in its docstring; functions with
no independent pin say "parity unpinned".
"""
