"""CPU oracle for Compressed Randomized UTV (CoR-UTV) and ALM-CoRUTV robust PCA.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package:
only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
use it.  It shares no code with the HIP library (no kernels, headers, tables or
helpers); the only thing both sides consume is the seeded input generator in
``workloads``, which holds none of the method's arithmetic.

Everything here is plain float64 numpy, written from the paper:

* ``philox``  -- the Gaussian test matrix (Sec. 3.1, "standard Gaussian matrix"
  drawn by a random number generator), as a counter-based Philox4x64-10 stream
  plus a Box-Muller transform whose ln/cos are defined by truncated series.
* ``dense``   -- Householder thin QR, column-pivoted QR (QRCP) of the core,
  one-sided Jacobi SVD (used only by pins).
* ``corutv``  -- CoR-UTV, basic form (eqs. 4-9) and with power iterations
  (Algorithm 1), in the literal and the re-orthonormalised form.
* ``rpca``    -- ALM-CoRUTV (Algorithm 2 with the operators of eq. 12 and the
  shrinkage operator of Sec. 4).
* ``bf16``    -- round-to-nearest-even emulation of bfloat16 and the 3-term
  split-bf16 product, for unit tests of the reduced-precision sketches.

Parity pins (closed forms, invariants, library cross-checks, brute force) live
in ``tests/test_oracle_*.py``.  Functions that no pin fixes say
"parity unpinned" in their docstring.
"""
