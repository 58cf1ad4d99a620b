"""CPU oracle for the Clifford-fullstate hybrid rotation path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the HIP library and never imports it; the two meet only through the
seeded inputs of the ``workloads`` package.

``oracle.sim``   ctypes front end of the C oracle (gate-by-gate ladder
                 simulator, sparse definition simulator, Heisenberg walk,
                 letter-by-letter expectation values) plus parameter-shift and
                 finite-difference gradients built on it.
``oracle.dense`` numpy/scipy dense-matrix checks for n <= 6 (matrix
                 exponentials, explicit conjugation U^dag P U).

Every function is pinned by a ``-m "not gpu"`` test against something other
than itself (dense matrix exponentials, textbook gate identities, closed forms
stated in the paper).  No function here is "parity unpinned".
"""
