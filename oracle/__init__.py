"""Plain, slow, obviously correct FP64 CPU oracle of the CP/N-GMRES method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call or
link this package: it exists so that ``tests/``, the smoke check and the
benchmark's CPU-baseline leg can check the GPU library against an independent
statement of the paper's definitions and algorithm.  It shares no code with
the GPU path; the only common input is the seeded generator module
``workloads``, which holds none of the method's arithmetic.

Modules
-------
``oracle.cp``         -- tensor definitions: MTTKRP (dense and COO), Grams and
                         their Hadamard products, gradient, objective,
                         normalisation/reordering, the ALS sweep.
``oracle.linesearch`` -- the Moré–Thuente line search, written from the
                         published method (More & Thuente, ACM TOMS 20(3),
                         1994).
``oracle.ngmres``     -- N-GMRES Step II and the full N-GMRES and ALS drivers
                         (Algorithm "N-GMRES optimization algorithm").

Every floating-point computation is float64 (float32 tensors are widened
exactly).  Pins: each function is checked by ``tests/test_oracle_*.py``
against values fixed by the paper or by mathematics (brute force on tiny
inputs, closed forms, finite differences, library routines for special cases).
Exact iteration counts and timings of the paper's tables are "parity
unpinned": the paper's seeds and MATLAB runs are not available.
"""
