"""CPU oracle for brute-force incoherent dedispersion.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, loads or
calls anything in this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg do.  It shares no code with the HIP library.

* ``oracle.dedisp``   -- plain numpy, FP64 / int64, written from the
  definition of the operator (see that module's header for every function's
  source passage).
* ``oracle/dedisp_ref.c`` -- the same definition as plain C with OpenMP over
  DM trials, for full-size references and for CPU timing.  ``oracle.cref``
  loads it with ctypes.
"""
