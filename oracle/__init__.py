"""FP64 CPU oracle for joint-cut hybrid Schroedinger-Feynman simulation.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package.  It
shares no code with the GPU library (no kernels, headers, tables or helpers);
the two meet only in the seeded circuit descriptions of ``circuitgen``.

Contents
  gates.py        gate matrices written from their definitions
  sv.c, sv.py     plain Schroedinger-style statevector simulation (Sec. II-A)
  hsf.py          plain HSF with joint cutting (Sec. II-B, III-A, IV-A):
                  hull, block product, operator-Schmidt SVD, path table,
                  per-path half-states, Kronecker sum, Gram-matrix norm
  grad.py         parameter-shift / finite-difference / adjoint gradients

Every floating-point result is complex128.  Parity status of each function
is listed in its docstring; "parity unpinned" marks the ones no test pins to
something outside the oracle.
"""
