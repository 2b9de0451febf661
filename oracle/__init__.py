"""CPU reference (oracle) for the circuit simulator.

TEST INFRASTRUCTURE ONLY: only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. The product path never
does, and this package imports nothing from the product package.

* :mod:`oracle.oracle` -- ctypes wrapper over ``qsv_oracle.c`` (complex128
  per-gate simulator, FP64 expectation values and adjoint gradients) plus
  parameter-shift and central finite-difference gradients built on its forward.
* :mod:`oracle.kron` -- NumPy brute force: full 2^n x 2^n operators built by
  Kronecker products as in Eq. (2), for n <= 8.
"""
