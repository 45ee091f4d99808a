"""CPU oracle for Chebyshev-filtered subspace iteration (ChFSI).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, complex128
reference written from the paper (Berljafa, Wortmann, Di Napoli, "An
optimized and scalable eigensolver for sequences of eigenvalue problems").
Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the GPU library never calls it and shares no code
with it.

Modules
  chebyshev   Chebyshev polynomials, convergence ratio, the filter (Alg. 2)
  eigh        dense Hermitian eigensolver (Householder tridiagonalisation +
              implicit symmetric QR with Wilkinson shift)
  counter_rng SplitMix64 counter-based generator (start vectors)
  chfsi       the ChFSI loop (Alg. 1): bounds, filter, QR, Rayleigh-Ritz,
              residuals, locking, degree optimisation, reduction to
              standard form
"""
