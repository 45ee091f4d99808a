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
  mlp         the degree network (forward, gradient, Adam), its features,
              training target and margin, and the learned degree rule

Not here, parity unpinned: the sequence-level degree optimisation the paper
calls Multiple Optimization (Sec. 3.1.1; the library's degree_mode 3).  The
paper defers that algorithm to another publication, so no definition exists
to write an oracle from; the library's form is tested against its own
definition and its eigenvalues against this oracle.
"""
