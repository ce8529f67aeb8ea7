"""CPU oracle for the staggered conjugate-gradient solve.

TEST INFRASTRUCTURE. Nothing in the product path (the HIP library and its
Python binding) imports, links or runs anything in this package; only the
tests, the smoke check and the CPU-baseline leg of the benchmark do.

The oracle is a plain, slow, obviously-correct restatement of what the paper
(Jang, Kim and Lee, "Multi GPU Performance of Conjugate Gradient Solver with
Staggered Fermions in Mixed Precision", Lattice 2011) computes:

* ``oracle.stag``   numpy, fp64: the staggered Dirac operator of Eq.4-5, the
  normal operator A = -D^2 + m^2 of Eq.2-3 restricted to even sites, CG as in
  Fig.1, iterative refinement as in Fig.2, and the corrected mixed-precision
  CG of Sec.3.2 (Eq.6 direction carry-over with reliable and group-wise
  updates) emulated with explicit storage quantisers;
* ``oracle.dense``  the same operator assembled as a dense matrix entry by
  entry from Eq.4 (brute force for tiny lattices) and the closed-form
  free-field / constant-twist spectra and FFT solves used to pin the above;
* ``oracle.c``      a plain C + OpenMP fp64 version of the Dirac operator, A
  and Fig.1 CG (the CPU baseline), loaded through ctypes.

Parity pins for every function are in tests/test_oracle_*.py. One function
carries no pin beyond its true residual: the FP16-with-per-site-scale mixed
emulation, whose iteration count the paper says nothing about ("parity
unpinned" for its iteration count; its solution is still pinned by the fp64
true residual).
"""
