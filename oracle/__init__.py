"""CPU oracle for the Friedkin-Johnsen equilibrium and its five indices.

TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package. The
GPU product path never calls it, links it or shares code with it.

Contents
  dense      dense FP64 forms (Section 2.1 Laplacian, Section 2.2 forest matrix,
             Eq. FJmodel02 equilibrium, Section 3.2 index definitions,
             Proposition 1 quadratic forms, Lemma 4.1 l2 norms)
  forest     brute-force enumeration of spanning rooted forests (Section 2.2)
  circulant  exact spectral solution on cycles and tori (Section 2.1 eigen-
             decomposition of L, specialised to circulant Laplacians)
  sparse     ctypes loader for fj_oracle.c: FP64 Jacobi-preconditioned CG for
             (I+L)z=s, index definitions with compensated sums, and the FJ
             update rule Eq. FJmodel iterated to its fixed point

Pins: see tests/test_oracle_pins.py. Every function here is pinned by at least
one value or property fixed by the paper or by mathematics; none is marked
"parity unpinned".
"""
