"""CPU ORACLE for the configuration-interaction hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
CPU statement of what the GPU library computes.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import, call or link
it; the GPU library never does, and the two share no code (only the seeded
input generator in `cigen`, which holds none of the method's arithmetic).

What it computes, and from which passage of the paper:

* the many-body basis of Slater determinants (Sec. 2, many-body basis states
  built from single-particle states (n, l, j, m)), enumerated by brute force
  over particle subsets and sorted by an explicit canonical key;
* the Hamiltonian matrix H_ij = <Phi_i|H|Phi_j> (Sec. 2, the many-body
  Hamiltonian as a sparse symmetric matrix; Fig. 1, steps 10-14) by applying the
  second-quantised operator strings to each ket bit string one operator at a
  time and looking the image up in a hash map -- a different route from the
  XOR/popcount Slater-Condon evaluation on the GPU;
* the sparsity pattern as every pair whose bit strings differ in at most four
  single-particle states (Sec. 2.1), found by brute force over all pairs;
* the counts-to-offsets prefix sum (Sec. 2.2, the recurrence y_1 = 0,
  y_{i+1} = y_i + x_i);
* Y = H X with the half-stored matrix expanded to both triangles, and the
  lowest eigenvalues by LAPACK / ARPACK (Sec. 2, the lowest eigenvalues of H;
  Fig. 1 step 15);
* `count_difference` of the index-tuple representation (Sec. 2.1, Listing 1 as
  a description).

Pins that tie it to something other than itself live in tests/test_oracle_*.py:
generating-function dimensions, class-pair nonzero counts, Jordan-Wigner Fock
space matrices, closed forms, the trace formula, LAPACK, symmetry and
conservation laws.
"""
from .ci_oracle import *  # noqa: F401,F403
