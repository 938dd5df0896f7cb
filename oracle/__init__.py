"""CPU oracle for Krylov time evolution of a spin-1/2 XXZ chain (test infrastructure).

This package is TEST INFRASTRUCTURE, not part of the product path.  Only the
test suite, the smoke check of the entry module and the CPU-baseline leg of the
benchmark may import it.  It shares no code, tables or helpers with the device
library: it is written from the paper (arXiv:1704.02770, Brenes, Varma,
Scardicchio, Girotto) in plain numpy/scipy, float64 / complex128 throughout,
favouring a form that can be checked against the paper by eye over speed.

Modules
  model        Sec. 2 "Models", Eq. (1): fields, bonds, Neel state.
  basis        Sec. 2 "Basis representation" and Sec. 3, Algorithms 2 and 3:
               the sorted integer basis, next-bit-permutation, section start,
               binary lookup.
  hamiltonian  Sec. 3 "Hamiltonian matrix construction": rows of H from bit
               operations plus lookup; exact-preallocation counts.
  exact        Sec. 2 Eqs. (2)-(3) and Sec. 4 Eq. for F(t): dense propagation.
  midsize      Same definition through scipy's expm_multiply (library routine).
  freefermion  Closed form of the return amplitude when the zz coupling is 0.
  krylov       Sec. 2 "Krylov subspace methods": Arnoldi + small exponential.
  gradient     Derivative of F(T) with respect to every on-site field.

Readings of the paper that the oracle fixes (model form, site/bit mapping,
boundary bonds) are listed at the top of `model`.
"""
