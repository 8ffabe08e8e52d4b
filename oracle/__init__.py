"""CPU oracle for the exact-diagonalisation hot path (test infrastructure only).

This package is the plain, slow, obviously correct reference that the HIP library is checked
against. It is imported only by the tests, by the smoke check and by the CPU-baseline leg of the
benchmark; the library itself never calls it and shares no code with it. Everything is float64 /
complex128 numpy + scipy, written from the paper's definitions:

  hamiltonian  H from Kronecker products of the rule sets (Sec. II, Eq. ed:eq:genericH, App. A)
  lanczos      ground state: eigsh as the paper does (Sec. II statics) and textbook Lanczos
  krylov       Krylov time step (Sec. ed:sec:krylov) and the exact propagator (Sec. ed:sec:expm)
  observables  <sigma^z_k>, energy, norm (Sec. IV), bond entropy (Sec. IV, S(l))
  rdm          single-site and two-site reduced density matrices (Sec. IV), trace distance and
               the error measures of the convergence study (Sec. V)
  trotter      Suzuki-Trotter layers of order 2 and 4 (Sec. ed:sec:trotter)
  philox       (none: the oracle draws with numpy's Philox4x64-10 bit generator)
  trajectories quantum trajectories (Sec. VI.A)
  liouville    Liouville-space superket evolution (Sec. VI.B, App. F, corrected form)
  adjoint      dense gradient of a final-time observable w.r.t. sliced bond couplings

Functions whose result has no independent pin say "parity unpinned" in their docstring.
"""
