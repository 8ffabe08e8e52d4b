"""CPU oracle for the exact-diagonalisation hot path (test infrastructure only).

This package is the plain, slow, obviously correct reference that the HIP library is checked
against. It is imported only by the tests, by the smoke check and by the CPU-baseline leg of the
benchmark; the library itself never calls it and shares no code with it. Everything is float64 /
complex128 numpy + scipy, written from the paper's definitions:

  hamiltonian  H from Kronecker products of the rule sets (Sec. ed:sec:statics, Eq. ed:eq:genericH, App. A)
  lanczos      ground state: eigsh as the paper does (Sec. ed:sec:statics) and textbook Lanczos
  krylov       Krylov time step (Sec. ed:sec:krylov) and the exact propagator (Sec. ed:sec:expm)
  observables  <sigma^z_k>, energy, norm (Sec. ed:sec:meas), bond entropy (Sec. ed:sec:meas, S(l))
  rdm          single-site and two-site reduced density matrices (Sec. ed:sec:meas), trace distance and
               the error measures of the convergence study (Sec. ed:sec:conv)
  trotter      Suzuki-Trotter layers of order 2 and 4 (Sec. ed:sec:trotter)
  philox       (none: the oracle draws with numpy's Philox4x64-10 bit generator)
  trajectories quantum trajectories (Sec. ed:sec:QT)
  liouville    Liouville-space superket evolution (Sec. ed:sec:Liouville, App. F, corrected form)
  adjoint      dense gradient of a final-time observable w.r.t. sliced bond couplings

Functions whose result has no independent pin say "parity unpinned" in their docstring.
"""
