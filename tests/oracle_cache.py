"""Oracle results that several GPU test files compare with, computed once per test process."""
import functools

import edinputs as E
from oracle import hamiltonian as OH
from oracle import lanczos as OL


@functools.lru_cache(maxsize=None)
def xxz_fields_ground(L):
    """Ground state of the XXZ chain with random fields (J = 1, Delta = 0.5, h ~ U[-0.5, 0.5],
    seed 2) from the oracle's sparse H and ARPACK (the paper's sparse statics, Sec. ed:sec:statics).
    Returns (desc, H, E0, psi0)."""
    desc = E.xxz(L, 1.0, 0.5, E.random_fields(L, 2))
    H = OH.hamiltonian_sparse(desc)
    e0, psi = OL.ground_state_eigsh(H, tol=1e-14)
    return desc, H, e0, psi
