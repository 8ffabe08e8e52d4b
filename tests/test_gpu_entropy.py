"""GPU parity of the bond entropy (Sec. IV) against the oracle's SVD of the reshaped state.

Tolerance: both sides resolve the Schmidt spectrum to about 1e-16 absolute, so eigenvalues below
that are noise; their share of S is at most n * 1e-16 * |log 1e-16| ~ 3e-11 at n = 8192. The
bound used is 1e-10 relative (plus 1e-12 absolute for S ~ 0)."""
import numpy as np
import pytest
import torch

import edinputs as E
import paper_1802_10052_amd as P
from oracle import hamiltonian as OH
from oracle import lanczos as OL
from oracle import observables as OO

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


@pytest.mark.parametrize("L,l", [(2, 1), (4, 2), (7, 3), (7, 5), (10, 5), (13, 4), (14, 7), (16, 8), (17, 9), (19, 6)])
def test_entropy_random_states(L, l):
    print(f"entropy L={L} l={l}", flush=True)
    psi = E.random_state(L, 30 + L, normalise=False)
    S, spec = P.entropy(dev(psi), L, l, spectrum=True)
    ref = OO.schmidt_spectrum(psi, L, l)
    Sref = OO.bond_entropy(psi, L, l)
    assert abs(S - Sref) <= 1e-10 * abs(Sref) + 1e-12
    assert np.max(np.abs(spec - ref)) < 1e-13


def test_entropy_special_states():
    L = 12
    S = P.entropy(dev(E.product_state(L, 1234)), L, 6)
    assert abs(S) < 1e-13
    psi = np.zeros(1 << L, np.complex128)
    up = [1] * L
    bell = [1] * 5 + [0, 0] + [1] * 5
    psi[E.basis_index(up)] = 1 / np.sqrt(2)
    psi[E.basis_index(bell)] = 1 / np.sqrt(2)
    assert abs(P.entropy(dev(psi), L, 6) - np.log(2)) < 1e-13
    assert abs(P.entropy(dev(psi), L, 0)) < 1e-14 and abs(P.entropy(dev(psi), L, L)) < 1e-14


def test_entropy_ground_state_L20():
    """Half-chain entropy of the XXZ ground state (Delta = 0.5, random fields) at L = 20 against
    the oracle's SVD of the oracle's own ground state."""
    L = 20
    print("entropy ground state L=20", flush=True)
    desc = E.xxz(L, 1.0, 0.5, E.random_fields(L, 2))
    H = OH.hamiltonian_sparse(desc)
    e0, psi = OL.ground_state_eigsh(H, tol=1e-14)
    S = P.entropy(dev(psi), L, L // 2)
    Sref = OO.bond_entropy(psi, L, L // 2)
    assert abs(S - Sref) <= 1e-10 * abs(Sref)
