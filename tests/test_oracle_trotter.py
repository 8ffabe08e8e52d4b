"""Pins of the Trotter oracle (Sec. ed:sec:trotter; Eqs. ed:eq:trotter2, ed:eq:trotter4,
ed:eq:trotter4c) against facts that do not come from its own code: exactness when all terms
commute, exactness for a single bond, the dense layer products at L = 3 built from the
independently pinned Kronecker Hamiltonian, the convergence orders 2 and 4 against the exact
propagator, and unitarity."""
import numpy as np
import pytest
import scipy.linalg as sla

import edinputs as E
from oracle import hamiltonian as OH
from oracle import trotter as OT


def _exact(desc, psi, t):
    return sla.expm(-1j * t * OH.hamiltonian_dense(desc)) @ psi


@pytest.mark.parametrize("order", [2, 4])
def test_commuting_terms_are_exact(order):
    """All terms built from sigma^x commute (and so do H_o and H_e): any splitting is exact."""
    L = 7
    rng = np.random.default_rng(1)
    desc = E.ModelDesc(L, site_ops=[E.SX], site_coef=rng.uniform(-1, 1, (1, L)),
                       bond_ops=[E.SXSX], bond_coef=rng.uniform(-1, 1, (1, L - 1)))
    psi0 = E.random_state(L, 2)
    psi, _ = OT.evolve(desc, psi0, 0.3, 4, order)
    assert np.linalg.norm(psi - _exact(desc, psi0, 1.2)) < 1e-12


@pytest.mark.parametrize("order", [2, 4])
def test_single_bond_is_exact(order):
    """L = 2: H is one bond of H_o (H_e is empty), so each step is exp(-i dt H) exactly."""
    desc = E.random_model(2, seed=3, hermitian=False)
    psi0 = E.random_state(2, 1)
    psi, _ = OT.evolve(desc, psi0, 0.37, 3, order)
    assert np.linalg.norm(psi - _exact(desc, psi0, 1.11)) < 1e-13


def test_three_sites_against_dense_layers():
    """L = 3: H_o = bond (1,2) + site 1 + site 2 / 2, H_e = bond (2,3) + site 2 / 2 + site 3, built
    as dense 8x8 matrices by the Kronecker oracle; the order-2 step is their exponential product."""
    L = 3
    desc = E.random_model(L, seed=7, hermitian=True)

    def part(bond_mask, site_w):
        return E.ModelDesc(L, site_ops=desc.site_ops, site_coef=desc.site_coef * np.array(site_w)[None, :],
                           bond_ops=desc.bond_ops, bond_coef=desc.bond_coef * np.array(bond_mask)[None, :])

    Ho = OH.hamiltonian_dense(part([1.0, 0.0], [1.0, 0.5, 0.0]))
    He = OH.hamiltonian_dense(part([0.0, 1.0], [0.0, 0.5, 1.0]))
    assert np.allclose(Ho + He, OH.hamiltonian_dense(desc), atol=1e-14)
    dt = 0.21
    psi0 = E.random_state(L, 4)
    ref = sla.expm(-0.5j * dt * He) @ (sla.expm(-1j * dt * Ho) @ (sla.expm(-0.5j * dt * He) @ psi0))
    psi, _ = OT.evolve(desc, psi0, dt, 1, 2)
    assert np.linalg.norm(psi - ref) < 1e-14


@pytest.mark.parametrize("order,lo,hi", [(2, 3.8, 4.2), (4, 15.0, 17.0)])
def test_convergence_order(order, lo, hi):
    """Global error at fixed T against exp(-i T H): halving dt divides it by 2^order."""
    L = 8
    desc = E.xxz(L, 1.0, 0.5, E.random_fields(L, 2))
    desc = E.ModelDesc(L, site_ops=np.concatenate([desc.site_ops, [E.SX]]),
                       site_coef=np.concatenate([desc.site_coef, np.full((1, L), 0.3)]),
                       bond_ops=desc.bond_ops, bond_coef=desc.bond_coef)
    psi0 = E.random_state(L, 5)
    ex = _exact(desc, psi0, 1.0)
    errs = [np.linalg.norm(OT.evolve(desc, psi0, dt, int(round(1.0 / dt)), order)[0] - ex) for dt in (0.1, 0.05)]
    assert lo < errs[0] / errs[1] < hi, errs


@pytest.mark.parametrize("order", [2, 4])
def test_unitary(order):
    L = 9
    desc = E.tfim(L, 0.7)
    psi0 = E.random_state(L, 6)
    psi, states = OT.evolve(desc, psi0, 0.05, 12, order)
    assert all(abs(np.linalg.norm(s) - 1.0) < 1e-13 for s in states)
