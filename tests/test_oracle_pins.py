"""Pins of the CPU oracle against closed forms, brute force, invariants and library special
cases (no GPU)."""
import numpy as np
import pytest
import scipy.linalg as sla

import edinputs as E
from oracle import hamiltonian as OH
from oracle import lanczos as OL
from oracle import krylov as OK
from oracle import observables as OO
from tests import closed_forms as CF


# ---------------------------------------------------------------- Hamiltonian (Eq. genericH)
@pytest.mark.parametrize("L", [2, 3, 5])
def test_H_matches_bruteforce_elements(L):
    desc = E.random_model(L, seed=100 + L, hermitian=False)
    H = OH.hamiltonian_sparse(desc).toarray()
    D = 1 << L
    B = np.array([[CF.brute_matrix_element(desc, x, y) for y in range(D)] for x in range(D)])
    assert np.max(np.abs(H - B)) < 1e-14


def test_dense_equals_sparse_and_hermitian():
    desc = E.random_model(6, seed=7)
    Hs = OH.hamiltonian_sparse(desc).toarray()
    Hd = OH.hamiltonian_dense(desc)
    assert np.max(np.abs(Hs - Hd)) < 1e-13
    assert np.max(np.abs(Hs - Hs.conj().T)) < 1e-14


def test_apply_H_entries_bruteforce():
    desc = E.xxz(7, 1.0, 0.5, E.random_fields(7, 2))
    psi = E.random_state(7, 11)
    y = OH.apply_H(desc, psi)
    for x in [0, 1, 5, 64, 127, 77]:
        assert abs(y[x] - CF.brute_apply_entry(desc, psi, x)) < 1e-13


def test_site_order_is_most_significant_digit():
    # sigma^z on site 1 only: sign flips at the top bit
    L = 3
    desc = E.ModelDesc(L, site_ops=[E.SZ], site_coef=[[1.0, 0, 0]], bond_ops=np.zeros((0, 4, 4)),
                       bond_coef=np.zeros((0, L - 1)))
    d = np.real(np.diag(OH.hamiltonian_sparse(desc).toarray()))
    assert list(d) == [1, 1, 1, 1, -1, -1, -1, -1]


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("L", [2, 3, 4, 6, 8])
def test_tfim_bdg_matches_bruteforce(L):
    for g in (0.3, 1.0, 2.5):
        H = OH.hamiltonian_dense(E.tfim(L, g))
        e0 = np.linalg.eigvalsh(H)[0]
        assert abs(e0 - CF.tfim_bdg_ground_energy(L, 1.0, g)) < 1e-12 * L


def test_xxz_two_site_closed_form():
    J, delta, h1, h2 = 1.0, 0.5, 0.3, -0.2
    H = OH.hamiltonian_dense(E.xxz(2, J, delta, [h1, h2]))
    ev = np.linalg.eigvalsh(H)
    assert np.allclose(ev, CF.xxz_two_site_spectrum(J, delta, h1, h2), atol=1e-14)
    assert np.allclose(ev, [-2.5615528128088303, 0.4, 0.6, 1.5615528128088303], atol=1e-13)


# ---------------------------------------------------------------- Lanczos ground state
@pytest.mark.parametrize("L", [4, 8, 10])
def test_lanczos_vs_eigvalsh(L):
    desc = E.xxz(L, 1.0, 0.5, E.random_fields(L, 2))
    H = OH.hamiltonian_sparse(desc)
    e_ex, v_ex = np.linalg.eigh(H.toarray())
    E0, psi, info = OL.lanczos_ground(lambda v: H @ v, E.random_state(L, 3), tol=1e-10)
    assert abs(E0 - e_ex[0]) <= 1e-10 * abs(e_ex[0])
    assert 1 - abs(np.vdot(psi, v_ex[:, 0])) < 1e-9
    assert info["residual"] < 1e-9


def test_lanczos_tfim_L14_bdg():
    L = 14
    H = OH.hamiltonian_sparse(E.tfim(L, 1.0))
    E0, psi, info = OL.lanczos_ground(lambda v: H @ v, E.random_state(L, 1), tol=1e-10, max_iter=200)
    ref = CF.tfim_bdg_ground_energy(L, 1.0, 1.0)
    assert abs(E0 - ref) <= 1e-10 * abs(ref)
    assert abs(E0 - (-17.47100405473177)) < 1e-9
    e_sh, _ = OL.ground_state_eigsh(H)
    assert abs(e_sh - ref) <= 1e-10 * abs(ref)


def test_lanczos_breakdown_on_eigenvector():
    L = 6
    H = OH.hamiltonian_sparse(E.tfim(L, 0.0))
    v0 = E.product_state(L, 0)                    # all up is an eigenstate at g = 0
    E0, psi, info = OL.lanczos_ground(lambda v: H @ v, v0)
    assert info["iters"] == 1 and abs(E0 + (L - 1)) < 1e-14


# ---------------------------------------------------------------- Krylov time step
@pytest.mark.parametrize("L,herm", [(6, True), (8, True), (6, False)])
def test_krylov_vs_expm(L, herm):
    desc = E.random_model(L, seed=30 + L, hermitian=herm)
    H = OH.hamiltonian_sparse(desc)
    psi = E.random_state(L, 5)
    dt = 0.05
    exact = OK.expm_step(H.toarray(), psi, dt)
    kr, m = OK.krylov_step(lambda v: H @ v, psi, dt, m_max=30, tol=1e-12, hermitian=herm)
    assert np.linalg.norm(kr - exact) < 1e-11
    assert 1 < m < 30


def test_krylov_norm_energy_conserved_and_eigenstate_phase():
    L = 10
    desc = E.tfim(L, 0.5)
    H = OH.hamiltonian_sparse(desc)
    psi = E.product_state(L, 0)
    e0 = OO.energy(H, psi)
    assert e0 == -(L - 1)
    for _ in range(20):
        psi, m = OK.krylov_step(lambda v: H @ v, psi, 0.05, m_max=20, tol=1e-10)
    assert abs(OO.norm(psi) - 1) < 1e-10
    assert abs(OO.energy(H, psi) - e0) < 1e-9
    sz = OO.sz_all(psi, L)
    assert np.allclose(sz, sz[::-1], atol=1e-10)           # reflection symmetry of the quench
    H0 = OH.hamiltonian_sparse(E.tfim(L, 0.0))
    v, m = OK.krylov_step(lambda v: H0 @ v, E.product_state(L, 0), 0.3)
    assert m == 1 and abs(v[0] - np.exp(1j * 0.3 * (L - 1))) < 1e-14


# ---------------------------------------------------------------- observables
def test_sz_all_product_and_operator_definition():
    L = 5
    idx = E.neel_index(L)
    assert np.array_equal(OO.sz_all(E.product_state(L, idx), L), [1, -1, 1, -1, 1])
    psi = E.random_state(L, 9, normalise=False)
    sz = OO.sz_all(psi, L)
    for k in range(1, L + 1):
        op = OH.site_operator(E.SZ, k, L)
        assert abs(sz[k - 1] - np.vdot(psi, op @ psi).real / np.vdot(psi, psi).real) < 1e-14


def test_entropy_pins():
    L = 8
    assert abs(OO.bond_entropy(E.product_state(L, 37), L, 4)) < 1e-14
    # Bell pair across the cut between sites 4 and 5, the rest up
    psi = np.zeros(1 << L, np.complex128)
    psi[E.basis_index([1, 1, 1, 1, 1, 1, 1, 1])] = 1 / np.sqrt(2)
    psi[E.basis_index([1, 1, 1, 0, 0, 1, 1, 1])] = 1 / np.sqrt(2)
    assert abs(OO.bond_entropy(psi, L, 4) - np.log(2)) < 1e-14
    # spectrum equals the eigenvalues of M M^dagger
    psi = E.random_state(10, 4)
    M = psi.reshape(32, 32)
    ev = np.sort(np.linalg.eigvalsh(M @ M.conj().T))[::-1]
    assert np.allclose(ev, OO.schmidt_spectrum(psi, 10, 5), atol=1e-15)
    # random state: Page value (l/2... ) within a loose band
    psi = E.random_state(14, 5)
    S = OO.bond_entropy(psi, 14, 7)
    assert abs(S - (7 * np.log(2) - 0.5)) < 0.05


# ---------------------------------------------------------------- random numbers
def test_philox_stream_matches_definition():
    from oracle.trajectories import PhiloxDraws
    d = PhiloxDraws(seed=4, traj_id=123)
    words = [d.raw() for _ in range(12)]
    ref = []
    for blk in range(1, 4):
        ref += CF.philox4x64_10([blk, 0, 0, 0], [4, 123])
    assert words == ref
    d = PhiloxDraws(seed=0, traj_id=0)
    u = [d.uniform() for _ in range(1000)]
    assert min(u) > 0 and max(u) <= 1


def test_apply_H_entries_matches_sparse():
    for desc in (E.random_model(7, seed=3, hermitian=False), E.tfim(9, 0.7), E.xxz(8, 1.0, 0.5, E.random_fields(8, 1))):
        psi = E.random_state(desc.L, 2)
        y = OH.apply_H(desc, psi)
        xs = np.arange(1 << desc.L)
        assert np.max(np.abs(OH.apply_H_entries(desc, psi, xs) - y)) < 1e-13
