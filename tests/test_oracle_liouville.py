"""Pins of the Liouville-space oracle (Sec. ed:sec:Liouville, Eqs. ed:eq:lioutrafo, ed:eq:liousuperket,
App. F, with the anticommutator of the master equation Eq. ed:eq:lindbladme) beyond the trace and
decay identities of the trajectory tests: the analytic solutions of single-qubit amplitude damping
and dephasing, the superket map O' rho O -> (O' (x) O^T)|rho>> on random matrices, trace
preservation <<1|Lcal = 0 and Hermiticity preservation for random Hamiltonians and jumps."""
import numpy as np
import scipy.sparse as sp

import edinputs as E
from oracle import liouville as OLv

SM = np.array([[0, 0], [1, 0]], np.complex128)   # sigma^- = |down><up|, index 0 = up


def test_superket_map_app_f():
    """O' rho O as a matrix product equals (O' (x) O^T) acting on the row-major vec(rho)."""
    rng = np.random.default_rng(1)
    D = 8
    A, B, R = (rng.standard_normal((3, D, D)) + 1j * rng.standard_normal((3, D, D)))
    assert np.abs(OLv.superket(A @ R @ B) - np.kron(A, B.T) @ OLv.superket(R)).max() < 1e-12


def test_amplitude_damping_closed_form():
    """H = (w/2) sigma^z, L = sqrt(g) sigma^-: rho_00(t) = rho_00 e^{-g t} (the up population),
    rho_01(t) = rho_01 e^{-g t/2} e^{-i w t}, and the trace stays 1."""
    w, g, t = 0.8, 0.3, 1.7
    H = sp.csr_matrix(0.5 * w * E.SZ)
    rho0 = np.array([[0.6, 0.2 - 0.3j], [0.2 + 0.3j, 0.4]])
    vec, = OLv.evolve_states(H, [np.sqrt(g) * SM], OLv.superket(rho0), t, 1)[1:]
    rho = vec.reshape(2, 2)
    assert abs(rho[0, 0] - 0.6 * np.exp(-g * t)) < 1e-13
    assert abs(rho[0, 1] - rho0[0, 1] * np.exp(-0.5 * g * t) * np.exp(-1j * w * t)) < 1e-13
    assert abs(np.trace(rho) - 1.0) < 1e-13


def test_dephasing_closed_form():
    """L = sqrt(g) sigma^z: populations stay, coherences decay as e^{-2 g t}."""
    g, t = 0.25, 0.9
    rho0 = np.array([[0.3, 0.1 + 0.4j], [0.1 - 0.4j, 0.7]])
    vec, = OLv.evolve_states(sp.csr_matrix((2, 2), dtype=complex), [np.sqrt(g) * E.SZ], OLv.superket(rho0), t, 1)[1:]
    rho = vec.reshape(2, 2)
    assert abs(rho[0, 0] - 0.3) < 1e-14 and abs(rho[1, 1] - 0.7) < 1e-14
    assert abs(rho[0, 1] - rho0[0, 1] * np.exp(-2 * g * t)) < 1e-13


def test_trace_and_hermiticity_preservation():
    L = 3
    D = 1 << L
    rng = np.random.default_rng(4)
    desc = E.random_model(L, seed=2, hermitian=True)
    from oracle import hamiltonian as OH
    H = OH.hamiltonian_sparse(desc)
    jumps = [sp.csr_matrix(rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))) for _ in range(2)]
    Lc = OLv.liouvillian(H, jumps)
    one = OLv.superket(np.eye(D))
    assert np.abs(Lc.T @ one).max() < 1e-12          # <<1| Lcal = 0: tr(Lcal rho) = 0 for all rho
    X = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    rho = X @ X.conj().T
    out = (Lc @ OLv.superket(rho)).reshape(D, D)
    assert np.abs(out - out.conj().T).max() < 1e-12
