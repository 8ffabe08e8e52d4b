"""Pins of the reduced-density-matrix oracle (Sec. ed:sec:meas) and of the error measures of the
convergence study (Sec. ed:sec:conv, Eqs. ed:eq:erhoi, ed:eq:erhoij, ed:eq:convrate) against facts that do
not come from its reshape/transpose code: entries recomputed by a loop over basis indices with
bit arithmetic, closed forms for product, GHZ and W states, partial-trace consistency, the
Bloch-vector form of the 2x2 trace distance, pure-state distances, and the convergence orders of
the Trotter propagators measured with eps_local and eps_corr."""
import numpy as np
import pytest
import scipy.linalg as sla

import edinputs as E
from oracle import hamiltonian as OH
from oracle import rdm as OR
from oracle import trotter as OT


def brute_rdm2(psi, L, k, j):
    """rho_{k,j}[(a,b),(a',b')] = sum over x with bits (a, b) at sites (k, j) of psi[x] psi*[x'],
    x' = x with those bits set to (a', b'); site k sits at bit L-k."""
    pk, pj = L - k, L - j
    rho = np.zeros((4, 4), complex)
    for x in range(1 << L):
        a, b = (x >> pk) & 1, (x >> pj) & 1
        for a2 in range(2):
            for b2 in range(2):
                y = (x & ~((1 << pk) | (1 << pj))) | (a2 << pk) | (b2 << pj)
                rho[2 * a + b, 2 * a2 + b2] += psi[x] * np.conj(psi[y])
    return rho


def test_two_site_entries_brute_force():
    L = 5
    psi = E.random_state(L, 3) * 1.7   # unnormalised on purpose
    rho2 = OR.rdm2_all(psi, L)
    for k in range(1, L + 1):
        for j in range(k + 1, L + 1):
            assert np.abs(rho2[OR.pair_index(k, j, L)] - brute_rdm2(psi, L, k, j)).max() < 1e-14


def test_single_site_entries_brute_force():
    L = 6
    psi = E.random_state(L, 4)
    rho1 = OR.rdm1_all(psi, L)
    for k in range(1, L + 1):
        p = L - k
        ref = np.zeros((2, 2), complex)
        for x in range(1 << L):
            a = (x >> p) & 1
            ref[a, a] += abs(psi[x]) ** 2
            ref[a, 1 - a] += psi[x] * np.conj(psi[x ^ (1 << p)])
        assert np.abs(rho1[k - 1] - ref).max() < 1e-15


def test_product_state_closed_form():
    L = 6
    rng = np.random.default_rng(5)
    phis = [v / np.linalg.norm(v) for v in rng.standard_normal((L, 2)) + 1j * rng.standard_normal((L, 2))]
    psi = phis[0]
    for v in phis[1:]:
        psi = np.kron(psi, v)
    rho1, rho2 = OR.rdm1_all(psi, L), OR.rdm2_all(psi, L)
    for k in range(1, L + 1):
        assert np.abs(rho1[k - 1] - np.outer(phis[k - 1], phis[k - 1].conj())).max() < 1e-15
        for j in range(k + 1, L + 1):
            v = np.kron(phis[k - 1], phis[j - 1])
            assert np.abs(rho2[OR.pair_index(k, j, L)] - np.outer(v, v.conj())).max() < 1e-15


def test_ghz_and_w_closed_forms():
    L = 7
    ghz = np.zeros(1 << L, complex)
    ghz[0] = ghz[-1] = 1 / np.sqrt(2)
    for r in OR.rdm1_all(ghz, L):
        assert np.abs(r - np.eye(2) / 2).max() < 1e-15
    for r in OR.rdm2_all(ghz, L):
        assert np.abs(r - np.diag([0.5, 0, 0, 0.5])).max() < 1e-15
    w = np.zeros(1 << L, complex)
    w[[1 << p for p in range(L)]] = 1 / np.sqrt(L)   # one down spin (index 1) anywhere
    ref = np.zeros((4, 4))
    ref[0, 0] = (L - 2) / L
    ref[1:3, 1:3] = 1 / L
    for r in OR.rdm2_all(w, L):
        assert np.abs(r - ref).max() < 1e-15
    for r in OR.rdm1_all(w, L):
        assert np.abs(r - np.diag([(L - 1) / L, 1 / L])).max() < 1e-15


def test_properties_and_partial_traces():
    L = 8
    psi = E.random_state(L, 6)
    rho1, rho2 = OR.rdm1_all(psi, L), OR.rdm2_all(psi, L)
    for k in range(1, L + 1):
        for j in range(k + 1, L + 1):
            r = rho2[OR.pair_index(k, j, L)].reshape(2, 2, 2, 2)
            assert np.abs(np.einsum("abcb->ac", r) - rho1[k - 1]).max() < 1e-15
            assert np.abs(np.einsum("abad->bd", r) - rho1[j - 1]).max() < 1e-15
    for r in list(rho1) + list(rho2):
        assert np.abs(r - r.conj().T).max() < 1e-15
        assert np.linalg.eigvalsh(r).min() > -1e-15
        assert abs(np.trace(r) - 1.0) < 1e-14


def test_trace_distance_bloch_and_pure_states():
    rng = np.random.default_rng(7)
    sig = [E.SX, E.SY, E.SZ]
    for _ in range(20):
        r1, r2 = [v / max(1.0, np.linalg.norm(v)) for v in rng.uniform(-1, 1, (2, 3))]
        a = 0.5 * (np.eye(2) + sum(c * s for c, s in zip(r1, sig)))
        b = 0.5 * (np.eye(2) + sum(c * s for c, s in zip(r2, sig)))
        assert abs(OR.trace_distance(a, b) - 0.5 * np.linalg.norm(r1 - r2)) < 1e-15
    for _ in range(10):
        u, v = [x / np.linalg.norm(x) for x in rng.standard_normal((2, 4)) + 1j * rng.standard_normal((2, 4))]
        D = OR.trace_distance(np.outer(u, u.conj()), np.outer(v, v.conj()))
        assert abs(D - np.sqrt(1 - abs(np.vdot(u, v)) ** 2)) < 1e-14
    assert OR.trace_distance(np.diag([1.0, 0, 0, 0]), np.diag([0, 1.0, 0, 0])) == 1.0


@pytest.mark.parametrize("order,lo,hi", [(2, 1.8, 2.2), (4, 3.6, 4.4)])
def test_convergence_rate_of_trotter_errors(order, lo, hi):
    """eps_local and eps_corr of the Trotter states against the matrix exponential (ME) at
    T = 1: the rate of Eq. ed:eq:convrate with alpha = 2 is the order of the splitting."""
    L = 8
    desc = E.tfim(L, 0.9)
    psi0 = E.random_state(L, 2)
    ex = sla.expm(-1j * OH.hamiltonian_dense(desc)) @ psi0
    r1x, r2x = OR.rdm1_all(ex, L), OR.rdm2_all(ex, L)
    el, ec = [], []
    for dt in (0.1, 0.05):
        psi, _ = OT.evolve(desc, psi0, dt, int(round(1 / dt)), order)
        el.append(OR.eps_local(OR.rdm1_all(psi, L), r1x))
        ec.append(OR.eps_corr(OR.rdm2_all(psi, L), r2x))
    assert lo < OR.convergence_rate(el[0], el[1], 2.0) < hi, el
    assert lo < OR.convergence_rate(ec[0], ec[1], 2.0) < hi, ec
