"""Pins of the trajectory, Liouville and adjoint parts of the oracle (no GPU)."""
import numpy as np
import pytest

import edinputs as E
from oracle import hamiltonian as OH
from oracle import krylov as OK
from oracle import liouville as OLv
from oracle import trajectories as OT
from oracle import adjoint as OA


def _xxz_open(L, gamma=0.1):
    H = OH.hamiltonian_sparse(E.xxz(L, 1.0, 1.0))
    return H, OT.lowering_jumps(L, gamma)


@pytest.mark.parametrize("L,traj", [(4, 0), (6, 3), (6, 7)])
def test_trajectory_jump_times_closed_form(L, traj):
    """From the Neel state with [H, N_up] = 0 the no-jump norm is exp(-gamma n t), so each
    jump time follows from the draws alone: t_j = t_{j-1} - ln(r_j)/(gamma n_{j-1})."""
    gamma, dt, steps = 0.1, 0.01, 500
    H, jumps = _xxz_open(L, gamma)
    psi0 = E.product_state(L, E.neel_index(L))
    res = OT.trajectory(H, jumps, psi0, dt, steps, 10, seed=4, traj_id=traj)
    draws = OT.PhiloxDraws(4, traj)
    n = L // 2
    t = 0.0
    expect = []
    r = draws.uniform()
    while n > 0:
        t = t - np.log(r) / (gamma * n)
        if t > dt * steps:
            break
        draws.uniform()          # the jump-choice draw
        r = draws.uniform()
        n -= 1
        expect.append(t)
    got = [tj for tj, _ in res["jumps"]]
    assert len(got) == len(expect)
    assert np.allclose(got, expect, rtol=1e-11, atol=1e-11)
    # the chosen site was up before the jump and is down afterwards; sz sums track N_up
    assert len({k for _, k in res["jumps"]}) == len(got)


def test_liouville_trace_and_decay_identity():
    L, gamma = 4, 0.1
    H, jumps = _xxz_open(L, gamma)
    psi0 = E.product_state(L, E.neel_index(L))
    rho0 = np.outer(psi0, psi0.conj())
    times = [0.0, 0.5, 1.0, 2.5, 5.0]
    for t, (sz, tr) in zip(times, OLv.evolve_sz(H, jumps, rho0, times)):
        assert abs(tr - 1) < 1e-12
        # N_up(t) = N_up(0) exp(-gamma t)  (the paper's decay identity, Eq. ed:eq:pjjexp)
        assert abs(sz.sum() - L * (np.exp(-gamma * t) - 1)) < 1e-12


def test_liouville_reduces_to_pure_state_at_zero_rate():
    L = 4
    H = OH.hamiltonian_sparse(E.xxz(L, 1.0, 0.5, [0.1, -0.3, 0.2, 0.05]))
    psi0 = E.random_state(L, 8)
    rho0 = np.outer(psi0, psi0.conj())
    (sz, tr), = OLv.evolve_sz(H, [], rho0, [0.7])
    psi = OK.expm_step(H.toarray(), psi0, 0.7)
    from oracle.observables import sz_all
    assert np.allclose(sz, sz_all(psi, L), atol=1e-12)


def test_trajectory_ensemble_vs_liouville():
    """Ensemble mean of <sigma^z_k>(t) over trajectories agrees with the exact Lindblad
    solution within 4 standard errors (law of large numbers, Sec. ed:sec:opencavities)."""
    L, gamma, dt, steps, stride, N = 4, 0.1, 0.05, 40, 10, 160
    H, jumps = _xxz_open(L, gamma)
    psi0 = E.product_state(L, E.neel_index(L))
    rho0 = np.outer(psi0, psi0.conj())
    runs = np.array([OT.trajectory(H, jumps, psi0, dt, steps, stride, seed=9, traj_id=t, tol=1e-10)["sz"]
                     for t in range(N)])
    mean = runs.mean(axis=0)
    se = runs.std(axis=0, ddof=1) / np.sqrt(N) + 1e-3
    times = [i * dt * stride for i in range(steps // stride + 1)]
    exact = np.array([sz for sz, _ in OLv.evolve_sz(H, jumps, rho0, times)])
    assert np.all(np.abs(mean - exact) < 4 * se)


def _adjoint_case(L, S, seed=5):
    tmpl = E.xxz_bond_scaled(L, 0.5, np.ones(L - 1))
    J = E.adjoint_couplings(S, L - 1, seed)
    psi0 = E.product_state(L, E.neel_index(L))
    w = np.array([(-1) ** k for k in range(L)]) / L
    return tmpl, J, psi0, w


def test_adjoint_frechet_vs_finite_differences():
    tmpl, J, psi0, w = _adjoint_case(5, 4)
    Delta = 0.1
    loss, g = OA.gradient_frechet(tmpl, J, psi0, Delta, w)
    assert abs(loss - OA.loss_only(tmpl, J, psi0, Delta, w)) < 1e-15
    h = 1e-6
    fd = np.zeros_like(g)
    for s in range(J.shape[0]):
        for b in range(J.shape[1]):
            Jp, Jm = J.copy(), J.copy()
            Jp[s, b] += h
            Jm[s, b] -= h
            fd[s, b] = (OA.loss_only(tmpl, Jp, psi0, Delta, w) - OA.loss_only(tmpl, Jm, psi0, Delta, w)) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-9
    assert np.max(np.abs(g)) > 1e-3


def test_adjoint_eig_vs_frechet():
    tmpl, J, psi0, w = _adjoint_case(6, 3)
    l1, g1 = OA.gradient_frechet(tmpl, J, psi0, 0.1, w)
    l2, g2 = OA.gradient_eig(tmpl, J, psi0, 0.1, w)
    assert abs(l1 - l2) < 1e-14
    assert np.max(np.abs(g1 - g2)) < 1e-13
    # Neel start: staggered magnetisation is 1 at t = 0
    assert abs(OA.loss_only(tmpl, J[:0], psi0, 0.1, w) - 1.0) < 1e-15
