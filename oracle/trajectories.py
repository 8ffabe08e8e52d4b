"""Quantum trajectories for the Lindblad equation (Sec. ed:sec:QT, after Dalibard et al.).

Per trajectory, with H_eff = H - (i/2) sum_nu L_nu^dagger L_nu:
  1. draw r; evolve the unnormalised state under H_eff until |psi|^2 drops to r;
  2. draw r_kappa; p_nu = <psi|L_nu^dagger L_nu|psi>, P_nu = cumulative p normalised by the sum;
  3. apply L_kappa with P_{kappa-1} < r_kappa <= P_kappa, renormalise, and go back to 1.
Readings where the paper is silent: the threshold is on the squared norm; the crossing time is
solved exactly inside the Krylov step (the step's basis gives psi(t + tau) for any tau, so the
root is found in the small space); after a jump the step's remainder is propagated and the
dt grid continues. Random numbers: numpy's Philox4x64-10 with key (seed, trajectory id);
draw n is 64-bit word n of the stream (counter block n//4 + 1, word n%4) mapped to
u = ((w >> 11) + 1) 2^-53 in (0, 1]. Each jump consumes one r_kappa and one new r.
"""
import numpy as np
import scipy.linalg as sla
import scipy.optimize as sopt
import scipy.sparse as sp

from .krylov import krylov_basis
from .observables import sz_all


class PhiloxDraws:
    """Uniform draws in (0, 1] from numpy's Philox4x64-10, key = (seed, trajectory id)."""

    def __init__(self, seed, traj_id):
        self.gen = np.random.Philox(key=[int(seed), int(traj_id)])
        self.n = 0

    def raw(self):
        self.n += 1
        return int(self.gen.random_raw())

    def uniform(self):
        return ((self.raw() >> 11) + 1) * 2.0 ** -53


def effective_hamiltonian(H, jump_ops):
    """H_eff = H - (i/2) sum_nu L_nu^dagger L_nu (the standard reading of Sec. ed:sec:QT)."""
    acc = sp.csr_matrix(H.shape, dtype=np.complex128)
    for Lnu in jump_ops:
        acc = acc + (Lnu.conj().T @ Lnu)
    return (H - 0.5j * acc).tocsr()


def trajectory(H, jump_ops, psi0, dt, n_steps, out_stride, seed, traj_id, m_max=30, tol=1e-12):
    """One quantum trajectory. Returns dict with the normalised <sigma^z_k> at output times
    t = n dt out_stride (n = 0..n_steps//out_stride), the jump list [(t, site index)], and the
    number of random draws used."""
    L = int(np.log2(H.shape[0]))
    Heff = effective_hamiltonian(H, jump_ops)
    mv = lambda v: Heff @ v
    rng = PhiloxDraws(seed, traj_id)
    psi = psi0 / np.linalg.norm(psi0)
    r = rng.uniform()
    out = [sz_all(psi, L)]
    jumps = []
    t = 0.0
    for step in range(n_steps):
        tau_left = dt
        while tau_left > 0.0:
            V, T, beta0, m = krylov_basis(mv, psi, m_max, tau_left, tol, hermitian=False)

            def state(tau):
                return beta0 * (V @ sla.expm(-1j * tau * T)[:, 0])

            def lognorm2(tau):
                u = sla.expm(-1j * tau * T)[:, 0]
                return np.log(beta0 ** 2 * np.vdot(u, u).real)

            if lognorm2(tau_left) > np.log(r):
                psi = state(tau_left)
                t += tau_left
                break
            tau = sopt.brentq(lambda x: lognorm2(x) - np.log(r), 0.0, tau_left, xtol=1e-15, rtol=1e-15)
            psi = state(tau)
            t += tau
            p = np.array([np.linalg.norm(Lnu @ psi) ** 2 for Lnu in jump_ops])
            P = np.cumsum(p) / p.sum()
            rk = rng.uniform()
            kappa = int(np.searchsorted(P, rk, side="left"))   # P[kappa-1] < rk <= P[kappa]
            kappa = min(kappa, len(P) - 1)
            psi = jump_ops[kappa] @ psi
            psi /= np.linalg.norm(psi)
            jumps.append((t, kappa))
            r = rng.uniform()
            tau_left -= tau
        if (step + 1) % out_stride == 0:
            out.append(sz_all(psi, L))
    return {"sz": np.array(out), "jumps": jumps, "draws": rng.n, "psi": psi}


def lowering_jumps(L, gamma):
    """L_k = sqrt(gamma) sigma^-_k for k = 1..L (site index order nu = k - 1)."""
    from .hamiltonian import site_operator
    sm = np.array([[0, 0], [1, 0]], np.complex128)
    return [np.sqrt(gamma) * site_operator(sm, k, L) for k in range(1, L + 1)]
