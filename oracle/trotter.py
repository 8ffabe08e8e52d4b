"""Suzuki-Trotter time evolution of a pure state (Sec. ed:sec:trotter: Eqs. ed:eq:trotter1,
ed:eq:trotter2, ed:eq:trotter4 and the constants of Eq. ed:eq:trotter4c).

Test infrastructure: imported only by the tests, the smoke check and the CPU baseline of the
benchmark; it shares no code with the HIP library.

H = H_o + H_e: H_o holds the bond terms (k, k+1) with k odd (1-based sites), H_e those with k
even. Site terms are split over the two bonds a site belongs to, weight 1/2 each; a site that
belongs to one bond only (sites 1 and L of the open chain) keeps weight 1 in it. The two-site
terms inside H_o (or H_e) act on different sites and commute, so exp(-i t H_o) is the product of
the two-site propagators exp(-i t h_k), each contracted with legs k, k+1 of the state seen as a
rank-L tensor (site 1 = most significant digit).
"""
import numpy as np
import scipy.linalg as sla

# Eq. ed:eq:trotter4c
TAU3 = 1.0 / (2.0 * (4.0 - 4.0 ** (1.0 / 3.0)))
TAU1 = 1.0 - 8.0 * TAU3
TAU2 = 0.5 * (1.0 - 6.0 * TAU3)
TAU4 = 2.0 * TAU3

# Layer sequences: (which part of H, fraction of dt). Eq. ed:eq:trotter2 and Eq. ed:eq:trotter4.
SEQUENCE = {
    2: [("e", 0.5), ("o", 1.0), ("e", 0.5)],
    4: [("e", TAU3), ("o", TAU4), ("e", TAU4), ("o", TAU4), ("e", TAU2), ("o", TAU1),
        ("e", TAU2), ("o", TAU4), ("e", TAU4), ("o", TAU4), ("e", TAU3)],
}


def site_weight(k, L):
    """Share of site k's terms given to each bond that contains it: 1 / (number of such bonds)."""
    nb = (1 if k > 1 else 0) + (1 if k < L else 0)
    return 1.0 / nb


def bond_hamiltonians(desc):
    """h_k for k = 1..L-1: the 4x4 two-site Hamiltonian of bond (k, k+1), index i_k*2 + i_{k+1}:
    its bond terms plus the weighted site terms of sites k and k+1."""
    L = desc.L
    I2 = np.eye(2)
    site = [sum((desc.site_coef[z, k - 1] * desc.site_ops[z] for z in range(len(desc.site_ops))),
                np.zeros((2, 2), np.complex128)) for k in range(1, L + 1)]
    hs = []
    for k in range(1, L):
        h = np.zeros((4, 4), np.complex128)
        for z in range(len(desc.bond_ops)):
            h += desc.bond_coef[z, k - 1] * desc.bond_ops[z]
        h += site_weight(k, L) * np.kron(site[k - 1], I2)
        h += site_weight(k + 1, L) * np.kron(I2, site[k])
        hs.append(h)
    return hs


def apply_two_site(psi, L, k, U):
    """U (4x4, index i_k*2 + i_{k+1}) contracted with legs k, k+1 of psi (rank-L tensor)."""
    T = np.asarray(psi).reshape(2 ** (k - 1), 4, 2 ** (L - k - 1))
    return np.einsum("ab,xbz->xaz", U, T).reshape(-1)


def apply_layer(psi, L, hs, which, t):
    """exp(-i t H_which) psi as the product of the commuting bond propagators of that part."""
    first = 1 if which == "o" else 2
    for k in range(first, L, 2):
        psi = apply_two_site(psi, L, k, sla.expm(-1j * t * hs[k - 1]))
    return psi


def trotter_step(psi, L, hs, dt, order):
    """One time step of the order-2 or order-4 decomposition."""
    for which, frac in SEQUENCE[order]:
        psi = apply_layer(psi, L, hs, which, frac * dt)
    return psi


def evolve(desc, psi0, dt, n_steps, order):
    """psi after n_steps Trotter steps, and the list of states after each step (index 0 = psi0)."""
    hs = bond_hamiltonians(desc)
    psi = np.asarray(psi0, np.complex128).copy()
    states = [psi.copy()]
    for _ in range(n_steps):
        psi = trotter_step(psi, desc.L, hs, dt, order)
        states.append(psi.copy())
    return psi, states
