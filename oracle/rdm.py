"""Reduced density matrices and the error measures built on them (Sec. ed:sec:meas, single-site and
two-site density matrices; Sec. ed:sec:conv, Eqs. ed:eq:erhoi, ed:eq:erhoij, ed:eq:eener, ed:eq:eentr and
the convergence rate of Eq. ed:eq:convrate).

Test infrastructure: imported only by the tests, the smoke check and the CPU baseline of the
benchmark; it shares no code with the HIP library.

rho of the sites K = (k_1 < k_2 < ...) is the partial trace of |psi><psi| over the other sites,
taken the way Sec. ed:sec:meas lays it out: psi is reshaped into a rank-L tensor (site 1 = first leg),
the kept legs are permuted to the front, the tensor is reshaped into a d^|K| x d^(L-|K|) matrix
A, and rho = A A^dagger. Row and column index of rho: i_{k_1} d^(|K|-1) + ... + i_{k_|K|}.
No normalisation: Tr rho = <psi|psi>.

The trace distance is D(rho, rho') = 1/2 Tr |rho - rho'| with |A| = sqrt(A^dagger A), i.e. half
the sum of the absolute eigenvalues of the Hermitian difference.
"""
import numpy as np


def rdm(psi, L, sites, d=2):
    """rho of the 1-based sites `sites` (ascending), by reshape, transpose and A A^dagger."""
    sites = list(sites)
    assert sites == sorted(sites) and len(set(sites)) == len(sites)
    t = np.asarray(psi).reshape((d,) * L)
    keep = [k - 1 for k in sites]
    rest = [a for a in range(L) if a not in keep]
    A = np.transpose(t, keep + rest).reshape(d ** len(keep), -1)
    return A @ A.conj().T


def pair_index(k, j, L):
    """Position of the pair (k, j), 1 <= k < j <= L, in the lexicographic list of all pairs."""
    return (k - 1) * L - (k - 1) * k // 2 + (j - k - 1)


def rdm1_all(psi, L):
    """[L, 2, 2]: rho_k for k = 1..L."""
    return np.stack([rdm(psi, L, [k]) for k in range(1, L + 1)])


def rdm2_all(psi, L):
    """[L(L-1)/2, 4, 4]: rho_{k,j} for all pairs k < j in lexicographic order."""
    return np.stack([rdm(psi, L, [k, j]) for k in range(1, L + 1) for j in range(k + 1, L + 1)])


def trace_distance(a, b):
    """D = 1/2 sum |lambda_i(a - b)| for Hermitian a, b."""
    return 0.5 * float(np.abs(np.linalg.eigvalsh(np.asarray(a) - np.asarray(b))).sum())


def eps_local(rho1, rho1_ref):
    """Eq. ed:eq:erhoi: the largest single-site trace distance."""
    return max(trace_distance(a, b) for a, b in zip(rho1, rho1_ref))


def eps_corr(rho2, rho2_ref):
    """Eq. ed:eq:erhoij: the largest two-site trace distance over all pairs k < j."""
    return max(trace_distance(a, b) for a, b in zip(rho2, rho2_ref))


def eps_energy(E, E_ref):
    """Eq. ed:eq:eener."""
    return abs(E - E_ref)


def eps_entropy(S, S_ref):
    """Eq. ed:eq:eentr (the caller passes S(L/2))."""
    return abs(S - S_ref)


def convergence_rate(eps_alpha_dt, eps_dt, alpha):
    """Eq. ed:eq:convrate: r = ln(eps(alpha dt) / eps(dt)) / ln(alpha)."""
    return float(np.log(eps_alpha_dt / eps_dt) / np.log(alpha))
