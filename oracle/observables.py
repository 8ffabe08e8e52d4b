"""Measurements on a pure state (Sec. ed:sec:meas).

sz_all       <sigma^z_k> for every site k, normalised by <psi|psi>; the diagonal of the
             single-site reduced density matrix rho_k (Sec. ed:sec:meas, the [A][B] block construction).
energy       <psi|H|psi>/<psi|psi>.
bond_entropy S(l) = -sum_j Lambda_j log Lambda_j with Lambda_j the eigenvalues of
             rho_l = M M^dagger, M = psi reshaped to d^l x d^(L-l) (Sec. ed:sec:meas, bond entropy; the
             paper notes the SVD of M gives the same spectrum). Natural log, 0 log 0 = 0.
"""
import numpy as np


def sz_all(psi, L):
    """<sigma^z_k>, k = 1..L, by reshaping psi into a rank-L tensor and summing |psi|^2 over all
    legs except k (site 1 is the first leg)."""
    p = (np.abs(psi) ** 2).reshape((2,) * L)
    nrm = p.sum()
    out = np.empty(L)
    for k in range(L):
        marg = np.moveaxis(p, k, 0).reshape(2, -1).sum(axis=1)
        out[k] = (marg[0] - marg[1]) / nrm
    return out


def energy(H, psi):
    return float(np.vdot(psi, H @ psi).real / np.vdot(psi, psi).real)


def norm(psi):
    return float(np.linalg.norm(psi))


def schmidt_spectrum(psi, L, l):
    """Eigenvalues of rho_l of the normalised state, from the SVD of M (descending)."""
    M = psi.reshape(2 ** l, 2 ** (L - l)) / np.linalg.norm(psi)
    s = np.linalg.svd(M, compute_uv=False)
    return s ** 2


def bond_entropy(psi, L, l):
    lam = schmidt_spectrum(psi, L, l)
    lam = lam[lam > 1e-300]
    return float(-(lam * np.log(lam)).sum())
