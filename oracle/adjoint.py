"""Gradient of a final-time observable with respect to piecewise-constant bond couplings.

Forward: psi_s = U_s psi_{s-1}, U_s = exp(-i H_s Delta), H_s = sum_b J_{s,b} h_b + H_site.
Loss: <psi_N|O|psi_N> with O = sum_k w_k sigma^z_k.
Costate: lam_N = O psi_N, lam_{s-1} = U_s^dagger lam_s.
Gradient: dLoss/dJ_{s,b} = 2 Re <lam_s| D_s[-i Delta h_b] psi_{s-1}>, with D_s the Frechet
derivative of the matrix exponential at -i H_s Delta.
  gradient_frechet  D_s from scipy.linalg.expm_frechet (the definition, small L);
  gradient_eig      D_s from the eigendecomposition H_s = Q diag(e) Q^dagger, where
                    D_s[E] = Q ((Q^dagger E Q) o Phi) Q^dagger, Phi_ij the divided difference of
                    exp(-i Delta x) at e_i, e_j (exact for Hermitian H_s; used at L = 10).
"""
import numpy as np
import scipy.linalg as sla

from .hamiltonian import hamiltonian_dense, site_operator


def _bond_dense(template, b):
    """Dense h_b: sum_zeta bond_coef[zeta, b] * bond_op[zeta] on sites b+1, b+2."""
    L = template.L
    op = np.zeros((4, 4), np.complex128)
    for z in range(len(template.bond_ops)):
        op += template.bond_coef[z, b] * template.bond_ops[z]
    return np.kron(np.kron(np.eye(2 ** b), op), np.eye(2 ** (L - b - 2)))


def _site_dense(template):
    L = template.L
    H = np.zeros((2 ** L, 2 ** L), np.complex128)
    for z in range(len(template.site_ops)):
        for k in range(L):
            c = template.site_coef[z, k]
            if c != 0.0:
                H += c * np.kron(np.kron(np.eye(2 ** k), template.site_ops[z]), np.eye(2 ** (L - k - 1)))
    return H


def observable_dense(L, w):
    sz = np.array([[1, 0], [0, -1]], np.complex128)
    O = np.zeros((2 ** L, 2 ** L), np.complex128)
    for k in range(L):
        O += w[k] * site_operator(sz, k + 1, L).toarray()
    return O


def forward(template, J, psi0, Delta, w):
    L = template.L
    hb = [_bond_dense(template, b) for b in range(L - 1)]
    Hs0 = _site_dense(template)
    O = observable_dense(L, w)
    psis = [psi0.astype(np.complex128)]
    for s in range(J.shape[0]):
        H = Hs0 + sum(J[s, b] * hb[b] for b in range(L - 1))
        psis.append(sla.expm(-1j * Delta * H) @ psis[-1])
    loss = float(np.vdot(psis[-1], O @ psis[-1]).real)
    return loss, psis, hb, Hs0, O


def gradient_frechet(template, J, psi0, Delta, w):
    loss, psis, hb, Hs0, O = forward(template, J, psi0, Delta, w)
    S, B = J.shape
    lam = O @ psis[-1]
    grad = np.zeros((S, B))
    for s in range(S, 0, -1):
        H = Hs0 + sum(J[s - 1, b] * hb[b] for b in range(B))
        A = -1j * Delta * H
        for b in range(B):
            U, dU = sla.expm_frechet(A, -1j * Delta * hb[b])
            grad[s - 1, b] = 2.0 * np.vdot(lam, dU @ psis[s - 1]).real
        lam = sla.expm(A).conj().T @ lam
    return loss, grad


def gradient_eig(template, J, psi0, Delta, w):
    loss, psis, hb, Hs0, O = forward(template, J, psi0, Delta, w)
    S, B = J.shape
    lam = O @ psis[-1]
    grad = np.zeros((S, B))
    for s in range(S, 0, -1):
        H = Hs0 + sum(J[s - 1, b] * hb[b] for b in range(B))
        e, Q = np.linalg.eigh(H)
        f = np.exp(-1j * Delta * e)
        de = e[:, None] - e[None, :]
        same = np.abs(de) < 1e-12
        # Phi_ij = (exp(a_i) - exp(a_j)) / (a_i - a_j) with a = -i Delta e; exp(a_i) if a_i = a_j
        Phi = np.where(same, f[:, None] * np.ones_like(de),
                       (f[:, None] - f[None, :]) / np.where(same, 1.0, -1j * Delta * de))
        lt = Q.conj().T @ lam
        pt = Q.conj().T @ psis[s - 1]
        G = np.conj(lt)[:, None] * pt[None, :] * Phi
        Y = Q @ G.T @ Q.conj().T          # sum_ij G_ij (Q^H E Q)_ij = sum_kl Y_lk E_kl
        for b in range(B):
            E = -1j * Delta * hb[b]
            grad[s - 1, b] = 2.0 * np.sum(Y.T * E).real
        lam = Q @ (np.conj(f) * lt)
    return loss, grad


def loss_only(template, J, psi0, Delta, w):
    return forward(template, J, psi0, Delta, w)[0]
