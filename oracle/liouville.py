"""Liouville-space evolution of the density matrix (Sec. ed:sec:Liouville, Eq. ed:eq:liousuperket, App. F).

With row-major vec(rho) (index j*D + k for rho_jk), A rho B -> (A (x) B^T) |rho>> (App. F), so
  Lcal = -i (H (x) 1 - 1 (x) H^T)
         + sum_nu [ L_nu (x) L_nu^*  - 1/2 (L_nu^dagger L_nu (x) 1 + 1 (x) (L_nu^dagger L_nu)^T) ].
The anticommutator term is written from the master equation (Eq. ed:eq:lindbladme); the printed
superket equation orders it as L L^dagger, which does not preserve the trace.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def liouvillian(H, jump_ops):
    D = H.shape[0]
    I = sp.identity(D, dtype=np.complex128, format="csr")
    H = sp.csr_matrix(H)
    Lc = -1j * (sp.kron(H, I) - sp.kron(I, H.T))
    for Lnu in jump_ops:
        Lnu = sp.csr_matrix(Lnu)
        LdL = (Lnu.conj().T @ Lnu).tocsr()
        Lc = Lc + sp.kron(Lnu, Lnu.conj()) - 0.5 * (sp.kron(LdL, I) + sp.kron(I, LdL.T))
    return Lc.tocsr()


def superket(rho):
    """|rho>> = row-major vec(rho): entry j*D + k is rho_jk (the row index is the high digit
    string: the rank-2L tensor with the L row legs first, then the L column legs)."""
    return np.ascontiguousarray(rho).reshape(-1).astype(np.complex128)


def measure(vec, L):
    """(<sigma^z_k> = tr(sigma^z_k rho)/tr(rho) for k = 1..L, tr(rho)) of a superket."""
    D = 1 << L
    rho = vec.reshape(D, D)
    diag = np.real(np.diag(rho))
    tr = float(diag.sum())
    p = diag.reshape((2,) * L)
    sz = []
    for k in range(L):
        m = np.moveaxis(p, k, 0).reshape(2, -1).sum(axis=1)
        sz.append((m[0] - m[1]) / tr)
    return np.array(sz), tr


def evolve_states(H, jump_ops, vec0, dt, n_steps):
    """Superkets at t = 0, dt, ..., n_steps dt: |rho(t)>> = exp(t Lcal)|rho(0)>> (expm_multiply)."""
    Lc = liouvillian(H, jump_ops)
    out = [np.asarray(vec0, np.complex128)]
    for _ in range(n_steps):
        out.append(spla.expm_multiply(Lc * dt, out[-1]))
    return out


def evolve_sz(H, jump_ops, rho0, times):
    """(<sigma^z_k>, tr rho) at the given times (expm_multiply on |rho>>)."""
    D = H.shape[0]
    L = int(np.log2(D))
    Lc = liouvillian(H, jump_ops)
    vec = superket(rho0)
    out = []
    t_prev = 0.0
    for t in times:
        if t > t_prev:
            vec = spla.expm_multiply(Lc * (t - t_prev), vec)
            t_prev = t
        sz, tr = measure(vec, L)
        out.append((sz * tr, tr))
    return out
