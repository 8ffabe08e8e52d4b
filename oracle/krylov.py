"""Time evolution of a pure state (Sec. ed:sec:dynamics).

expm_step     method 1: psi(t+dt) = exp(-i H dt) psi(t) with the full propagator (Sec. ed:sec:expm).
krylov_step   method 3: psi(t+dt) ~ sum_i xi_i v_i with xi = |psi| [exp(-i dt T_m)]_{:,1} on the
              Krylov basis of psi (Sec. ed:sec:krylov). Hermitian H: Lanczos with full
              reorthogonalisation, T_m tridiagonal; non-Hermitian H: Arnoldi, upper Hessenberg
              T_m (Sec. ed:sec:Liouville, last paragraph).
Stopping rule (the paper only names a tolerance): the a-posteriori estimate
err_m = |psi| beta_m |[exp(-i dt T_m)]_{m,1}| <= tol, or happy breakdown beta_m <= 1e-14 |T|.
"""
import numpy as np
import scipy.linalg as sla


def expm_step(H_dense, psi, dt):
    """Exact propagation by the dense matrix exponential (method 1)."""
    return sla.expm(-1j * dt * H_dense) @ psi


def krylov_basis(matvec, psi, m_max, dt, tol, hermitian=True, fixed_m=0):
    """Build the Krylov basis of psi with the stopping rule above.

    Returns (V (D x m), T (m x m), beta0, m). Hermitian: alpha/beta recurrence plus two classical
    Gram-Schmidt passes against the whole basis; non-Hermitian: Arnoldi (same orthogonalisation,
    all projections kept in T).
    """
    beta0 = np.linalg.norm(psi)
    Vr = np.zeros((m_max + 1, psi.shape[0]), np.complex128)   # basis vectors as rows
    Vr[0] = psi / beta0
    T = np.zeros((m_max + 1, m_max + 1), np.complex128)
    m = 0
    for j in range(m_max):
        w = matvec(Vr[j])
        Vj = Vr[:j + 1]
        h = np.conj(Vj @ np.conj(w))           # V^H w
        w = w - Vj.T @ h
        h2 = np.conj(Vj @ np.conj(w))
        w = w - Vj.T @ h2
        h = h + h2
        if hermitian:
            T[j, j] = h[j].real
            if j > 0:
                T[j - 1, j] = T[j, j - 1]
        else:
            T[:j + 1, j] = h
        b = np.linalg.norm(w)
        m = j + 1
        Tm = T[:m, :m]
        u = sla.expm(-1j * dt * Tm)[:, 0]
        err = beta0 * b * abs(u[-1])
        tnorm = np.abs(Tm).sum(axis=0).max()
        if fixed_m:
            if m >= fixed_m or b <= 1e-14 * max(tnorm, 1.0):
                break
        elif err <= tol or b <= 1e-14 * max(tnorm, 1.0):
            break
        T[j + 1, j] = b
        Vr[j + 1] = w / b
    return Vr[:m].T.copy(), T[:m, :m].copy(), beta0, m


def krylov_step(matvec, psi, dt, m_max=20, tol=1e-10, hermitian=True, fixed_m=0):
    """One Krylov time step psi -> |psi| V_m exp(-i dt T_m) e_1; returns (psi_new, m)."""
    V, T, beta0, m = krylov_basis(matvec, psi, m_max, dt, tol, hermitian, fixed_m)
    u = sla.expm(-1j * dt * T)[:, 0]
    return beta0 * (V @ u), m
