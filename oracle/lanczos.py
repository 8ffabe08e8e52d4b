"""Ground state (Sec. ed:sec:statics; the Krylov basis of Sec. ed:sec:krylov).

ground_state_eigsh follows the paper's statics (scipy.sparse.linalg.eigsh on the full sparse H,
Sec. ed:sec:statics). lanczos_ground is the textbook Lanczos recurrence with full reorthogonalisation
(classical Gram-Schmidt applied twice), which is what the GPU path computes matrix-free.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def ground_state_eigsh(H, v0=None, tol=0.0):
    """Lowest eigenpair of a Hermitian sparse H by ARPACK, as the paper's sparse statics."""
    vals, vecs = spla.eigsh(H, k=1, which="SA", v0=v0, tol=tol)
    return float(vals[0]), vecs[:, 0]


def lanczos_ground(matvec, v0, tol=1e-10, max_iter=200):
    """Textbook Lanczos ground state.

    v_1 = v0/|v0|; for j = 1, 2, ...: w = H v_j; alpha_j = Re<v_j|w>;
    w -= alpha_j v_j + beta_{j-1} v_{j-1}; w -= V(V^H w) twice; beta_j = |w|;
    the lowest Ritz pair (theta, s) of T_j stops the loop when beta_j |s_j| <= tol, or at
    breakdown beta_j <= 1e-14 * max(|theta|, 1). Returns (E0, psi0, info) with the explicit
    residual |H psi0 - E0 psi0| in info.
    """
    v = v0 / np.linalg.norm(v0)
    V = [v]
    alpha, beta = [], []
    theta, s = None, None
    it = 0
    for j in range(max_iter):
        it = j + 1
        w = matvec(V[j])
        a = np.vdot(V[j], w).real
        alpha.append(a)
        w = w - a * V[j]
        if j > 0:
            w = w - beta[j - 1] * V[j - 1]
        Vm = np.stack(V, axis=1)
        for _ in range(2):
            w = w - Vm @ (Vm.conj().T @ w)
        b = np.linalg.norm(w)
        if j == 0:
            theta_all, S = np.array([a]), np.ones((1, 1))
        else:
            theta_all, S = sla.eigh_tridiagonal(np.array(alpha), np.array(beta))
        theta, s = theta_all[0], S[:, 0]
        if b * abs(s[-1]) <= tol or b <= 1e-14 * max(abs(theta), 1.0):
            break
        beta.append(b)
        V.append(w / b)
    Vm = np.stack(V[:len(s)], axis=1)
    psi = Vm @ s
    psi /= np.linalg.norm(psi)
    r = np.linalg.norm(matvec(psi) - theta * psi)
    return float(theta), psi, {"iters": it, "residual": float(r), "alpha": np.array(alpha),
                               "beta": np.array(beta)}
