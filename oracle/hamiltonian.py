"""H built on the full Hilbert space from Kronecker products (Sec. ed:sec:statics, Eqs. ed:eq:genericH and
ed:eq:OH; site, bond and InfiniteFunc rules of App. A, Eqs. ed:eq:appsiters / ed:eq:appbondrs /
ed:eq:appinfrs).

A site rule term c_k O_k is I_{d^(k-1)} (x) O (x) I_{d^(L-k)}; a bond rule term c'_k O_k O'_{k+1}
is I_{d^(k-1)} (x) B (x) I_{d^(L-k-1)} with B = O (x) O' given as a d^2 x d^2 matrix; an
InfiniteFunc term c''_k f(j-k) O_k O'_j (k < j, phase operators Q = identity) is
I_{d^(k-1)} (x) O (x) I_{d^(j-k-1)} (x) O' (x) I_{d^(L-j)}. Site 1 is the leftmost Kronecker factor,
i.e. the most significant digit of the state index.
"""
import numpy as np
import scipy.sparse as sp


def _embed(op, k, width, L, d, fmt="coo"):
    """I_{d^(k-1)} (x) op (x) I_{d^(L-k-width+1)} for an operator on sites k..k+width-1 (1-based)."""
    left = sp.identity(d ** (k - 1), dtype=np.complex128, format="csr")
    right = sp.identity(d ** (L - k - width + 1), dtype=np.complex128, format="csr")
    return sp.kron(sp.kron(left, sp.csr_matrix(op), format="csr"), right, format=fmt)


def _inf_terms(desc):
    """(coefficient, k, j, O, O') of every InfiniteFunc term with a nonzero coefficient."""
    L = desc.L
    out = []
    for z in range(len(desc.inf_ops)):
        for k in range(1, L):
            for j in range(k + 1, L + 1):
                c = desc.inf_coef[z, k - 1] * desc.inf_f[z, j - k - 1]
                if c != 0.0:
                    out.append((c, k, j, desc.inf_ops[z], desc.inf_ops2[z]))
    return out


def _embed_pair(o1, k, o2, j, L, d, fmt="coo"):
    """I (x) o1 (x) I (x) o2 (x) I with o1 on site k and o2 on site j > k (1-based)."""
    mid = sp.kron(sp.kron(sp.csr_matrix(o1), sp.identity(d ** (j - k - 1), dtype=np.complex128, format="csr"),
                          format="csr"), sp.csr_matrix(o2), format="csr")
    return _embed(mid, k, j - k + 1, L, d, fmt)


def hamiltonian_sparse(desc):
    """Sparse CSR H = sum_zeta sum_k c_k O_k + sum_zeta sum_k c'_k O_k O'_{k+1}
    + sum_zeta sum_{k<j} c''_k f(j-k) O_k O'_j."""
    L, d = desc.L, desc.d
    D = d ** L
    rows, cols, vals = [], [], []
    terms = []
    for z in range(len(desc.site_ops)):
        for k in range(1, L + 1):
            c = desc.site_coef[z, k - 1]
            if c != 0.0:
                terms.append(c * _embed(desc.site_ops[z], k, 1, L, d))
    for z in range(len(desc.bond_ops)):
        for k in range(1, L):
            c = desc.bond_coef[z, k - 1]
            if c != 0.0:
                terms.append(c * _embed(desc.bond_ops[z], k, 2, L, d))
    for c, k, j, o1, o2 in _inf_terms(desc):
        terms.append(c * _embed_pair(o1, k, o2, j, L, d))
    for t in terms:
        t = t.tocoo()
        rows.append(t.row)
        cols.append(t.col)
        vals.append(t.data)
    if not terms:
        return sp.csr_matrix((D, D), dtype=np.complex128)
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(D, D)).tocsr()   # duplicates are summed
    H.eliminate_zeros()
    return H


def hamiltonian_dense(desc):
    """Dense H by numpy.kron (the paper's dense build, Sec. ed:sec:statics)."""
    L, d = desc.L, desc.d
    D = d ** L
    H = np.zeros((D, D), np.complex128)
    for z in range(len(desc.site_ops)):
        for k in range(1, L + 1):
            c = desc.site_coef[z, k - 1]
            if c != 0.0:
                H += c * np.kron(np.kron(np.eye(d ** (k - 1)), desc.site_ops[z]), np.eye(d ** (L - k)))
    for z in range(len(desc.bond_ops)):
        for k in range(1, L):
            c = desc.bond_coef[z, k - 1]
            if c != 0.0:
                H += c * np.kron(np.kron(np.eye(d ** (k - 1)), desc.bond_ops[z]), np.eye(d ** (L - k - 1)))
    for c, k, j, o1, o2 in _inf_terms(desc):
        op = np.kron(np.kron(o1, np.eye(d ** (j - k - 1))), o2)
        H += c * np.kron(np.kron(np.eye(d ** (k - 1)), op), np.eye(d ** (L - j)))
    return H


def apply_H(desc, psi, H=None):
    """y = H psi with the explicit sparse H (Krylov mode 1 of Sec. ed:sec:krylov)."""
    if H is None:
        H = hamiltonian_sparse(desc)
    return H @ psi


def site_operator(op, k, L, d=2):
    """Sparse I (x) op (x) I for op on site k (1-based)."""
    return _embed(op, k, 1, L, d, fmt="csr")


def apply_H_entries(desc, psi, xs):
    """(H psi)[x] for the indices xs, evaluated term by term from the rule definitions: a site
    term on site k maps psi to sum_{i'} O[i_k(x), i'] psi[x with i_k = i'], a bond term likewise on
    the two digits of sites k, k+1, an InfiniteFunc term on the digits of sites k and j; all other
    digits are untouched (the identity factors of the Kronecker product). Used where the full
    sparse H does not fit in memory."""
    L = desc.L
    xs = np.asarray(xs, dtype=np.int64)
    acc = np.zeros(len(xs), np.complex128)
    for z in range(len(desc.site_ops)):
        for k in range(1, L + 1):
            c = desc.site_coef[z, k - 1]
            if c == 0.0:
                continue
            p = L - k
            b = (xs >> p) & 1
            for bp in (0, 1):
                y = (xs & ~np.int64(1 << p)) | (np.int64(bp) << p)
                acc += c * desc.site_ops[z][b, bp] * psi[y]
    for z in range(len(desc.bond_ops)):
        for k in range(1, L):
            c = desc.bond_coef[z, k - 1]
            if c == 0.0:
                continue
            p_left, p_right = L - k, L - k - 1
            row = 2 * ((xs >> p_left) & 1) + ((xs >> p_right) & 1)
            for col in range(4):
                y = (xs & ~np.int64((1 << p_left) | (1 << p_right))) \
                    | (np.int64(col >> 1) << p_left) | (np.int64(col & 1) << p_right)
                acc += c * desc.bond_ops[z][row, col] * psi[y]
    for c, k, j, o1, o2 in _inf_terms(desc):
        pk, pj = L - k, L - j
        bk, bj = (xs >> pk) & 1, (xs >> pj) & 1
        for ck in (0, 1):
            for cj in (0, 1):
                y = (xs & ~np.int64((1 << pk) | (1 << pj))) | (np.int64(ck) << pk) | (np.int64(cj) << pj)
                acc += c * o1[bk, ck] * o2[bj, cj] * psi[y]
    return acc
