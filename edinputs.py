"""Seeded synthetic inputs shared by the CPU oracle tests and the GPU path.

This module holds data only: the local operator matrices of the spin-1/2 models, coefficient
arrays and seeded random vectors. No Hamiltonian, Krylov or measurement arithmetic lives here,
so that the oracle and the HIP library share nothing but their inputs.

Conventions (the paper is silent on them; the readings are listed in the design notes):
  * local basis: index 0 = up (sigma^z = +1), index 1 = down;
  * state index x = sum_k i_k 2^(L-k): site 1 is the most significant digit, as in the
    row-major rank-L tensor view of the state (Sec. ed:sec:meas, single-site density matrix);
  * bond operators are 4x4 with row/column index i_k*2 + i_{k+1} (site k is the left factor
    of the Kronecker product, App. A bond rule).
"""
from dataclasses import dataclass

import numpy as np

# --- local operators (2x2, complex128) -------------------------------------------------
SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
SMINUS = np.array([[0, 0], [1, 0]], dtype=np.complex128)   # |down><up|
SPLUS = np.array([[0, 1], [0, 0]], dtype=np.complex128)    # |up><down|
NUP = np.array([[1, 0], [0, 0]], dtype=np.complex128)      # |up><up|

# --- two-site operators written out (4x4, index i_k*2 + i_{k+1}) ----------------------
SXSX = np.array([[0, 0, 0, 1],
                 [0, 0, 1, 0],
                 [0, 1, 0, 0],
                 [1, 0, 0, 0]], dtype=np.complex128)
SYSY = np.array([[0, 0, 0, -1],
                 [0, 0, 1, 0],
                 [0, 1, 0, 0],
                 [-1, 0, 0, 0]], dtype=np.complex128)
SZSZ = np.array([[1, 0, 0, 0],
                 [0, -1, 0, 0],
                 [0, 0, -1, 0],
                 [0, 0, 0, 1]], dtype=np.complex128)


@dataclass
class ModelDesc:
    """Rule-set description of H = sum_sites c_k O_k + sum_bonds c'_k O_k (x) O'_{k+1}
    + sum_inf sum_{k<j} c''_k f(j-k) O_k (x) O'_j (Eq. ed:eq:genericH; site, bond and
    InfiniteFunc rules of App. A, the latter without phase operators), with w*c_k folded into
    the coefficient arrays.

    site_ops  (n_site, 2, 2) complex128;  site_coef (n_site, L) float64
    bond_ops  (n_bond, 4, 4) complex128;  bond_coef (n_bond, L-1) float64
    inf_ops, inf_ops2 (n_inf, 2, 2) complex128 (O, O');  inf_coef (n_inf, L) float64 (c''_k);
    inf_f (n_inf, L-1) float64 (f(r) for r = 1..L-1)
    """
    L: int
    site_ops: np.ndarray
    site_coef: np.ndarray
    bond_ops: np.ndarray
    bond_coef: np.ndarray
    d: int = 2
    inf_ops: np.ndarray = None
    inf_ops2: np.ndarray = None
    inf_coef: np.ndarray = None
    inf_f: np.ndarray = None

    def __post_init__(self):
        self.site_ops = np.ascontiguousarray(np.asarray(self.site_ops, np.complex128).reshape(-1, 2, 2))
        self.site_coef = np.ascontiguousarray(np.asarray(self.site_coef, np.float64).reshape(len(self.site_ops), self.L))
        self.bond_ops = np.ascontiguousarray(np.asarray(self.bond_ops, np.complex128).reshape(-1, 4, 4))
        self.bond_coef = np.ascontiguousarray(
            np.asarray(self.bond_coef, np.float64).reshape(len(self.bond_ops), max(self.L - 1, 0)))
        n_inf = 0 if self.inf_ops is None else len(np.asarray(self.inf_ops).reshape(-1, 2, 2))
        self.inf_ops = np.ascontiguousarray(
            np.zeros((0, 2, 2)) if n_inf == 0 else np.asarray(self.inf_ops, np.complex128).reshape(-1, 2, 2),
            dtype=np.complex128)
        self.inf_ops2 = np.ascontiguousarray(
            np.zeros((0, 2, 2)) if n_inf == 0 else np.asarray(self.inf_ops2, np.complex128).reshape(-1, 2, 2),
            dtype=np.complex128)
        self.inf_coef = np.ascontiguousarray(
            np.zeros((0, self.L)) if n_inf == 0 else np.asarray(self.inf_coef, np.float64).reshape(n_inf, self.L))
        self.inf_f = np.ascontiguousarray(
            np.zeros((0, max(self.L - 1, 0))) if n_inf == 0
            else np.asarray(self.inf_f, np.float64).reshape(n_inf, max(self.L - 1, 0)))

    @property
    def dim(self):
        return self.d ** self.L


def tfim(L, g, J=1.0):
    """Quantum Ising chain H = -J sum sz sz - g sum sx (Eq. ed:eq:HQI with h = g)."""
    return ModelDesc(L,
                     site_ops=[SX], site_coef=np.full((1, L), -g),
                     bond_ops=[SZSZ], bond_coef=np.full((1, L - 1), -J))


def xxz(L, J, delta, h=None):
    """XXZ chain H = J sum (sx sx + sy sy + delta sz sz) + sum_k h_k sz_k (Pauli matrices)."""
    h = np.zeros(L) if h is None else np.asarray(h, np.float64)
    return ModelDesc(L,
                     site_ops=[SZ], site_coef=h.reshape(1, L),
                     bond_ops=[SXSX, SYSY, SZSZ],
                     bond_coef=np.stack([np.full(L - 1, J), np.full(L - 1, J), np.full(L - 1, J * delta)]))


def xxz_bond_scaled(L, delta, Jb):
    """XXZ bonds J_b (sx sx + sy sy + delta sz sz) with per-bond couplings J_b, no fields."""
    Jb = np.asarray(Jb, np.float64)
    return ModelDesc(L,
                     site_ops=np.zeros((0, 2, 2)), site_coef=np.zeros((0, L)),
                     bond_ops=[SXSX, SYSY, SZSZ],
                     bond_coef=np.stack([Jb, Jb, delta * Jb]))


def lrqi(L, phi, alpha):
    """Long-range quantum Ising chain: H = -sum_{k<k'} cos(phi)/(k'-k)^alpha sz_k sz_k'
    - sin(phi) sum_k sx_k (the H_LRQI of the thermalisation section); the zz part is one
    InfiniteFunc rule with f(r) = r^-alpha."""
    r = np.arange(1, L, dtype=np.float64)
    return ModelDesc(L, site_ops=[SX], site_coef=np.full((1, L), -np.sin(phi)),
                     bond_ops=np.zeros((0, 4, 4)), bond_coef=np.zeros((0, L - 1)),
                     inf_ops=[SZ], inf_ops2=[SZ], inf_coef=np.full((1, L), -np.cos(phi)),
                     inf_f=(r ** -float(alpha)).reshape(1, L - 1))


def random_fields(L, seed, lo=-0.5, hi=0.5):
    return np.random.default_rng(seed).uniform(lo, hi, size=L)


def random_model(L, seed, n_site=2, n_bond=3, hermitian=True):
    """A generic dense-operator model (every entry of every local op nonzero) for parity tests."""
    rng = np.random.default_rng(seed)
    def rnd(shape):
        a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        if hermitian:
            a = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
        return a
    return ModelDesc(L,
                     site_ops=rnd((n_site, 2, 2)), site_coef=rng.uniform(-1, 1, (n_site, L)),
                     bond_ops=rnd((n_bond, 4, 4)), bond_coef=rng.uniform(-1, 1, (n_bond, L - 1)))


def random_state(L, seed, normalise=True, real=False):
    """Complex-normal state of length 2^L (seeded); with real=True a real-normal one (complex
    dtype, every imaginary part exactly zero)."""
    rng = np.random.default_rng(seed)
    D = 1 << L
    v = rng.standard_normal(D) + (0j if real else 1j * rng.standard_normal(D))
    if normalise:
        v /= np.linalg.norm(v)
    return v


def basis_index(spins_up):
    """Index of the product state with site k up iff spins_up[k-1] (site 1 = top digit)."""
    L = len(spins_up)
    x = 0
    for k, up in enumerate(spins_up):
        if not up:
            x |= 1 << (L - 1 - k)
    return x


def neel_index(L):
    """Neel state up,down,up,... with site 1 up."""
    return basis_index([k % 2 == 0 for k in range(L)])


def product_state(L, index):
    v = np.zeros(1 << L, np.complex128)
    v[index] = 1.0
    return v


def adjoint_couplings(n_slices, n_bonds, seed, lo=0.5, hi=1.5):
    """J[s, b] drawn independently U[lo, hi] in (slice, bond) row-major order."""
    return np.random.default_rng(seed).uniform(lo, hi, size=(n_slices, n_bonds))


def trajectory_lengths(n_traj, lengths=(8, 10, 12, 14, 16)):
    """Chain length of trajectory t is lengths[t mod len(lengths)]."""
    return np.array([lengths[t % len(lengths)] for t in range(n_traj)], dtype=np.int32)


def random_state_device(L, seed, device, real=False):
    """Complex-normal normalised state of length 2^L generated directly on a torch device
    (seeded torch generator), for sizes where a host copy would only cost time; with real=True
    a real-normal one (complex dtype, every imaginary part exactly zero)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    if real:
        v = torch.randn(1 << L, dtype=torch.float64, device=device, generator=g).to(torch.complex128)
    else:
        v = torch.randn(1 << L, dtype=torch.complex128, device=device, generator=g)
    v /= torch.linalg.vector_norm(v)
    return v


def graded_schmidt_state(L, l, rank, decay, seed, real=False):
    """State of length 2^L whose matrix view M (2^l rows = sites 1..l) is A diag(s) B^dagger,
    with complex-normal A (2^l x rank) and B (2^(L-l) x rank) and s_k = exp(-k / decay): a
    Schmidt spectrum that falls off geometrically like a ground state's, of rank <= rank.
    Normalised. Seeded. With real=True, A and B are real-normal (complex dtype, zero imaginary
    parts)."""
    rng = np.random.default_rng(seed)
    n, K = 1 << l, 1 << (L - l)
    A = rng.standard_normal((n, rank)) + (0j if real else 1j * rng.standard_normal((n, rank)))
    B = rng.standard_normal((K, rank)) + (0j if real else 1j * rng.standard_normal((K, rank)))
    s = np.exp(-np.arange(rank) / float(decay))
    v = ((A * s) @ B.conj().T).reshape(-1)
    return v / np.linalg.norm(v)
