"""Independent closed forms and brute-force evaluations used to pin the oracle.

Nothing here imports the oracle or the HIP library."""
import numpy as np


def tfim_bdg_ground_energy(L, J, g):
    """Open transverse-field Ising chain H = -J sum sz sz - g sum sx: after the Jordan-Wigner
    map the quasi-particle energies are 2 s_k with s_k the singular values of the L x L upper
    bidiagonal matrix (diagonal g, super-diagonal J); E0 = -sum_k s_k."""
    M = np.diag(np.full(L, float(g))) + np.diag(np.full(L - 1, float(J)), 1)
    return -np.linalg.svd(M, compute_uv=False).sum()


def xxz_two_site_spectrum(J, delta, h1, h2):
    """Eigenvalues of J(sx sx + sy sy + delta sz sz) + h1 sz1 + h2 sz2 (Pauli matrices)."""
    r = np.sqrt(4 * J * J + (h1 - h2) ** 2)
    return np.sort([J * delta + h1 + h2, J * delta - h1 - h2, -J * delta + r, -J * delta - r])


def bit(x, k, L):
    """Local index of site k (1-based) in basis state x: site 1 is the most significant digit."""
    return (x >> (L - k)) & 1


def brute_matrix_element(desc, x, y):
    """<x|H|y> straight from the rule definitions with explicit deltas on untouched sites."""
    L = desc.L
    val = 0j
    for z in range(len(desc.site_ops)):
        for k in range(1, L + 1):
            if all(bit(x, j, L) == bit(y, j, L) for j in range(1, L + 1) if j != k):
                val += desc.site_coef[z, k - 1] * desc.site_ops[z][bit(x, k, L), bit(y, k, L)]
    for z in range(len(desc.bond_ops)):
        for k in range(1, L):
            if all(bit(x, j, L) == bit(y, j, L) for j in range(1, L + 1) if j not in (k, k + 1)):
                r = 2 * bit(x, k, L) + bit(x, k + 1, L)
                c = 2 * bit(y, k, L) + bit(y, k + 1, L)
                val += desc.bond_coef[z, k - 1] * desc.bond_ops[z][r, c]
    return val


def brute_apply_entry(desc, psi, x):
    """(H psi)[x] by summing over the basis states y that differ from x on at most two
    neighbouring sites (every other <x|H|y> vanishes for site and bond rules)."""
    L = desc.L
    ys = {x}
    for p in range(L):
        ys.add(x ^ (1 << p))
    for p in range(L - 1):
        ys.add(x ^ (3 << p))
    return sum(brute_matrix_element(desc, x, y) * psi[y] for y in ys)


M64 = (1 << 64) - 1
PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)


def philox4x64_10(ctr, key):
    """Philox4x64 with 10 rounds, from Salmon et al. (SC'11): two 64x64->128 multiplies per
    round, the key bumped by the Weyl constants between rounds."""
    x = list(ctr)
    k0, k1 = key
    for _ in range(10):
        p0 = PHILOX_M[0] * x[0]
        p1 = PHILOX_M[1] * x[2]
        x = [((p1 >> 64) ^ x[1] ^ k0) & M64, p1 & M64, ((p0 >> 64) ^ x[3] ^ k1) & M64, p0 & M64]
        k0 = (k0 + PHILOX_W[0]) & M64
        k1 = (k1 + PHILOX_W[1]) & M64
    return x
