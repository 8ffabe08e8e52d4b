"""Pins of the oracle's InfiniteFunc rule (App. A, Eq. ed:eq:appinfrs, without phase operators)
and of the long-range quantum Ising chain H_LRQI: the nearest-neighbour limit alpha -> infinity
(only f(1) survives) equals the bond rule; at alpha = 0 the zz part is -J (M^2 - L)/2 with
M = sum_k z_k; term-by-term evaluation, sparse and dense builds agree; the spectrum is
Hermitian-real and, at phi = 0, the ferromagnetic ground energy of the all-to-all model is
-J L(L-1)/2."""
import numpy as np
import pytest

import edinputs as E
from oracle import hamiltonian as OH


def test_nearest_neighbour_limit_equals_bond_rule():
    L = 8
    J = -0.8
    inf = E.ModelDesc(L, site_ops=[E.SX], site_coef=np.full((1, L), 0.4), bond_ops=np.zeros((0, 4, 4)),
                      bond_coef=np.zeros((0, L - 1)), inf_ops=[E.SZ], inf_ops2=[E.SZ],
                      inf_coef=np.full((1, L), J), inf_f=np.r_[1.0, np.zeros(L - 2)].reshape(1, L - 1))
    nn = E.ModelDesc(L, site_ops=[E.SX], site_coef=np.full((1, L), 0.4), bond_ops=[E.SZSZ],
                     bond_coef=np.full((1, L - 1), J))
    d = OH.hamiltonian_sparse(inf) - OH.hamiltonian_sparse(nn)
    assert abs(d).max() == 0.0


def test_all_to_all_closed_form():
    """alpha = 0, no field: sum_{k<j} z_k z_j = (M^2 - L) / 2 on every basis state."""
    L, J = 9, 0.7
    desc = E.lrqi(L, 0.0, 0.0)   # cos(0) = 1: -sum_{k<j} z z
    H = OH.hamiltonian_sparse(desc)
    x = np.arange(1 << L)
    M = sum(1 - 2 * ((x >> p) & 1) for p in range(L))
    assert np.allclose(H.diagonal(), -(M ** 2 - L) / 2, atol=1e-13)
    assert abs(H - np.diag(H.diagonal())).max() < 1e-15
    # ferromagnetic ground energy
    assert np.isclose(H.diagonal().real.min(), -L * (L - 1) / 2)
    desc2 = E.ModelDesc(L, site_ops=np.zeros((0, 2, 2)), site_coef=np.zeros((0, L)), bond_ops=np.zeros((0, 4, 4)),
                        bond_coef=np.zeros((0, L - 1)), inf_ops=[E.SZ], inf_ops2=[E.SZ],
                        inf_coef=np.full((1, L), -J), inf_f=np.ones((1, L - 1)))
    assert np.allclose(OH.hamiltonian_sparse(desc2).diagonal(), -J * (M ** 2 - L) / 2, atol=1e-13)


@pytest.mark.parametrize("hop", [False, True])
def test_term_by_term_sparse_dense_agree(hop):
    """A generic InfiniteFunc rule (diagonal zz and, with hop, the sigma+ sigma- hopping at any
    distance): bit-level evaluation, sparse Kronecker and dense Kronecker builds agree."""
    L = 7
    rng = np.random.default_rng(3)
    ops1, ops2 = [E.SZ], [E.NUP]
    if hop:
        ops1, ops2 = [E.SZ, E.SPLUS], [E.NUP, E.SMINUS]
    n = len(ops1)
    desc = E.ModelDesc(L, site_ops=[E.SX, E.SZ], site_coef=rng.uniform(-1, 1, (2, L)), bond_ops=[E.SXSX],
                       bond_coef=rng.uniform(-1, 1, (1, L - 1)), inf_ops=ops1, inf_ops2=ops2,
                       inf_coef=rng.uniform(-1, 1, (n, L)), inf_f=rng.uniform(0, 1, (n, L - 1)))
    Hs = OH.hamiltonian_sparse(desc)
    Hd = OH.hamiltonian_dense(desc)
    assert np.abs(Hs.toarray() - Hd).max() < 1e-14
    psi = E.random_state(L, 4)
    xs = np.arange(1 << L)
    assert np.abs(OH.apply_H_entries(desc, psi, xs) - Hs @ psi).max() < 1e-13


def test_lrqi_hermitian_and_symmetric():
    L = 8
    H = OH.hamiltonian_dense(E.lrqi(L, np.pi / 4, 1.5))
    assert np.abs(H - H.conj().T).max() == 0.0
    # Z2: the spin flip of every site commutes with H
    X = np.array([[0, 1], [1, 0]])
    P = X
    for _ in range(L - 1):
        P = np.kron(P, X)
    assert np.abs(P @ H @ P - H).max() < 1e-13
