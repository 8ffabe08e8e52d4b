"""GPU adjoint gradient of the staggered magnetisation with respect to sliced XXZ bond couplings,
against the oracle's dense Frechet-derivative gradient (L <= 10) and central finite differences
through the forward-only path (L = 20, h = 1e-6)."""
import numpy as np
import pytest
import torch

import edinputs as E
import paper_1802_10052_amd as P
from oracle import adjoint as OA

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def case(L, S, seed=5):
    tmpl = E.xxz_bond_scaled(L, 0.5, np.ones(L - 1))
    J = E.adjoint_couplings(S, L - 1, seed)
    psi0 = E.product_state(L, E.neel_index(L))
    w = np.array([(-1) ** k for k in range(L)], np.float64) / L
    return tmpl, J, psi0, w


@pytest.mark.parametrize("L,S", [(6, 3), (8, 5)])
def test_adjoint_vs_dense_oracle_small(L, S):
    tmpl, J, psi0, w = case(L, S)
    m = P.Model(tmpl)
    loss, g = P.evolve_adjoint(m, J, torch.from_numpy(psi0).to(DEV), 0.1, w, substeps=2, quad_nodes=8)
    lr, gr = OA.gradient_eig(tmpl, J, psi0, 0.1, w)
    assert abs(loss - lr) < 1e-11
    assert np.max(np.abs(g - gr)) <= 1e-9 * max(np.max(np.abs(gr)), 1e-3)


def test_adjoint_vs_dense_oracle_L10():
    """L = 10, 50 slices of 0.1, J ~ U[0.5, 1.5] (seed 5), Neel start, staggered magnetisation."""
    print("adjoint L=10 vs dense oracle", flush=True)
    tmpl, J, psi0, w = case(10, 50)
    m = P.Model(tmpl)
    loss, g = P.evolve_adjoint(m, J, torch.from_numpy(psi0).to(DEV), 0.1, w, substeps=2, quad_nodes=8)
    lr, gr = OA.gradient_eig(tmpl, J, psi0, 0.1, w)
    assert abs(loss - lr) < 1e-10
    scale = np.max(np.abs(gr))
    assert np.all(np.abs(g - gr) <= 1e-6 * np.maximum(np.abs(gr), 1e-3 * scale))
    assert np.max(np.abs(g - gr)) <= 1e-9 * scale


def test_adjoint_quadrature_self_check():
    tmpl, J, psi0, w = case(12, 6)
    m = P.Model(tmpl)
    p0 = torch.from_numpy(psi0).to(DEV)
    _, g8 = P.evolve_adjoint(m, J, p0, 0.1, w, substeps=2, quad_nodes=8)
    _, g16 = P.evolve_adjoint(m, J, p0, 0.1, w, substeps=2, quad_nodes=16)
    assert np.max(np.abs(g8 - g16)) <= 1e-11 * np.max(np.abs(g16))


def test_adjoint_vs_finite_differences_L20():
    """L = 20, 50 slices: sampled parameters by central differences (h = 1e-6) through the
    forward-only path with a fixed Krylov dimension (so the map is analytic in J)."""
    print("adjoint L=20 vs FD", flush=True)
    tmpl, J, psi0, w = case(20, 50)
    m = P.Model(tmpl)
    p0 = torch.from_numpy(psi0).to(DEV)
    kw = dict(substeps=2, m_fixed=20, m_max=30)
    loss, g = P.evolve_adjoint(m, J, p0, 0.1, w, quad_nodes=8, **kw)
    rng = np.random.default_rng(0)
    picks = [(49, 9), (0, 0), (25, 18)] + [tuple(x) for x in zip(rng.integers(0, 50, 5), rng.integers(0, 19, 5))]
    h = 1e-6
    scale = np.max(np.abs(g))
    for s, b in picks:
        Jp, Jm = J.copy(), J.copy()
        Jp[s, b] += h
        Jm[s, b] -= h
        fd = (P.evolve_loss(m, Jp, p0, 0.1, w, **kw) - P.evolve_loss(m, Jm, p0, 0.1, w, **kw)) / (2 * h)
        assert abs(g[s, b] - fd) <= 1e-6 * max(abs(fd), 1e-3 * scale), (s, b, g[s, b], fd)


def test_autograd_function():
    tmpl, J, psi0, w = case(8, 4)
    m = P.Model(tmpl)
    Jt = torch.from_numpy(J.copy()).requires_grad_(True)
    loss = P.AdjointEvolve.apply(Jt, m, torch.from_numpy(psi0).to(DEV), 0.1, w)
    (3.0 * loss).backward()
    _, gr = OA.gradient_eig(tmpl, J, psi0, 0.1, w)
    assert np.max(np.abs(Jt.grad.numpy() - 3.0 * gr)) <= 1e-9 * 3 * np.max(np.abs(gr))
