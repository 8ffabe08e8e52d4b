"""GPU parity of the Liouville-space path (Sec. ed:sec:Liouville, Eqs. ed:eq:lioutrafo, ed:eq:liousuperket,
App. F): the Liouvillian model's product i Lcal |rho>> against the oracle's Kronecker-built
superoperator, Arnoldi time steps against the oracle's exact propagation, and full-size
invariants (trace and Hermiticity preservation of any rho; the decay identity of the dissipative
XXZ chain, Eq. ed:eq:pjjexp).

Tolerances: products 1e-13 relative (as for H psi: a few dozen terms per entry); time evolution
1e-10 (Krylov tolerance 1e-12 per step); identities 1e-10 relative to the largest entry."""
import ctypes as C

import numpy as np
import pytest
import torch

import edinputs as E
import paper_1802_10052_amd as P
from oracle import hamiltonian as OH
from oracle import liouville as OLv

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SM = np.array([[0, 0], [1, 0]], np.complex128)


def to_dev(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


def jump_list(jops, rates, L):
    return [np.sqrt(rates[z][k]) * OH.site_operator(J, k + 1, L)
            for z, J in enumerate(jops) for k in range(L) if rates[z][k] != 0.0]


def case(L, seed):
    rng = np.random.default_rng(seed)
    desc = E.ModelDesc(L, site_ops=[E.SX, E.SZ], site_coef=rng.uniform(-1, 1, (2, L)),
                       bond_ops=[E.SXSX, E.SYSY, E.SZSZ], bond_coef=rng.uniform(-1, 1, (3, L - 1)))
    Jg = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    jops = [SM, E.SZ, Jg]
    rates = rng.uniform(0, 0.5, (3, L))
    rates[2, ::2] = 0.0   # the generic jump on every other site only
    return desc, jops, rates


def random_rho(L, seed):
    rng = np.random.default_rng(seed)
    D = 1 << L
    X = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    rho = X @ X.conj().T
    return rho / np.trace(rho).real


@pytest.mark.parametrize("L", [2, 3, 4, 6, 8])
def test_liouvillian_product(L):
    print(f"liouville apply L={L}", flush=True)
    desc, jops, rates = case(L, 10 + L)
    m = P.Liouville(desc, jops, rates)
    H = OH.hamiltonian_sparse(desc)
    Lc = OLv.liouvillian(H, jump_list(jops, rates, L))
    vec = OLv.superket(random_rho(L, 3)) + 0.1 * E.random_state(2 * L, 4)   # not Hermitian either
    ref = 1j * (Lc @ vec)
    got = P.apply_H(m, to_dev(vec)).cpu().numpy()
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13


@pytest.mark.parametrize("L", [7, 9])
def test_liouvillian_every_plan(L):
    """2L = 14 and 18 bits: several streaming plans, all with the jump gather pass after them."""
    print(f"liouville plans L={L}", flush=True)
    desc, jops, rates = case(L, 20 + L)
    m = P.Liouville(desc, jops, rates)
    Lc = OLv.liouvillian(OH.hamiltonian_sparse(desc), jump_list(jops, rates, L))
    vec = E.random_state(2 * L, 6)
    ref = 1j * (Lc @ vec)
    x = to_dev(vec)
    for i in range(m.plans[0]):
        m.select_plan(i)
        got = P.apply_H(m, x).cpu().numpy()
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13, (i, m.describe_plan(i))


@pytest.mark.parametrize("L", [3, 5])
def test_liouville_evolution_vs_oracle(L):
    print(f"liouville evolve L={L}", flush=True)
    desc, jops, rates = case(L, 30 + L)
    m = P.Liouville(desc, jops, rates)
    vec0 = OLv.superket(random_rho(L, 7))
    dt, steps = 0.1, 5
    refs = OLv.evolve_states(OH.hamiltonian_sparse(desc), jump_list(jops, rates, L), vec0, dt, steps)
    rho = to_dev(vec0)
    _, obs, info = P.krylov_evolve(m, rho, dt, steps, m_max=40, tol=1e-12, hermitian=False)
    assert np.linalg.norm(rho.cpu().numpy() - refs[-1]) < 1e-10
    for s, ref in enumerate(refs):
        sz, tr = OLv.measure(ref, L)
        assert np.abs(obs["sz"][s] - sz).max() < 1e-10
        assert abs(obs["norm"][s] - tr) < 1e-10
    sz, tr = P.liouville_measure(rho, L)
    assert abs(tr - 1.0) < 1e-10 and np.abs(sz - OLv.measure(refs[-1], L)[0]).max() < 1e-10
    # the same evolution with the observables written through device pointers
    rho2 = to_dev(vec0)
    _, obs2, _ = P.krylov_evolve(m, rho2, dt, steps, m_max=40, tol=1e-12, hermitian=False, device_obs=True)
    assert np.array_equal(obs2["sz"].cpu().numpy(), obs["sz"]) and np.array_equal(obs2["norm"].cpu().numpy(), obs["norm"])


def test_liouvillian_invariants_L14():
    """2^28 superket: for any rho, tr(Lcal rho) = 0, and for Hermitian rho, Lcal rho is Hermitian
    (so i Lcal rho is anti-Hermitian)."""
    L = 14
    D = 1 << L
    print("liouville invariants L=14", flush=True)
    desc, jops, rates = case(L, 44)
    m = P.Liouville(desc, jops, rates)
    g = torch.Generator(device=DEV)
    g.manual_seed(5)
    X = torch.randn((D, D), dtype=torch.complex128, device=DEV, generator=g)
    rho = X + X.conj().T.contiguous()
    del X
    torch.cuda.empty_cache()
    out = P.apply_H(m, rho.reshape(-1)).reshape(D, D)
    scale = out.abs().max().item()
    assert abs(torch.diagonal(out).sum().item()) < 1e-12 * scale * D
    herm = (out + out.conj().T).abs().max().item()
    assert herm < 1e-12 * scale, herm


def test_liouville_decay_identity_L14():
    """Dissipative XXZ (Delta = 1, gamma = 0.1 sigma^- on every site) from the Neel state, 2^28
    superket: N_up commutes with H, so sum_k <sigma^z_k>(t) = L (e^{-gamma t} - 1) exactly, and the
    trace stays 1."""
    L, gamma, dt, steps = 14, 0.1, 0.1, 5
    print("liouville decay identity L=14", flush=True)
    m = P.Liouville(E.xxz(L, 1.0, 1.0), [SM], np.full((1, L), gamma))
    D = 1 << L
    rho = torch.zeros(D * D, dtype=torch.complex128, device=DEV)
    n = E.neel_index(L)
    rho[n * D + n] = 1.0
    _, obs, info = P.krylov_evolve(m, rho, dt, steps, m_max=30, tol=1e-11, hermitian=False)
    t = dt * np.arange(steps + 1)
    assert np.abs(obs["sz"].sum(axis=1) - L * (np.exp(-gamma * t) - 1)).max() < 1e-9
    assert np.abs(obs["norm"] - 1.0).max() < 1e-10


def test_liouville_unsupported_paths():
    from paper_1802_10052_amd import _lib
    lib = _lib.lib()
    m = P.Liouville(E.xxz(4, 1.0, 1.0), [SM], np.full((1, 4), 0.1))
    n = C.c_int()
    assert lib.ed_model_liouville_sites(m.handle, C.byref(n)) == 0 and n.value == 4
    rho = torch.zeros(1 << 8, dtype=torch.complex128, device=DEV)
    with pytest.raises(P.EdError):
        P.lanczos_ground(m, rho)
    with pytest.raises(P.EdError):
        P.trotter_evolve(m, rho, 0.1, 1)
    with pytest.raises(ValueError):
        P.krylov_evolve(m, rho, 0.1, 1, hermitian=True)


def test_trajectory_ensemble_vs_liouville_L8():
    """The Liouville path as the exact reference of the batched trajectories (same Lindblad
    equation, Sec. ed:sec:open): 2048 GPU trajectories of the dissipative XXZ chain at L = 8 (dt = 0.01,
    T = 1) against the GPU superket evolution; every site's ensemble mean of <sigma^z_k>(t) lies
    within 4 standard errors (+1e-3) of tr(sigma^z_k rho(t))."""
    L, gamma, n_traj, dt, steps, stride, seed = 8, 0.1, 2048, 0.01, 100, 10, 21
    print("trajectory ensemble vs liouville L=8", flush=True)
    models = [P.Model(E.xxz(L, 1.0, 1.0))]
    psi0 = [to_dev(E.product_state(L, E.neel_index(L)))]
    mo = np.zeros(n_traj, np.int32)
    res = P.trajectories(models, E.SMINUS, [np.full(L, gamma)], psi0, mo, dt, steps, stride, seed, m_max=20,
                         tol=1e-10)
    sz = res["sz"][:, :, :L]
    mean = sz.mean(axis=0)
    se = sz.std(axis=0, ddof=1) / np.sqrt(n_traj)
    m = P.Liouville(E.xxz(L, 1.0, 1.0), [SM], np.full((1, L), gamma))
    D = 1 << L
    rho = torch.zeros(D * D, dtype=torch.complex128, device=DEV)
    n = E.neel_index(L)
    rho[n * D + n] = 1.0
    _, obs, _ = P.krylov_evolve(m, rho, dt * stride, steps // stride, m_max=30, tol=1e-12, hermitian=False)
    assert mean.shape == obs["sz"].shape
    assert np.all(np.abs(mean - obs["sz"]) < 4 * se + 1e-3), np.abs(mean - obs["sz"]).max()
