"""GPU parity of the quantum-trajectory paths (Sec. ed:sec:QT) against the oracle on the same Philox
streams, plus the closed forms that pin every trajectory of the dissipative XXZ chain:
from the Neel state with [H, N_up] = 0 the no-jump norm is exp(-gamma n t), so jump times follow
from the draws alone, and sum_k <sigma^z_k> = -2 (number of jumps so far) exactly."""
import numpy as np
import pytest
import torch

import edinputs as E
import paper_1802_10052_amd as P
from oracle import hamiltonian as OH
from oracle import trajectories as OT
from tests import closed_forms as CF

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GAMMA = 0.1


def setup_batch(lengths, n_traj, seed=4):
    models = [P.Model(E.xxz(L, 1.0, 1.0)) for L in lengths]
    rates = [np.full(L, GAMMA) for L in lengths]
    psi0 = [torch.from_numpy(E.product_state(L, E.neel_index(L))).to(DEV) for L in lengths]
    mo = np.array([t % len(lengths) for t in range(n_traj)], np.int32)
    return models, rates, psi0, mo


def expected_jump_times(seed, tr, L, T):
    d = OT.PhiloxDraws(seed, tr)
    n, t, out = L // 2, 0.0, []
    r = d.uniform()
    while n > 0:
        t = t - np.log(r) / (GAMMA * n)
        if t > T:
            break
        d.uniform()
        r = d.uniform()
        n -= 1
        out.append(t)
    return out


def test_philox_words_match_definition_and_numpy():
    w = P.philox_words(4, 123, 1 << 20)
    ref = np.random.Philox(key=[4, 123]).random_raw(1 << 20)
    assert np.array_equal(w, ref)
    first = CF.philox4x64_10([1, 0, 0, 0], [4, 123]) + CF.philox4x64_10([2, 0, 0, 0], [4, 123])
    assert [int(x) for x in w[:8]] == first


ORACLE_CASE = dict(lengths=[8, 10, 12], n_traj=6, dt=0.01, steps=200, stride=10, seed=4, compare=(1, 2, 3))


@pytest.fixture(scope="module")
def oracle_runs():
    """The oracle's trajectories 1, 2, 3 of the batch (L = 10, 12, 8; 4 jumps up to T = 2)."""
    c = ORACLE_CASE
    out = {}
    for tr in c["compare"]:
        L = c["lengths"][tr % len(c["lengths"])]
        print(f"  oracle trajectory {tr} (L={L})", flush=True)
        H = OH.hamiltonian_sparse(E.xxz(L, 1.0, 1.0))
        out[tr] = OT.trajectory(H, OT.lowering_jumps(L, GAMMA), E.product_state(L, E.neel_index(L)), c["dt"],
                                c["steps"], c["stride"], c["seed"], tr, tol=1e-12)
    return out


@pytest.mark.parametrize("plain", [False, True])
def test_trajectories_vs_oracle(plain, oracle_runs):
    c = ORACLE_CASE
    lengths, n_traj, dt, steps, stride, seed = c["lengths"], c["n_traj"], c["dt"], c["steps"], c["stride"], c["seed"]
    models, rates, psi0, mo = setup_batch(lengths, n_traj, seed)
    print(f"trajectories vs oracle plain={plain}", flush=True)
    res = P.trajectories(models, E.SMINUS, rates, psi0, mo, dt, steps, stride, seed, m_max=20, tol=1e-12,
                         plain=plain)
    print("  batched/plain call done", flush=True)
    assert sum(len(r["jumps"]) for r in oracle_runs.values()) >= 3
    for tr, ref in oracle_runs.items():
        L = lengths[mo[tr]]
        nj = res["n_jumps"][tr]
        assert nj == len(ref["jumps"]), (tr, nj, ref["jumps"])
        assert np.allclose(res["jump_t"][tr, :nj], [j[0] for j in ref["jumps"]], rtol=0, atol=1e-10)
        assert list(res["jump_site"][tr, :nj]) == [j[1] for j in ref["jumps"]]
        assert np.max(np.abs(res["sz"][tr, :, :L] - ref["sz"])) < 1e-9


CONFIG_LENGTHS = [8, 10, 12, 14, 16]
LARGE_CASE = dict(n_traj=60, dt=0.01, steps=100, stride=10, seed=4, per_length=2)


def _ids_with_most_jumps(L, c):
    """Trajectory ids of length L in the config's mix (L = lengths[t mod 5]) whose closed-form
    jump times put the most jumps inside T (so the compared runs cross thresholds and jump)."""
    ids = [t for t in range(c["n_traj"]) if CONFIG_LENGTHS[t % 5] == L]
    T = c["dt"] * c["steps"]
    ids.sort(key=lambda t: (-len(expected_jump_times(c["seed"], t, L, T)), t))
    return ids[:c["per_length"]]


@pytest.fixture(scope="module")
def large_oracle_runs():
    c = LARGE_CASE
    out = {}
    for L in (14, 16):
        H = OH.hamiltonian_sparse(E.xxz(L, 1.0, 1.0))
        for tr in _ids_with_most_jumps(L, c):
            print(f"  oracle trajectory {tr} (L={L})", flush=True)
            out[tr] = OT.trajectory(H, OT.lowering_jumps(L, GAMMA), E.product_state(L, E.neel_index(L)), c["dt"],
                                    c["steps"], c["stride"], c["seed"], tr, tol=1e-12)
    return out


@pytest.mark.parametrize("plain", [False, True])
def test_trajectories_vs_oracle_L14_L16(plain, large_oracle_runs):
    """Per-trajectory parity at the two longest chains of the batched workload, where a state
    spans several tiles of the trajectory kernel (4 at L = 14, 16 at L = 16): the config's mix of
    lengths in one call (60 trajectories, Delta = 1, gamma = 0.1, dt = 0.01, T = 1), and for two
    trajectories of each of L = 14 and 16 the jump count, times (1e-10), sites and per-site
    <sigma^z_k>(t) (1e-9) against the oracle on the same Philox streams."""
    c = LARGE_CASE
    models, rates, psi0, mo = setup_batch(CONFIG_LENGTHS, c["n_traj"], c["seed"])
    print(f"trajectories L=14/16 vs oracle plain={plain}", flush=True)
    res = P.trajectories(models, E.SMINUS, rates, psi0, mo, c["dt"], c["steps"], c["stride"], c["seed"], m_max=20,
                         tol=1e-12, plain=plain)
    print("  batched/plain call done", flush=True)
    assert res["info"]["unconverged_steps"] == 0
    checked_jumps = 0
    for tr, ref in large_oracle_runs.items():
        L = CONFIG_LENGTHS[mo[tr]]
        nj = res["n_jumps"][tr]
        assert nj == len(ref["jumps"]), (tr, nj, ref["jumps"])
        assert np.allclose(res["jump_t"][tr, :nj], [j[0] for j in ref["jumps"]], rtol=0, atol=1e-10)
        assert list(res["jump_site"][tr, :nj]) == [j[1] for j in ref["jumps"]]
        assert np.max(np.abs(res["sz"][tr, :, :L] - ref["sz"])) < 1e-9
        checked_jumps += nj
    assert checked_jumps >= 4


def test_trajectory_closed_forms_mixed_lengths():
    """The batched-trajectory workload (mixed L = 8..16, Delta = 1, gamma = 0.1, dt = 0.01) over T = 2."""
    lengths = [8, 10, 12, 14, 16]
    n_traj, dt, steps, stride, seed = 60, 0.01, 200, 10, 4
    models, rates, psi0, mo = setup_batch(lengths, n_traj, seed)
    print("trajectory closed forms", flush=True)
    res = P.trajectories(models, E.SMINUS, rates, psi0, mo, dt, steps, stride, seed, m_max=20, tol=1e-10)
    print("  batched call done", flush=True)
    n_out = steps // stride + 1
    times = np.arange(n_out) * dt * stride
    for tr in range(n_traj):
        L = lengths[mo[tr]]
        exp_t = expected_jump_times(seed, tr, L, dt * steps)
        nj = res["n_jumps"][tr]
        assert nj == len(exp_t), (tr, nj, exp_t)
        assert np.allclose(res["jump_t"][tr, :nj], exp_t, rtol=0, atol=1e-8)
        jumps_before = np.array([np.sum(np.array(exp_t) <= t) for t in times])
        tot = res["sz"][tr, :, :L].sum(axis=1)
        assert np.allclose(tot, -2.0 * jumps_before, atol=1e-8), tr
        # every jump lowers a different site (each site can decay once)
        assert len(set(res["jump_site"][tr, :nj])) == nj


def test_batched_equals_plain():
    lengths = [8, 12, 14]
    n_traj, dt, steps, stride, seed = 6, 0.01, 60, 5, 9
    models, rates, psi0, mo = setup_batch(lengths, n_traj, seed)
    a = P.trajectories(models, E.SMINUS, rates, psi0, mo, dt, steps, stride, seed)
    b = P.trajectories(models, E.SMINUS, rates, psi0, mo, dt, steps, stride, seed, plain=True)
    # the batched call again, after the plain path's eager work: a replay of the stream's graph
    a2 = P.trajectories(models, E.SMINUS, rates, psi0, mo, dt, steps, stride, seed)
    assert a2["info"]["graph_replayed"]
    for x in (a, a2):
        assert np.array_equal(x["n_jumps"], b["n_jumps"])
        assert np.max(np.abs(x["sz"] - b["sz"])) < 1e-10
        for tr in range(n_traj):
            nj = x["n_jumps"][tr]
            assert np.allclose(x["jump_t"][tr, :nj], b["jump_t"][tr, :nj], atol=1e-12)


def test_batched_deterministic():
    lengths = [10, 16]
    models, rates, psi0, mo = setup_batch(lengths, 8, 3)
    a = P.trajectories(models, E.SMINUS, rates, psi0, mo, 0.01, 50, 10, 3)
    b = P.trajectories(models, E.SMINUS, rates, psi0, mo, 0.01, 50, 10, 3)
    # the second call replays the stream's executable graph (updated with its own arguments)
    assert b["info"]["graph_replayed"]
    assert np.array_equal(a["sz"], b["sz"]) and np.array_equal(a["jump_t"], b["jump_t"])
    c = P.trajectories(models, E.SMINUS, rates, psi0, mo, 0.01, 50, 10, 3)
    assert c["info"]["graph_replayed"] and np.array_equal(a["sz"], c["sz"])
    # every workgroup reports its busy time; the plain path reports none
    bz = c["info"]["busy_ms"]
    assert 0.0 < bz["min"] <= bz["mean"] <= bz["max"], bz
