"""Host-side checks of the reduced-density-matrix path (no GPU): the pass plan of ed_rdm
evaluates every pair of index bits exactly once with at most 32 pairs per pass (and the
single-site plan every bit once, at most 12 per pass), the argument checks, and ed_trace_distances against numpy's
Hermitian eigenvalues and the oracle's trace distance."""
import ctypes as C

import numpy as np
import pytest

import paper_1802_10052_amd as P
from oracle import rdm as OR
from paper_1802_10052_amd import _lib


@pytest.mark.parametrize("L", range(2, 31))
def test_plan_covers_every_pair_once(L):
    pairs, pass_of = P.rdm_plan(L)
    got = sorted(map(tuple, pairs.tolist()))
    assert got == [(p, q) for p in range(L) for q in range(p + 1, L)]
    assert np.bincount(pass_of).max() <= 32
    bits, bpass = P.rdm_plan_sites(L)
    assert sorted(bits.tolist()) == list(range(L))
    assert np.bincount(bpass).max() <= 12
    assert bpass.max() + 1 == max(1, -(-(L - 4) // 8))


def test_pass_counts():
    """C(m, 2) tiles of 4 low bits + two groups of 4 high bits cover all pairs: m = 6 at L = 28;
    tiles of 4 low bits + 8 others cover every single site in ceil(24 / 8) = 3 passes."""
    assert P.rdm_plan(28)[1].max() + 1 == 15
    assert P.rdm_plan_sites(28)[1].max() + 1 == 3
    assert P.rdm_plan(12)[1].max() + 1 == 3   # one tile, 66 pairs in 3 passes


def test_argument_errors():
    lib = _lib.lib()
    nb = C.c_size_t()
    assert lib.ed_rdm_workspace(1, C.byref(nb)) == -1
    assert lib.ed_rdm_workspace(31, C.byref(nb)) == -1
    assert lib.ed_rdm_workspace(28, C.byref(nb)) == 0 and nb.value == 28 * 27 // 2 * 128 + 32 * 1024 * 96 + 1025 * 4096 * 8
    assert lib.ed_rdm(None, 10, None, None, None, 0, None) == -1
    assert lib.ed_rdm_plan_pairs(1, None, 0, None) == -1
    assert lib.ed_rdm_plan_sites(31, None, 0, None) == -1
    assert lib.ed_trace_distances(0, 1, None, None, None) == -1
    assert lib.ed_trace_distances(2, 1, None, None, None) == -1
    assert lib.ed_trace_distances(2, 0, None, None, None) == 0


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16])
def test_trace_distances_vs_eigvalsh(n):
    rng = np.random.default_rng(n)
    count = 12
    def herm():
        a = rng.standard_normal((count, n, n)) + 1j * rng.standard_normal((count, n, n))
        return 0.5 * (a + np.conj(np.swapaxes(a, 1, 2)))
    a, b = herm(), herm()
    got = P.trace_distances(a, b)
    ref = np.array([0.5 * np.abs(np.linalg.eigvalsh(x - y)).sum() for x, y in zip(a, b)])
    assert np.abs(got - ref).max() < 1e-13 * max(1.0, ref.max())
    ref2 = np.array([OR.trace_distance(x, y) for x, y in zip(a, b)])
    assert np.abs(got - ref2).max() < 1e-13 * max(1.0, ref.max())


def test_trace_distance_density_matrices():
    """Pure states: D = sqrt(1 - |<u|v>|^2); equal matrices: 0; orthogonal projectors: 1."""
    rng = np.random.default_rng(3)
    u, v = [x / np.linalg.norm(x) for x in rng.standard_normal((2, 4)) + 1j * rng.standard_normal((2, 4))]
    d = P.trace_distances(np.outer(u, u.conj()), np.outer(v, v.conj()))[0]
    assert abs(d - np.sqrt(1 - abs(np.vdot(u, v)) ** 2)) < 1e-14
    assert P.trace_distances(np.outer(u, u.conj()), np.outer(u, u.conj()))[0] == 0.0
    assert P.trace_distances(np.diag([1.0, 0]), np.diag([0, 1.0]))[0] == 1.0
