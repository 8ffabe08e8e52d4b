"""GPU parity of ed_apply_H against the oracle's explicit sparse H (Sec. ed:sec:krylov, Eq. ed:eq:OKrylov).

Relative 2-norm error <= 1e-13: both sides sum at most 3L+1 products per entry in float64, so
the rounding difference is a few ulp of the largest term."""
import os

import numpy as np
import pytest
import torch

import edinputs as E
import paper_1802_10052_amd as P
from oracle import hamiltonian as OH

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def models(L):
    return {
        "tfim": E.tfim(L, 0.5),
        "xxz": E.xxz(L, 1.0, 0.5, E.random_fields(L, 2)),
        "generic": E.random_model(L, seed=40 + L, hermitian=False),
        "xxz_decay": E.ModelDesc(L, site_ops=[E.SZ, -0.5j * E.NUP], site_coef=np.stack([E.random_fields(L, 3), np.full(L, 0.1)]),
                                 bond_ops=[E.SXSX, E.SYSY, E.SZSZ], bond_coef=np.ones((3, L - 1))),
    }


def to_dev(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


@pytest.mark.parametrize("L", [2, 3, 5, 8, 11, 12, 13, 14, 15, 17, 20, 21])
@pytest.mark.parametrize("kind", ["tfim", "xxz", "generic", "xxz_decay"])
def test_apply_H_parity(L, kind):
    print(f"apply_H parity L={L} kind={kind}", flush=True)
    desc = models(L)[kind]
    psi = E.random_state(L, 11)
    ref = OH.apply_H(desc, psi)
    m = P.Model(desc)
    out = P.apply_H(m, to_dev(psi))
    got = out.cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 1e-13, (L, kind, err, m.passes)


@pytest.mark.parametrize("L,kind", [(22, "generic"), (25, "xxz"), (25, "generic"), (26, "tfim"), (26, "xxz"),
                                    (26, "generic"), (27, "xxz_decay"), (28, "tfim"), (28, "xxz"), (28, "generic")])
def test_apply_H_sampled_entries_large(L, kind):
    """Sampled entries at sizes where the pass plan uses gathered bits (L >= 25: G = L - 24 in the
    window pass; the first pass gathers 4 bits from L = 21 on)."""
    print(f"apply_H sampled L={L} kind={kind}", flush=True)
    desc = models(L)[kind]
    psi = E.random_state(L, 11)
    m = P.Model(desc)
    assert m.passes == (2 if L <= 28 else 3)
    out = P.apply_H(m, to_dev(psi)).cpu().numpy()
    rng = np.random.default_rng(5)
    xs = np.concatenate([rng.integers(0, 1 << L, 4000), [0, (1 << L) - 1, 1 << (L - 1), (1 << 12) - 1, 1 << 12]])
    ref = OH.apply_H_entries(desc, psi, xs)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(out[xs] - ref)) < 1e-13 * scale * L


def test_apply_H_hermitian_property_large():
    """<phi|H psi> = conj(<psi|H phi>) for Hermitian H at L = 26 (holds at any size)."""
    L = 26
    desc = E.xxz(L, 1.0, 0.5, E.random_fields(L, 2))
    m = P.Model(desc)
    phi = to_dev(E.random_state(L, 21))
    psi = to_dev(E.random_state(L, 22))
    a = torch.vdot(phi, P.apply_H(m, psi)).item()
    b = torch.vdot(psi, P.apply_H(m, phi)).item()
    assert abs(a - b.conjugate()) < 1e-11


def test_apply_H_deterministic():
    L = 20
    m = P.Model(E.random_model(L, seed=3))
    psi = to_dev(E.random_state(L, 1))
    a = P.apply_H(m, psi)
    b = P.apply_H(m, psi)
    assert torch.equal(a, b)


def _plan_model(L, kind):
    """Models for the plan tests: 'flip' has single and double bond flips (passes overlap by one
    bit); 'rtfim' is a disordered transverse-field Ising chain (no bond flips: passes edge to
    edge, real kernel variant); 'cfield' has complex site fields and no bond flips (edge-to-edge
    passes on the general kernel variant, whose bond masks are then empty)."""
    rng = np.random.default_rng(100 + L)
    if kind == "flip":
        return E.random_model(L, seed=9, hermitian=False)
    if kind == "rtfim":
        return E.ModelDesc(L, site_ops=[E.SX], site_coef=rng.uniform(-1.5, -0.5, (1, L)),
                           bond_ops=[E.SZSZ], bond_coef=rng.uniform(-1.5, -0.5, (1, L - 1)))
    return E.ModelDesc(L, site_ops=[E.SX, E.SY, E.SZ], site_coef=rng.uniform(-1, 1, (3, L)),
                       bond_ops=[E.SZSZ], bond_coef=rng.uniform(-1, 1, (1, L - 1)))


@pytest.mark.parametrize("L,kind", [(21, "flip"), (21, "rtfim"), (21, "cfield"), (25, "flip"), (25, "rtfim"),
                                    (25, "cfield"), (28, "rtfim"), (28, "flip")])
def test_apply_H_every_candidate_plan(L, kind):
    """Every candidate pass plan of the autotuner computes the same H psi (sampled entries against
    the oracle; whole vectors against each other to rounding), and tuning selects one of them."""
    print(f"apply_H plans L={L} {kind}", flush=True)
    desc = _plan_model(L, kind)
    psi_h = E.random_state(L, 3)
    psi = to_dev(psi_h)
    m = P.Model(desc)
    n, sel = m.plans
    # a new model starts on the tuned plan cached under its key, else on the planner's first
    cached = P.plan_cache_get(m.plan_key)
    expect = 0 if cached is None else [m.describe_plan(i) for i in range(n)].index(cached)
    assert n >= 2 and sel == expect, (sel, cached)
    rng = np.random.default_rng(1)
    xs = rng.integers(0, 1 << L, 2000)
    ref = OH.apply_H_entries(desc, psi_h, xs)
    first = None
    for i in range(n):
        m.select_plan(i)
        print(f"  plan {i}: {m.describe_plan(i)}", flush=True)
        out = P.apply_H(m, psi)
        got = out[torch.from_numpy(xs).to(DEV)].cpu().numpy()
        assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref)) * L, (L, i)
        if first is None:
            first = out
        else:
            assert (torch.linalg.vector_norm(out - first) / torch.linalg.vector_norm(first)).item() < 1e-14
        del out
    best, times = m.tune(psi, reps=2)
    assert 0 <= best < n and len(times) == n and all(t > 0 for t in times)
    assert m.plans[1] == best
    assert P.plan_cache_get(m.plan_key) == m.describe_plan(best)
    if cached is not None:      # keep the shipped choice for the models created after this test
        P.plan_cache_put(m.plan_key, cached)


def test_tuned_plan_cache_selects_at_creation(tmp_path):
    """ed_model_tune stores its choice; a new model of the same kind created after the cache is
    saved, cleared and reloaded starts on that plan; a model of another L does not match it."""
    L = 22
    P.plan_cache_clear()
    m = P.Model(E.tfim(L, 0.5))
    psi = E.random_state_device(L, 11, DEV)
    best, ms = m.tune(psi, reps=1)
    key, desc = m.plan_key, m.describe_plan(best)
    assert key.startswith("gfx") and f" L={L} " in key
    assert P.plan_cache_get(key) == desc
    path = tmp_path / "plans.tsv"
    P.plan_cache_save(path)
    P.plan_cache_clear()
    assert P.Model(E.tfim(L, 0.5)).plans[1] == 0        # no entry: the planner's first candidate
    assert P.plan_cache_load(path) == 1
    m2 = P.Model(E.tfim(L, 0.5))
    assert m2.describe_plan() == desc and m2.plans[1] == best
    assert P.Model(E.tfim(L + 2, 0.5)).plan_key != key
    P.plan_cache_clear()
    P.plan_cache_load(P._lib.DEFAULT_PLANS) if os.path.exists(P._lib.DEFAULT_PLANS) else None
