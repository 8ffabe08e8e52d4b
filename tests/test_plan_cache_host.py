"""Host checks of the tuned-plan cache of the C ABI (no GPU needed): entries put, read back,
saved to a file, cleared, and loaded again; malformed files are rejected with a message."""
import ctypes as C
import os

import pytest

from paper_1802_10052_amd import _lib


@pytest.fixture()
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libed.so not built")
    return _lib.lib()


def _get(lib, key):
    buf = C.create_string_buffer(256)
    code = lib.ed_plan_cache_get(key.encode(), buf, 256)
    return buf.value.decode() if code == 0 else None


def test_plan_cache_round_trip(lib, tmp_path):
    assert lib.ed_plan_cache_clear() == 0
    entries = {"gfx950 L=28 class=25 liouville=0 lr=0 far=0 cands=0123456789abcdef": "first +G5 wide | c4 h17 +G3",
               "gfx950 L=26 class=19 liouville=0 lr=0 far=0 cands=fedcba9876543210": "first +G6 | c4 h17 +G3 pair"}
    for k, v in entries.items():
        assert lib.ed_plan_cache_put(k.encode(), v.encode()) == 0
    for k, v in entries.items():
        assert _get(lib, k) == v
    assert _get(lib, "no such key") is None
    path = tmp_path / "plans.tsv"
    assert lib.ed_plan_cache_save(str(path).encode()) == 0
    text = path.read_text().splitlines()
    assert text[0].startswith("#") and sorted(text[1:]) == sorted(f"{k}\t{v}" for k, v in entries.items())
    assert lib.ed_plan_cache_clear() == 0
    assert _get(lib, next(iter(entries))) is None
    n = C.c_int()
    assert lib.ed_plan_cache_load(str(path).encode(), C.byref(n)) == 0 and n.value == 2
    for k, v in entries.items():
        assert _get(lib, k) == v
    # a later file overrides an entry
    path2 = tmp_path / "more.tsv"
    k0 = next(iter(entries))
    path2.write_text(f"# comment\n{k0}\tfirst +G6 wide | c4 h18 +G2 wide\n")
    assert lib.ed_plan_cache_load(str(path2).encode(), C.byref(n)) == 0 and n.value == 1
    assert _get(lib, k0) == "first +G6 wide | c4 h18 +G2 wide"
    lib.ed_plan_cache_clear()


def test_plan_cache_errors(lib, tmp_path):
    n = C.c_int()
    bad = tmp_path / "bad.tsv"
    bad.write_text("key without a tab\n")
    assert _lib.STATUS[lib.ed_plan_cache_load(str(bad).encode(), C.byref(n))] == "ED_ERR_ARG"
    assert b":1:" in lib.ed_last_error()
    assert _lib.STATUS[lib.ed_plan_cache_load(str(tmp_path / "missing.tsv").encode(), C.byref(n))] == "ED_ERR_ARG"
    assert _lib.STATUS[lib.ed_plan_cache_put(b"a\tb", b"plan")] == "ED_ERR_ARG"
    buf = C.create_string_buffer(4)
    assert lib.ed_plan_cache_put(b"k", b"a long plan description") == 0
    assert _lib.STATUS[lib.ed_plan_cache_get(b"k", buf, 4)] == "ED_ERR_ARG"
    lib.ed_plan_cache_clear()


def test_shipped_plan_table_parses(lib):
    path = _lib.DEFAULT_PLANS
    if not os.path.exists(path):
        pytest.skip("no shipped plan table")
    n = C.c_int()
    assert lib.ed_plan_cache_load(path.encode(), C.byref(n)) == 0 and n.value > 0
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        key, plan = line.rstrip("\n").split("\t")
        assert key.split()[0].startswith("gfx") and " L=" in key and "cands=" in key
        assert plan.startswith(("first", "small"))


def test_tune_keeps_the_faster_choice_per_key():
    """Models sharing a key keep the faster of their tuned plans (the earlier one on a tie)."""
    from paper_1802_10052_amd.tune_plans import keep_faster
    kept = {}
    assert keep_faster(kept, "k", 4.78, "first +G6 wide | c4 h18 +G2 wide") == "first +G6 wide | c4 h18 +G2 wide"
    assert keep_faster(kept, "k", 4.81, "first +G5 wide | c4 h17 +G3") == "first +G6 wide | c4 h18 +G2 wide"
    assert keep_faster(kept, "k", 4.78, "first +G5 wide | c4 h17 +G3") == "first +G6 wide | c4 h18 +G2 wide"
    assert keep_faster(kept, "k", 4.60, "first +G5 wide | c4 h17 +G3") == "first +G5 wide | c4 h17 +G3"
    assert kept["k"] == (4.60, "first +G5 wide | c4 h17 +G3")
    assert keep_faster(kept, "other", 9.0, "first | c4 h12") == "first | c4 h12"
