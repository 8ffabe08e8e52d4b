"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer. libed_san.so
(the same sources with the host code instrumented; paper_1802_10052_amd/build.py) runs the CPU
boundary tests in a subprocess with the sanitizer runtime preloaded: an invalid memory access or
an undefined operation in the host code they reach (argument checks, pass planning for every
length, the long-range and Liouville validation, the plan cache's parser and writer, the RDM
wave-program replay) ends that run with an error report."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BOUNDARY_TESTS = ["tests/test_capi.py", "tests/test_plan_cache_host.py", "tests/test_rdm_plan_host.py"]


def _sanitized_library():
    from paper_1802_10052_amd import build as b
    try:
        rt = b.asan_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    srcs = glob.glob(os.path.join(b.CSRC, "*")) + [os.path.join(ROOT, "include", "ed.h")]
    if not os.path.exists(b.SAN_LIB) or os.path.getmtime(b.SAN_LIB) < max(os.path.getmtime(f) for f in srcs):
        b.build(sanitize=True)
    return rt, b.SAN_LIB


def test_boundary_tests_under_host_sanitizers():
    rt, lib = _sanitized_library()
    env = dict(os.environ, LD_PRELOAD=rt, ED_LIB=lib, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    # the sanitized build is the one the binding maps
    probe = ("import paper_1802_10052_amd._lib as L; L.lib(); "
             "print(any(l.rstrip().endswith('libed_san.so') for l in open('/proc/self/maps')))")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("True"), r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *BOUNDARY_TESTS], cwd=ROOT,
                       env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
