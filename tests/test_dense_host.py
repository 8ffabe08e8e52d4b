"""Host checks of the library's small dense solvers (dense.cpp), compiled with g++ on the CPU
and compared with LAPACK/scipy on the same matrices."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.linalg as sla

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1802_10052_amd", "csrc")

DRIVER = r'''
#include "dense.h"
#include <cstdio>
#include <vector>
using namespace ed;
int main() {
    int mode, n; if (scanf("%d %d", &mode, &n) != 2) return 1;
    if (mode == 0) {  // tridiagonal QL with vectors
        std::vector<double> d(n), e(n), Z(n * n, 0.0);
        for (auto& v : d) scanf("%lf", &v);
        for (int i = 0; i < n - 1; ++i) scanf("%lf", &e[i]);
        for (int i = 0; i < n; ++i) Z[i * n + i] = 1.0;
        tridiag_ql(n, d.data(), e.data(), Z.data());
        for (double v : d) printf("%.17g\n", v);
        for (double v : Z) printf("%.17g\n", v);
    } else if (mode == 1) {  // Jacobi
        std::vector<double> A(n * n), w(n), Z(n * n);
        for (auto& v : A) scanf("%lf", &v);
        sym_eig_jacobi(n, A.data(), w.data(), Z.data());
        for (double v : w) printf("%.17g\n", v);
        for (double v : Z) printf("%.17g\n", v);
    } else if (mode == 2) {  // lowest eigenpair of a tridiagonal
        std::vector<double> a(n), b(n), s(n); double th;
        for (auto& v : a) scanf("%lf", &v);
        for (int i = 0; i < n - 1; ++i) scanf("%lf", &b[i]);
        tridiag_lowest(n, a.data(), b.data(), &th, s.data());
        printf("%.17g\n", th);
        for (double v : s) printf("%.17g\n", v);
    } else {  // complex expm
        std::vector<cplx> A(n * n), E(n * n);
        for (auto& v : A) { double re, im; scanf("%lf %lf", &re, &im); v = cplx(re, im); }
        expm_complex(n, A.data(), E.data());
        for (auto v : E) printf("%.17g %.17g\n", v.real(), v.imag());
    }
    return 0;
}
'''


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("dense")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run([gxx, "-O2", "-std=c++17", f"-I{CSRC}", str(src), os.path.join(CSRC, "dense.cpp"), "-o", str(exe)],
                   check=True)
    def run(inp):
        r = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
        return np.array([list(map(float, l.split())) for l in r.stdout.strip().splitlines()], dtype=object)
    return run


def _fmt(*arrs):
    return " ".join(" ".join(f"{v:.17g}" for v in np.ravel(a)) for a in arrs)


def test_tridiag_ql(driver):
    rng = np.random.default_rng(0)
    for n in (1, 2, 7, 40):
        a, b = rng.standard_normal(n), rng.standard_normal(max(n - 1, 0))
        out = driver(f"0 {n} " + _fmt(a, b))
        w = np.array([float(x[0]) for x in out[:n]])
        Z = np.array([float(x[0]) for x in out[n:]]).reshape(n, n)
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        assert np.allclose(w, np.linalg.eigvalsh(T), atol=1e-13)
        assert np.allclose(T @ Z, Z * w, atol=1e-12)


def test_jacobi(driver):
    rng = np.random.default_rng(1)
    for n in (3, 25):
        A = rng.standard_normal((n, n))
        A = A + A.T
        out = driver(f"1 {n} " + _fmt(A))
        w = np.array([float(x[0]) for x in out[:n]])
        Z = np.array([float(x[0]) for x in out[n:]]).reshape(n, n)
        assert np.allclose(w, np.linalg.eigvalsh(A), atol=1e-12)
        assert np.allclose(A @ Z, Z * w, atol=1e-11)


def test_tridiag_lowest(driver):
    rng = np.random.default_rng(2)
    for n in (1, 5, 150):
        a, b = rng.standard_normal(n), rng.standard_normal(max(n - 1, 0))
        out = driver(f"2 {n} " + _fmt(a, b))
        th = float(out[0][0])
        s = np.array([float(x[0]) for x in out[1:]])
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        w, V = np.linalg.eigh(T)
        assert abs(th - w[0]) < 1e-13 * max(1, abs(w[0]))
        assert abs(abs(s @ V[:, 0]) - 1) < 1e-10


def test_expm_complex(driver):
    rng = np.random.default_rng(3)
    for n, sc in ((1, 1.0), (6, 0.3), (20, 3.0)):
        A = sc * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
        out = driver(f"3 {n} " + " ".join(f"{v.real:.17g} {v.imag:.17g}" for v in A.ravel()))
        E = np.array([float(x[0]) + 1j * float(x[1]) for x in out]).reshape(n, n)
        ref = sla.expm(A)
        assert np.linalg.norm(E - ref) <= 1e-13 * np.linalg.norm(ref)


def test_tridiag_ql_graded_spectrum(driver):
    """A Schmidt-like spectrum 1 .. 1e-30 hidden in a tridiagonal matrix with rounding-level
    couplings: QL must converge and reproduce LAPACK to the rounding level of |T|."""
    rng = np.random.default_rng(4)
    n = 400
    lam = np.exp(-np.linspace(0, 70, n))
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * lam) @ Q.T
    from scipy.linalg import hessenberg
    T = hessenberg(A)                       # symmetric -> tridiagonal up to rounding
    a, b = np.diag(T).copy(), np.diag(T, -1).copy()
    out = driver(f"0 {n} " + _fmt(a, b))
    w = np.array([float(x[0]) for x in out[:n]])
    ref = sla.eigvalsh_tridiagonal(a, b)
    assert np.max(np.abs(w - ref)) < 2e-14 * np.max(np.abs(ref))
