"""Host checks of the library's small dense solvers (dense.cpp), compiled with g++ on the CPU
(with AddressSanitizer and UndefinedBehaviorSanitizer) and compared with LAPACK/scipy on the same
matrices."""
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
    } else if (mode == 4) {  // tridiagonal QR, values only
        std::vector<double> d(n), e(n);
        for (auto& v : d) scanf("%lf", &v);
        for (int i = 0; i < n - 1; ++i) scanf("%lf", &e[i]);
        if (!tridiag_ql(n, d.data(), e.data(), nullptr)) return 2;
        for (double v : d) printf("%.17g\n", v);
    } else if (mode == 5) {  // exp(-i tau T) e_1 from the extended-precision eigenpairs
        double tau; if (scanf("%lf", &tau) != 1) return 1;
        std::vector<xreal> d(n), e(n, 0.0L), Z(n * n, 0.0L);
        for (auto& v : d) { double x; scanf("%lf", &x); v = x; }
        for (int i = 0; i < n - 1; ++i) { double x; scanf("%lf", &x); e[i] = x; }
        for (int i = 0; i < n; ++i) Z[i * n + i] = 1.0L;
        if (!tridiag_ql_ext(n, d.data(), e.data(), Z.data())) return 2;
        std::vector<cplx> u(n);
        expm_col_sym_ext(n, d.data(), Z.data(), tau, u.data());
        for (int i = 0; i < n; ++i) printf("%.17g\n", double(d[i]));
        for (auto v : u) printf("%.17g %.17g\n", v.real(), v.imag());
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
    # built with AddressSanitizer and UndefinedBehaviorSanitizer: any out-of-bounds access or
    # undefined operation in the solvers ends the driver with an error, which fails the test
    subprocess.run([gxx, "-O2", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", f"-I{CSRC}", str(src), os.path.join(CSRC, "dense.cpp"),
                    "-o", str(exe)], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")

    def run(inp):
        r = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True, env=env)
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


def _ql(driver, a, b):
    n = len(a)
    out = driver(f"0 {n} " + _fmt(a, b))
    w = np.array([float(x[0]) for x in out[:n]])
    Z = np.array([float(x[0]) for x in out[n:]]).reshape(n, n)
    return w, Z


def test_tridiag_qr_special_matrices(driver):
    """Closed forms and hard cases for the implicit QR: the 2x2 block, a matrix that splits into
    blocks (exact zero couplings), the Wilkinson matrix W21+ (eigenvalue pairs that agree to
    1e-14), and the second-difference matrix with eigenvalues 2 - 2 cos(k pi / (n + 1))."""
    # 2 x 2: eigenvalues (a+c)/2 -+ sqrt(((a-c)/2)^2 + b^2)
    a, b, c = 0.3, -1.7, 2.2
    w, Z = _ql(driver, np.array([a, c]), np.array([b]))
    m, r = 0.5 * (a + c), np.hypot(0.5 * (a - c), b)
    assert np.allclose(w, [m - r, m + r], rtol=0, atol=1e-15)
    T = np.array([[a, b], [b, c]])
    assert np.allclose(T @ Z, Z * w, atol=1e-14) and np.allclose(Z.T @ Z, np.eye(2), atol=1e-15)
    # split blocks
    a = np.array([1.0, 4.0, -2.0, 0.5, 3.0, 3.0])
    b = np.array([0.5, 0.0, 1.0, 0.0, 1e-3])
    w, Z = _ql(driver, a, b)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    assert np.allclose(w, np.linalg.eigvalsh(T), atol=1e-15)
    assert np.allclose(T @ Z, Z * w, atol=1e-14)
    # Wilkinson W21+
    a = np.abs(np.arange(-10, 11)).astype(float)
    b = np.ones(20)
    w, Z = _ql(driver, a, b)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    assert np.allclose(w, sla.eigvalsh_tridiagonal(a, b), atol=2e-14)
    assert np.allclose(Z.T @ Z, np.eye(21), atol=1e-13)
    assert np.allclose(T @ Z, Z * w, atol=1e-13)
    # second difference, n = 300
    n = 300
    w, Z = _ql(driver, 2.0 * np.ones(n), -np.ones(n - 1))
    exact = 2.0 - 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    assert np.max(np.abs(w - exact)) < 1e-13


def test_tridiag_qr_graded_vectors(driver):
    """Eigenvectors of a graded (1 .. 1e-30) tridiagonal: orthonormal to rounding and with
    residuals at the rounding level of |T|, as the Krylov time step and the adjoint need."""
    rng = np.random.default_rng(5)
    n = 120
    lam = np.exp(-np.linspace(0, 69, n)) * rng.choice([-1.0, 1.0], n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    from scipy.linalg import hessenberg
    T = hessenberg((Q * lam) @ Q.T)
    a, b = np.diag(T).copy(), np.diag(T, -1).copy()
    w, Z = _ql(driver, a, b)
    Tt = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    # backward-stable level: a few tens of ulps of |T| = 1 for n = 120
    assert np.max(np.abs(w - sla.eigvalsh_tridiagonal(a, b))) < 1e-14
    assert np.max(np.abs(Z.T @ Z - np.eye(n))) < 1e-13
    assert np.max(np.abs(Tt @ Z - Z * w)) < 1e-14


def test_tridiag_qr_large_values_only(driver):
    """n = 4096 without vectors (the size class of the entropy's tridiagonal): random entries and
    a Schmidt-like graded spectrum, both against LAPACK."""
    rng = np.random.default_rng(6)
    n = 4096
    a, b = rng.standard_normal(n), rng.standard_normal(n - 1)
    drv_in = f"4 {n} " + _fmt(a, b)
    out = driver(drv_in)
    w = np.array([float(x[0]) for x in out])
    ref = sla.eigvalsh_tridiagonal(a, b)
    assert np.max(np.abs(w - ref)) < 1e-12
    # graded: diagonal 1 .. 1e-30 with couplings at the geometric mean scale
    d = np.exp(-np.linspace(0, 69, n))
    e = 0.3 * np.sqrt(d[:-1] * d[1:])
    out = driver(f"4 {n} " + _fmt(d, e))
    w = np.array([float(x[0]) for x in out])
    ref = sla.eigvalsh_tridiagonal(d, e)
    assert np.max(np.abs(w - ref)) < 1e-13 * np.max(np.abs(ref))   # eps |T| times a modest p(n)
    assert np.all(w[:-1] <= w[1:])


def test_tridiag_ext_expm_column(driver):
    """The extended-precision instance: eigenvalues against LAPACK and exp(-i tau T) e_1 against
    scipy's expm of the same tridiagonal, to FP64 rounding."""
    rng = np.random.default_rng(7)
    for n, tau in ((1, 0.3), (2, 0.05), (20, 0.05), (40, 0.5)):
        a, b = 5 * rng.standard_normal(n), 5 * rng.standard_normal(max(n - 1, 0))
        out = driver(f"5 {n} {tau!r} " + _fmt(a, b))
        w = np.array([float(x[0]) for x in out[:n]])
        u = np.array([float(x[0]) + 1j * float(x[1]) for x in out[n:]])
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        assert np.allclose(w, np.linalg.eigvalsh(T), rtol=0, atol=1e-13 * max(1, np.max(np.abs(a))))
        ref = sla.expm(-1j * tau * T)[:, 0]
        assert np.max(np.abs(u - ref)) < 1e-14
