// Small dense FP64 solvers for the m x m projected matrices of the Krylov methods (m <= a few
// hundred): eigenpairs of real symmetric / tridiagonal matrices and the complex matrix
// exponential. These are the "exponential transformed to the Krylov basis" of Sec. III.C; they
// run on the host because m is tiny next to D.
#include "dense.h"

#include <algorithm>
#include <cmath>

namespace ed {

// Implicit symmetric QL with Wilkinson shifts on a tridiagonal matrix (Golub & Van Loan,
// Sec. 8.3). d[n] diagonal, e[n] sub-diagonal in e[0..n-2]. Z (n x n, row-major) is updated by
// the rotations (pass the identity to get the eigenvectors of T). Eigenvalues sorted ascending
// with the columns of Z. Returns false if an eigenvalue fails to converge in 60 sweeps.
bool tridiag_ql(int n, double* d, double* e, double* Z) {
    if (n <= 0) return true;
    e[n - 1] = 0.0;
    // An off-diagonal entry is dropped when it is negligible next to its two diagonal neighbours
    // or next to the whole matrix: the second test matters for graded spectra (a ground-state
    // Schmidt spectrum spans 1 .. 1e-30) whose tail sits at the rounding level of |T|, where a
    // purely relative test never fires. Dropping |e| <= 1e-17 |T| moves eigenvalues by less than
    // the rounding of the reduction that produced T.
    double tnorm = 0.0;
    for (int i = 0; i < n; ++i) tnorm = std::max(tnorm, std::fabs(d[i]) + 2.0 * std::fabs(e[i]));
    const double abs_tol = 1e-17 * tnorm;
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        while (true) {
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-17 * dd || std::fabs(e[m]) <= abs_tol || std::fabs(e[m]) < 1e-300) break;
            }
            if (m == l) break;
            if (++iter > 200) return false;
            // Wilkinson-type shift from the leading 2x2 block
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            bool early = false;
            for (; i >= l; --i) {
                double f = s * e[i];
                const double b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    early = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                if (Z) {
                    for (int k = 0; k < n; ++k) {
                        f = Z[k * n + i + 1];
                        Z[k * n + i + 1] = s * Z[k * n + i] + c * f;
                        Z[k * n + i] = c * Z[k * n + i] - s * f;
                    }
                }
            }
            if (early) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    // sort ascending
    for (int i = 0; i < n - 1; ++i) {
        int k = i;
        for (int j = i + 1; j < n; ++j)
            if (d[j] < d[k]) k = j;
        if (k != i) {
            std::swap(d[i], d[k]);
            if (Z)
                for (int r = 0; r < n; ++r) std::swap(Z[r * n + i], Z[r * n + k]);
        }
    }
    return true;
}

// Cyclic Jacobi for a dense real symmetric matrix A (row-major, destroyed). Eigenvalues
// ascending in w, eigenvectors in the columns of Z.
bool sym_eig_jacobi(int n, double* A, double* w, double* Z) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Z[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A[i * n + j] * A[i * n + j];
                if (i != j) off += A[i * n + j] * A[i * n + j];
            }
        if (off <= 1e-34 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[p * n + q];
                if (apq == 0.0) continue;
                const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // A <- A J
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // A <- J^T A
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double zkp = Z[k * n + p], zkq = Z[k * n + q];
                    Z[k * n + p] = c * zkp - s * zkq;
                    Z[k * n + q] = s * zkp + c * zkq;
                }
            }
        }
    }
    for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
    for (int i = 0; i < n - 1; ++i) {
        int k = i;
        for (int j = i + 1; j < n; ++j)
            if (w[j] < w[k]) k = j;
        if (k != i) {
            std::swap(w[i], w[k]);
            for (int r = 0; r < n; ++r) std::swap(Z[r * n + i], Z[r * n + k]);
        }
    }
    return true;
}

// Number of eigenvalues of the symmetric tridiagonal (a, b) smaller than x (Sturm count).
static int sturm_count(int n, const double* a, const double* b, double x) {
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < n; ++i) {
        const double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
        q = a[i] - x - (i > 0 ? bb / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// Lowest eigenpair of a symmetric tridiagonal matrix: bisection on the Sturm count to full
// precision, then inverse iteration for the eigenvector (unit norm, first nonzero positive).
void tridiag_lowest(int n, const double* a, const double* b, double* theta, double* s) {
    double lo = a[0], hi = a[0];
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < n - 1 ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(n, a, b, mid) >= 1) hi = mid;
        else lo = mid;
    }
    const double th = hi;
    *theta = th;
    if (!s) return;
    // inverse iteration: (T - th') y = x with a tiny perturbation of the shift
    const double scale = std::max(std::fabs(lo), std::fabs(hi)) + 1.0;
    const double shift = th - 1e-14 * scale;
    std::vector<double> dg(n), up(n), lw(n), x(n, 1.0), sub(n), sup(n);
    for (int it = 0; it < 3; ++it) {
        // solve (T - shift) y = x by Gaussian elimination with partial pivoting on the tridiagonal
        std::vector<double> d(n), du(n, 0.0), du2(n, 0.0), dl(n, 0.0), rhs(x);
        std::vector<int> piv(n, 0);
        for (int i = 0; i < n; ++i) d[i] = a[i] - shift;
        for (int i = 0; i < n - 1; ++i) {
            du[i] = b[i];
            dl[i] = b[i];
        }
        for (int i = 0; i < n - 1; ++i) {
            if (std::fabs(d[i]) >= std::fabs(dl[i])) {
                if (d[i] == 0.0) d[i] = 1e-300;
                const double f = dl[i] / d[i];
                dl[i] = f;
                d[i + 1] -= f * du[i];
                du2[i] = 0.0;
            } else {
                const double f = d[i] / dl[i];
                d[i] = dl[i];
                dl[i] = f;
                const double tmp = du[i];
                du[i] = d[i + 1];
                d[i + 1] = tmp - f * d[i + 1];
                if (i < n - 2) {
                    du2[i] = du[i + 1];
                    du[i + 1] = -f * du[i + 1];
                }
                piv[i] = 1;
            }
        }
        if (d[n - 1] == 0.0) d[n - 1] = 1e-300;
        for (int i = 0; i < n - 1; ++i) {
            if (piv[i]) std::swap(rhs[i], rhs[i + 1]);
            rhs[i + 1] -= dl[i] * rhs[i];
        }
        rhs[n - 1] /= d[n - 1];
        if (n > 1) rhs[n - 2] = (rhs[n - 2] - du[n - 2] * rhs[n - 1]) / d[n - 2];
        for (int i = n - 3; i >= 0; --i) rhs[i] = (rhs[i] - du[i] * rhs[i + 1] - du2[i] * rhs[i + 2]) / d[i];
        double nr = 0.0;
        for (int i = 0; i < n; ++i) nr += rhs[i] * rhs[i];
        nr = std::sqrt(nr);
        for (int i = 0; i < n; ++i) x[i] = rhs[i] / nr;
    }
    int k = 0;
    while (k < n && x[k] == 0.0) ++k;
    const double sg = (k < n && x[k] < 0.0) ? -1.0 : 1.0;
    for (int i = 0; i < n; ++i) s[i] = sg * x[i];
}

// exp(A) for a small complex matrix by scaling and squaring of the Taylor series: A is scaled
// by 2^-j so that |A|_1 <= 1/2, the series is summed until the terms stop contributing, and the
// result is squared j times.
void expm_complex(int n, const cplx* A, cplx* E) {
    double nrm = 0.0;
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += std::abs(A[i * n + j]);
        nrm = std::max(nrm, s);
    }
    int sq = 0;
    while (nrm > 0.5) {
        nrm *= 0.5;
        ++sq;
    }
    const double sc = std::ldexp(1.0, -sq);
    std::vector<cplx> As(size_t(n) * n), term(size_t(n) * n), tmp(size_t(n) * n);
    for (int i = 0; i < n * n; ++i) As[i] = A[i] * sc;
    for (int i = 0; i < n * n; ++i) {
        E[i] = 0.0;
        term[i] = 0.0;
    }
    for (int i = 0; i < n; ++i) {
        E[i * n + i] = 1.0;
        term[i * n + i] = 1.0;
    }
    for (int k = 1; k <= 40; ++k) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                cplx acc = 0.0;
                for (int l = 0; l < n; ++l) acc += term[i * n + l] * As[l * n + j];
                tmp[i * n + j] = acc / double(k);
            }
        double tn = 0.0;
        for (int i = 0; i < n * n; ++i) {
            term[i] = tmp[i];
            E[i] += tmp[i];
            tn = std::max(tn, std::abs(tmp[i]));
        }
        if (tn < 1e-18) break;
    }
    for (int s = 0; s < sq; ++s) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                cplx acc = 0.0;
                for (int l = 0; l < n; ++l) acc += E[i * n + l] * E[l * n + j];
                tmp[i * n + j] = acc;
            }
        for (int i = 0; i < n * n; ++i) E[i] = tmp[i];
    }
}

// First column of exp(-i tau T) for a real symmetric T given by its eigenpairs (w, Z):
// u = Z diag(exp(-i tau w)) Z^T e_1.
void expm_col_sym(int n, const double* w, const double* Z, double tau, cplx* u) {
    for (int i = 0; i < n; ++i) {
        cplx acc = 0.0;
        for (int k = 0; k < n; ++k) acc += Z[i * n + k] * std::exp(cplx(0.0, -tau * w[k])) * Z[0 * n + k];
        u[i] = acc;
    }
}

}  // namespace ed
