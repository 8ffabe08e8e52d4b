// Small dense solvers for the m x m projected matrices of the Krylov methods (m <= a few
// hundred): eigenpairs of real symmetric / tridiagonal matrices and the complex matrix
// exponential. These are the "exponential transformed to the Krylov basis" of Sec. ed:sec:krylov; they
// run on the host because m is tiny next to D. The tridiagonal eigensolver also has an x87
// extended-precision instance: the Krylov time step and the adjoint's bases form
// exp(-i tau T) e_1 with it, so that the coefficients carry FP64 rounding only (not the
// eigensolver's backward error, a few ulps of |T|) and the propagation is a smooth function of
// the couplings at the level of FP64 rounding.
#include "dense.h"

#include <algorithm>
#include <cmath>
#include <limits>

namespace ed {

// Eigenvalues (and optionally eigenvectors) of a real symmetric tridiagonal matrix by the
// implicit symmetric QR algorithm with Wilkinson shifts (Golub & Van Loan, "Matrix
// Computations", Algorithms 8.3.2 and 8.3.3). d[n] holds the diagonal, e[0..n-2] the
// off-diagonal (e[i] couples rows i and i+1); both are overwritten, d with the eigenvalues in
// ascending order. Z (n x n, row-major) may be null; otherwise it is multiplied on the right by
// every rotation, so passing the identity returns the eigenvectors in its columns, sorted with
// the eigenvalues. Returns false if the active block has not split after 50 sweeps per
// eigenvalue on average.
//
// Structure: the trailing end of the unreduced part is found by scanning upward from the bottom
// for a negligible off-diagonal entry; the block above it that is still coupled gets one QR sweep
// (shift from its trailing 2 x 2, then a Givens rotation that introduces a bulge below the
// diagonal and a chain of rotations that chases it off the bottom of the block).
namespace {

// Off-diagonal entry e between diagonals a and b counts as zero when it is below the rounding of
// its neighbours, or below the rounding of the whole matrix. The second test matters for graded
// spectra (a ground-state Schmidt spectrum spans 1 .. 1e-30): their tail sits at the rounding
// level of |T|, where a purely relative test never fires, and dropping |e| <= 1e-17 |T| moves
// no eigenvalue by more than the rounding of the reduction that produced T.
template <typename R>
inline bool negligible(R e, R a, R b, R rel_tol, R abs_tol) {
    const R ae = std::fabs(e);
    return ae <= rel_tol * (std::fabs(a) + std::fabs(b)) || ae <= abs_tol || ae < R(1e-300);
}

// Eigenvalue of the 2 x 2 block [[a, b], [b, c]] closer to c (the Wilkinson shift), written so
// that it does not cancel: c - b^2 / (delta + sign(delta) sqrt(delta^2 + b^2)), delta = (a - c)/2.
template <typename R>
inline R wilkinson_shift(R a, R b, R c) {
    const R delta = R(0.5) * (a - c);
    const R root = std::hypot(delta, b);
    const R den = delta >= R(0) ? delta + root : delta - root;
    if (den == R(0)) return c;  // b = 0 and a = c
    return c - b * (b / den);
}

// One implicit QR sweep with shift mu on the block lo..hi (hi > lo, all e[lo..hi-1] nonzero).
// The rotation in the plane (k, k+1) is G = [[c, s], [-s, c]], applied as T <- G T G^T; the
// first one is fixed by the shifted first column (d[lo] - mu, e[lo]), each later one zeroes the
// bulge T(k+1, k-1) left by its predecessor against T(k, k-1).
template <typename R>
void qr_sweep(int n, int lo, int hi, R mu, R* d, R* e, R* Z) {
    R x = d[lo] - mu;  // entry the rotation keeps
    R z = e[lo];       // entry the rotation removes
    for (int k = lo; k < hi; ++k) {
        const R r = std::hypot(x, z);
        R c = 1, s = 0;
        if (r != R(0)) {
            c = x / r;
            s = z / r;
        }
        if (k > lo) e[k - 1] = r;  // T(k, k-1) after the bulge is removed
        // similarity on rows/columns k, k+1 of the 2 x 2 diagonal block [[a, b], [b, f]]
        const R a = d[k], b = e[k], f = d[k + 1];
        const R cc = c * c, ss = s * s, cs = c * s;
        d[k] = cc * a + R(2) * cs * b + ss * f;
        d[k + 1] = ss * a - R(2) * cs * b + cc * f;
        e[k] = cs * (f - a) + (cc - ss) * b;
        if (k + 1 < hi) {
            // row k+2 only couples to column k+1: the rotation spreads it onto column k (bulge)
            const R g = e[k + 1];
            z = s * g;
            e[k + 1] = c * g;
            x = e[k];
        }
        if (Z) {
            for (int row = 0; row < n; ++row) {
                R* zr = Z + size_t(row) * n;
                const R u = zr[k], v = zr[k + 1];
                zr[k] = c * u + s * v;
                zr[k + 1] = c * v - s * u;
            }
        }
    }
}

// The whole algorithm for one real type. Rounding-level tolerances scale with the type's epsilon
// (eps / 22, about 1e-17 for double).
template <typename R>
bool tridiag_qr(int n, R* d, R* e, R* Z) {
    if (n <= 0) return true;
    e[n - 1] = 0;
    const R rel_tol = std::numeric_limits<R>::epsilon() / R(22);
    R tnorm = 0;
    for (int i = 0; i < n; ++i) tnorm = std::max(tnorm, std::fabs(d[i]) + R(2) * std::fabs(e[i]));
    const R abs_tol = rel_tol * tnorm;
    long sweeps = 0;
    const long max_sweeps = 50L * n;
    int hi = n - 1;  // rows hi+1.. are converged
    while (hi > 0) {
        if (negligible(e[hi - 1], d[hi - 1], d[hi], rel_tol, abs_tol)) {
            e[hi - 1] = 0;
            --hi;
            continue;
        }
        int lo = hi - 1;  // grow the unreduced block upward
        while (lo > 0 && !negligible(e[lo - 1], d[lo - 1], d[lo], rel_tol, abs_tol)) --lo;
        if (lo > 0) e[lo - 1] = 0;
        if (++sweeps > max_sweeps) return false;
        qr_sweep(n, lo, hi, wilkinson_shift(d[hi - 1], e[hi - 1], d[hi]), d, e, Z);
    }
    // ascending order, carrying the eigenvector columns along
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int i, int j) { return d[i] < d[j]; });
    std::vector<R> w(d, d + n);
    for (int i = 0; i < n; ++i) d[i] = w[order[i]];
    if (Z) {
        std::vector<R> row(n);
        for (int r = 0; r < n; ++r) {
            R* zr = Z + size_t(r) * n;
            for (int i = 0; i < n; ++i) row[i] = zr[order[i]];
            std::copy(row.begin(), row.end(), zr);
        }
    }
    return true;
}

}  // namespace

bool tridiag_ql(int n, double* d, double* e, double* Z) { return tridiag_qr<double>(n, d, e, Z); }

bool tridiag_ql_ext(int n, xreal* d, xreal* e, xreal* Z) { return tridiag_qr<xreal>(n, d, e, Z); }

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

// The same column from eigenpairs held in extended precision; the sums run in extended precision
// and only the result is rounded to double.
void expm_col_sym_ext(int n, const xreal* w, const xreal* Z, double tau, cplx* u) {
    std::vector<xreal> cr(n), ci(n);
    for (int k = 0; k < n; ++k) {
        const xreal ph = xreal(tau) * w[k];
        cr[k] = std::cos(ph) * Z[k];  // Z[0 * n + k]
        ci[k] = -std::sin(ph) * Z[k];
    }
    for (int i = 0; i < n; ++i) {
        xreal re = 0, im = 0;
        for (int k = 0; k < n; ++k) {
            re += Z[size_t(i) * n + k] * cr[k];
            im += Z[size_t(i) * n + k] * ci[k];
        }
        u[i] = cplx(double(re), double(im));
    }
}

}  // namespace ed
