// Small dense FP64 solvers (dense.cpp) for the projected Krylov matrices.
#pragma once
#include <complex>
#include <vector>

namespace ed {

using cplx = std::complex<double>;
// x87 extended precision (64-bit mantissa) for the tiny projected matrices of the Krylov steps
using xreal = long double;

bool tridiag_ql(int n, double* d, double* e, double* Z);
bool tridiag_ql_ext(int n, xreal* d, xreal* e, xreal* Z);
bool sym_eig_jacobi(int n, double* A, double* w, double* Z);
void tridiag_lowest(int n, const double* a, const double* b, double* theta, double* s);
void expm_complex(int n, const cplx* A, cplx* E);
void expm_col_sym(int n, const double* w, const double* Z, double tau, cplx* u);
void expm_col_sym_ext(int n, const xreal* w, const xreal* Z, double tau, cplx* u);

}  // namespace ed
