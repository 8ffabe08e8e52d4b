// Small dense FP64 solvers (dense.cpp) for the projected Krylov matrices.
#pragma once
#include <complex>
#include <vector>

namespace ed {

using cplx = std::complex<double>;

bool tridiag_ql(int n, double* d, double* e, double* Z);
bool sym_eig_jacobi(int n, double* A, double* w, double* Z);
void tridiag_lowest(int n, const double* a, const double* b, double* theta, double* s);
void expm_complex(int n, const cplx* A, cplx* E);
void expm_col_sym(int n, const double* w, const double* Z, double tau, cplx* u);

}  // namespace ed
