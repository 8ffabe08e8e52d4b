// Liouville-space evolution (Sec. ed:sec:Liouville, Eqs. ed:eq:lioutrafo, ed:eq:liousuperket, App. F): the
// density matrix of an L-site system as the superket |rho>> of 2L digits (row-major vec(rho): the
// row index is the high L bits, the column index the low L bits), and
//   i Lcal = H_eff (x) 1 - 1 (x) H_eff^* + i sum_nu gamma_nu J_nu (x) J_nu^*,
//   H_eff = H - (i/2) sum_nu gamma_nu J_nu^dagger J_nu,
// so that exp(-i t (i Lcal)) = exp(t Lcal) and the Krylov time step applies unchanged (Arnoldi:
// i Lcal is not Hermitian). The first two terms are a local operator on the 2L-bit chain (site and
// bond terms on the row half and on the column half, nothing on the middle bond) and run through
// the streaming H psi passes; the jump sandwiches couple row bit L + (L - k) with column bit L - k
// of the same site k, L bits apart, and are applied here as far terms by a gather pass.
#include <algorithm>
#include <cmath>
#include <vector>

#include "ed_internal.h"

namespace ed {
namespace {

constexpr int kFarThreads = 256;

// out[x] += sum_f sum_c K_f[r(x)][c] psi[x with bits (q_f, p_f) set to c], r(x) = 2 bit q + bit p
__global__ __launch_bounds__(kFarThreads) void far_terms(const double2* __restrict__ psi, double2* __restrict__ out,
                                                         const FarTerm* __restrict__ terms, int nterms, int64_t D) {
    for (int64_t x = int64_t(blockIdx.x) * kFarThreads + threadIdx.x; x < D; x += int64_t(gridDim.x) * kFarThreads) {
        double2 acc = out[x];
        for (int f = 0; f < nterms; ++f) {
            const int p = terms[f].p, q = terms[f].q;
            const uint32_t mask = terms[f].mask;
            const int r = int((((x >> q) & 1) << 1) | ((x >> p) & 1));
            const int64_t base = x & ~((int64_t(1) << p) | (int64_t(1) << q));
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if ((mask >> (4 * r + c)) & 1u) {
                    const int64_t y = base | (int64_t(c >> 1) << q) | (int64_t(c & 1) << p);
                    const double2 k = terms[f].K[4 * r + c];
                    const double2 v = psi[y];
                    acc.x = fma(k.x, v.x, fma(-k.y, v.y, acc.x));
                    acc.y = fma(k.x, v.y, fma(k.y, v.x, acc.y));
                }
            }
        }
        out[x] = acc;
    }
}

// one workgroup: res[0] = sum_j Re rho_jj, res[k] = sum_j Re rho_jj z_k(j) (site k at bit Ls - k of
// j, z = +1 for bit 0), in a fixed order
__global__ __launch_bounds__(256) void superket_diag_kernel(const double2* __restrict__ rho, int Ls,
                                                            double2* __restrict__ res) {
    __shared__ double red[256];
    const int64_t D = int64_t(1) << Ls;
    const int t = threadIdx.x;
    double acc[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) acc[i] = 0.0;
    for (int64_t j = t; j < D; j += 256) {
        const double v = rho[j * (D + 1)].x;
        acc[0] += v;
#pragma unroll
        for (int b = 0; b < 31; ++b)
            if (b < Ls) acc[1 + b] += ((j >> b) & 1) ? -v : v;
    }
    for (int i = 0; i <= Ls; ++i) {
        red[t] = acc[0];
#pragma unroll
        for (int b = 0; b < 31; ++b)
            if (i == 1 + b) red[t] = acc[1 + b];
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (t < h) red[t] += red[t + h];
            __syncthreads();
        }
        // bit b = i - 1 is site Ls - b
        if (t == 0) res[i == 0 ? 0 : Ls - (i - 1)] = make_double2(red[0], 0.0);
        __syncthreads();
    }
}

}  // namespace

ed_status launch_far_terms(const ed_model* m, const double2* psi, double2* out, hipStream_t s) {
    const int64_t D = int64_t(1) << m->L;
    const int64_t blocks = std::min<int64_t>((D + kFarThreads - 1) / kFarThreads, 4096);
    hipLaunchKernelGGL(far_terms, dim3(unsigned(blocks)), dim3(kFarThreads), 0, s, psi, out, m->d_far,
                       int(m->far.size()), D);
    ED_HIP_TRY(hipGetLastError());
    return ED_OK;
}

ed_status superket_diag(const double2* rho, int Ls, double2* res, hipStream_t s) {
    hipLaunchKernelGGL(superket_diag_kernel, dim3(1), dim3(256), 0, s, rho, Ls, res);
    ED_HIP_TRY(hipGetLastError());
    return ED_OK;
}

}  // namespace ed
