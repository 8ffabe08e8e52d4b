// Host launchers of the vector kernels (vec.hip). All pointers are device memory; `part` is a
// scratch area of kRedBlocks * kPartLd complex values taken from the caller's workspace (the
// sigma^z reduction uses at most kSzBlocks rows of it).
#pragma once
#include "ed_internal.h"

namespace ed {

constexpr int kRedBlocks = 4096;  // max blocks of a partial reduction (and of a vector sweep)
constexpr int kSzBlocks = 1024;   // max blocks of the all-site sigma^z reduction
constexpr int kPartLd = 64;       // complex entries per block row of the partial buffer
constexpr int kDotGroup = 16;     // basis vectors per dot/axpy launch
constexpr int kMaxComb = 64;      // max terms of a Krylov combination
constexpr int kChunk = 64;        // basis vectors per subtraction sweep
constexpr int kKeepDots = 16;     // dots of the next pass taken inside a subtraction sweep
constexpr int kMultiIn = 96;      // inputs of one multi-output combination
constexpr int kMultiOut = 8;      // outputs of one multi-output combination
constexpr size_t kPartBytes = size_t(kRedBlocks) * kPartLd * sizeof(double2);

int reduction_blocks(int64_t D);
// out[i] = <V_i|w>, i < n (V_i = V + i*ldv)
hipError_t dots(const double2* V, int64_t ldv, int n, const double2* w, int64_t D, double2* out,
                double2* part, hipStream_t s);
// w += sign * sum_i coef[i] V_i  (coef device)
hipError_t axpy_multi(const double2* V, int64_t ldv, int n, const double2* coef, double sign, double2* w,
                      int64_t D, hipStream_t s);
// out[i] = sum_b part[b][i] for i < n, b < nblk (fixed order)
hipError_t reduce_partial_rows(const double2* part, int nblk, int n, double2* out, hipStream_t s);
// out[0].x = |w|^2
hipError_t norm2(const double2* w, int64_t D, double2* out, double2* part, hipStream_t s);
// dst = src / sqrt(nrm2_dev[0].x)
hipError_t normalize(const double2* src, double2* dst, const double2* nrm2_dev, int64_t D, hipStream_t s);
// dst = a * src
hipError_t scale(const double2* src, double2* dst, double2 a, int64_t D, hipStream_t s);
// y = a x + b y  (complex a, b)
hipError_t axpby(const double2* x, double2* y, double2 a, double2 b, int64_t D, hipStream_t s);
// out = sum_i c[i] V_i  (c host; any n); out must not alias any V_i
hipError_t combination(const double2* V, int64_t ldv, int n, const double2* c, double2* out, int64_t D,
                       hipStream_t s);
// out[0].x = |psi|^2, out[1+p].x = sum |psi_x|^2 (1 - 2 bit_p(x))  (p = bit, site L-p)
hipError_t sz_all(const double2* psi, int L, double2* out, double2* part, hipStream_t s);

// out[0] = sum of part[0..n) in a fixed order
hipError_t sum_partials(const double2* part, int64_t n, double2* out, hipStream_t s);
// *dst = v, ordered on the stream like a kernel
hipError_t set_scalar(double2* dst, double2 v, hipStream_t s);

// Scaled-basis variants: vectors given as pointer lists.
// out[i] = <U_i|w>, i < n
hipError_t dots_ptr(const double2* const* U, int n, const double2* w, int64_t D, double2* out, double2* part,
                    hipStream_t s);
// w -= sum_i scale[i] coef[i] U_i (coef device, scale host); nrm_out[0].x = |w_new|^2. One sweep
// of w per kChunk vectors.
hipError_t axpy_norm_ptr(const double2* const* U, int n, const double2* coef, const double* scale, double2* w,
                         int64_t D, double2* nrm_out, double2* part, hipStream_t s);
// w -= sum_i scale[i] coef[i] U_i, then dots_out[i] = <U_i|w_new> for i < n; for n <= kChunk the
// subtraction and the dots of the first kKeepDots vectors share one sweep.
hipError_t axpy_dots_ptr(const double2* const* U, int n, const double2* coef, const double* scale, double2* w,
                         int64_t D, double2* dots_out, double2* part, hipStream_t s);
// w -= sum_i scale[i] coef[i] U_i in one sweep (n <= kChunk) that also gives dots_out[i] = <U_i|w_new>
// for i < *ndots = min(n, kKeepDots) and nrm_out[0].x = |w_new|^2; for n > kChunk only the
// subtraction and the norm (*ndots = 0).
hipError_t axpy_dots_norm_ptr(const double2* const* U, int n, const double2* coef, const double* scale, double2* w,
                              int64_t D, double2* dots_out, double2* nrm_out, int* ndots, double2* part,
                              hipStream_t s);
// out_o = sum_i C[i * n_out + o] U_i for o < n_out (C device, real, n_in x n_out row-major), in one
// sweep; outputs may alias inputs. n_in <= kMultiIn, n_out <= kMultiOut.
hipError_t combination_multi(const double2* const* U, int n_in, const double* C, double2* const* out, int n_out,
                             int64_t D, hipStream_t s);
// out = sum_i c[i] U_i (c host); out may be U_0 when n <= kMaxComb
hipError_t combination_ptr(const double2* const* U, int n, const double2* c, double2* out, int64_t D, hipStream_t s);

}  // namespace ed
