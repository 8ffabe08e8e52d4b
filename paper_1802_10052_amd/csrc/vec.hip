// Vector kernels of the Krylov methods (Sec. ed:sec:krylov and Sec. ed:sec:statics, computed matrix-free):
// deterministic dot products against several basis vectors at once, the matching multi-axpy,
// norm + scaling, the Krylov combination psi = sum_i c_i v_i, and the all-site <sigma^z>
// reduction of Sec. ed:sec:meas. Every reduction uses a fixed grid, a fixed per-thread assignment and a
// fixed tree, so results are bitwise reproducible from run to run.
#include "ed_vec.h"

namespace ed {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Block-reduce NA doubles per thread; thread i < NA of the block receives total i.
template <int NA>
__device__ __forceinline__ void block_sum(double (&a)[NA], double* lds /* kWaves * NA */) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        double s = wave_sum(a[i]);
        if (lane == 0) lds[wv * NA + i] = s;
    }
    __syncthreads();
    if (threadIdx.x < NA) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s += lds[w * NA + threadIdx.x];
        a[0] = s;
    }
    __syncthreads();
}

// Partial dots over block b's chunk: part[b][i] = sum_x conj(V_i[x]) * w[x], i < n <= kDotGroup.
template <int NG>
__global__ __launch_bounds__(kThreads) void dot_partial(const double2* __restrict__ V, int64_t ldv, int n,
                                                        const double2* __restrict__ w, int64_t D,
                                                        double2* __restrict__ part, int part_ld) {
    __shared__ double lds[kWaves * 2 * NG];
    double a[2 * NG];
#pragma unroll
    for (int i = 0; i < 2 * NG; ++i) a[i] = 0.0;
    const int64_t chunk = (D + gridDim.x - 1) / gridDim.x;
    const int64_t lo = int64_t(blockIdx.x) * chunk;
    const int64_t hi = lo + chunk < D ? lo + chunk : D;
    for (int64_t x = lo + threadIdx.x; x < hi; x += kThreads) {
        const double2 y = w[x];
#pragma unroll
        for (int i = 0; i < NG; ++i) {
            if (i < n) {
                const double2 v = V[int64_t(i) * ldv + x];
                a[2 * i] = fma(v.x, y.x, fma(v.y, y.y, a[2 * i]));
                a[2 * i + 1] = fma(v.x, y.y, fma(-v.y, y.x, a[2 * i + 1]));
            }
        }
    }
    block_sum<2 * NG>(a, lds);
    if (threadIdx.x < 2 * n) {
        double* p = reinterpret_cast<double*>(part + int64_t(blockIdx.x) * part_ld);
        p[threadIdx.x] = a[0];
    }
}

// Sum partials in fixed order: out[i] = scale * sum_b part[b][i] (+ out[i] if accumulate).
__global__ __launch_bounds__(kThreads) void reduce_partials(const double2* __restrict__ part, int part_ld,
                                                            int nblk, int n, double2* __restrict__ out,
                                                            int accumulate) {
    __shared__ double lds[kWaves * 2];
    for (int i = 0; i < n; ++i) {
        double a[2] = {0.0, 0.0};
        for (int b = threadIdx.x; b < nblk; b += kThreads) {
            const double2 v = part[int64_t(b) * part_ld + i];
            a[0] += v.x;
            a[1] += v.y;
        }
        block_sum<2>(a, lds);
        if (threadIdx.x < 2) {
            double* o = reinterpret_cast<double*>(out + i);
            o[threadIdx.x] = accumulate ? o[threadIdx.x] + a[0] : a[0];
        }
        __syncthreads();
    }
}

// w[x] += sign * sum_i coef[i] * V_i[x]  (coef in device memory)
template <int NG>
__global__ __launch_bounds__(kThreads) void multi_axpy(const double2* __restrict__ V, int64_t ldv, int n,
                                                       const double2* __restrict__ coef, double sign,
                                                       double2* __restrict__ w, int64_t D) {
    double2 c[NG];
#pragma unroll
    for (int i = 0; i < NG; ++i) c[i] = i < n ? coef[i] : make_double2(0.0, 0.0);
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t x = int64_t(blockIdx.x) * kThreads + threadIdx.x; x < D; x += stride) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < NG; ++i) {
            if (i < n) {
                const double2 v = V[int64_t(i) * ldv + x];
                acc.x = fma(c[i].x, v.x, fma(-c[i].y, v.y, acc.x));
                acc.y = fma(c[i].x, v.y, fma(c[i].y, v.x, acc.y));
            }
        }
        double2 y = w[x];
        y.x = fma(sign, acc.x, y.x);
        y.y = fma(sign, acc.y, y.y);
        w[x] = y;
    }
}

// out[x] = sum_i c_i V_i[x] (+ out[x] when accumulate), c given by value.
struct CombArgs {
    double2 c[kMaxComb];
};

__global__ __launch_bounds__(kThreads) void combine(const double2* __restrict__ V, int64_t ldv, int n,
                                                    CombArgs ca, double2* __restrict__ out, int64_t D,
                                                    int accumulate) {
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t x = int64_t(blockIdx.x) * kThreads + threadIdx.x; x < D; x += stride) {
        double2 acc = accumulate ? out[x] : make_double2(0.0, 0.0);
        for (int i = 0; i < n; ++i) {
            const double2 v = V[int64_t(i) * ldv + x];
            acc.x = fma(ca.c[i].x, v.x, fma(-ca.c[i].y, v.y, acc.x));
            acc.y = fma(ca.c[i].x, v.y, fma(ca.c[i].y, v.x, acc.y));
        }
        out[x] = acc;
    }
}

// norm^2 partials
__global__ __launch_bounds__(kThreads) void norm2_partial(const double2* __restrict__ w, int64_t D,
                                                          double2* __restrict__ part, int part_ld) {
    __shared__ double lds[kWaves];
    double a[1] = {0.0};
    const int64_t chunk = (D + gridDim.x - 1) / gridDim.x;
    const int64_t lo = int64_t(blockIdx.x) * chunk;
    const int64_t hi = lo + chunk < D ? lo + chunk : D;
    for (int64_t x = lo + threadIdx.x; x < hi; x += kThreads) {
        const double2 y = w[x];
        a[0] = fma(y.x, y.x, fma(y.y, y.y, a[0]));
    }
    block_sum<1>(a, lds);
    if (threadIdx.x == 0) part[int64_t(blockIdx.x) * part_ld] = make_double2(a[0], 0.0);
}

// dst[x] = src[x] * (1/sqrt(nrm2[0].x)) ; nrm2 is device memory
__global__ __launch_bounds__(kThreads) void scale_by_invnorm(const double2* __restrict__ src,
                                                             double2* __restrict__ dst,
                                                             const double2* __restrict__ nrm2, int64_t D) {
    const double s = 1.0 / sqrt(nrm2[0].x);
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t x = int64_t(blockIdx.x) * kThreads + threadIdx.x; x < D; x += stride) {
        double2 y = src[x];
        dst[x] = make_double2(y.x * s, y.y * s);
    }
}

// dst[x] = a * src[x] (complex a by value); src == dst is allowed (each element is read before
// the same thread writes it)
__global__ __launch_bounds__(kThreads) void scale_copy(const double2* src, double2* dst,
                                                       double2 a, int64_t D) {
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t x = int64_t(blockIdx.x) * kThreads + threadIdx.x; x < D; x += stride) {
        const double2 y = src[x];
        dst[x] = make_double2(a.x * y.x - a.y * y.y, a.x * y.y + a.y * y.x);
    }
}

// *dst = v (one scalar set on the stream, in order with the sweeps around it)
__global__ void set_value(double2* dst, double2 v) {
    if (threadIdx.x == 0) *dst = v;
}

// y[x] = a * x[x] + b * y[x] (complex a, b by value)
__global__ __launch_bounds__(kThreads) void axpby_kernel(const double2* __restrict__ xv, double2* __restrict__ y,
                                                         double2 a, double2 b, int64_t D) {
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t x = int64_t(blockIdx.x) * kThreads + threadIdx.x; x < D; x += stride) {
        const double2 u = xv[x], v = y[x];
        y[x] = make_double2(a.x * u.x - a.y * u.y + b.x * v.x - b.y * v.y,
                            a.x * u.y + a.y * u.x + b.x * v.y + b.y * v.x);
    }
}

// All-site <sigma^z> partials: part[b][0] = sum |psi|^2, part[b][1 + p] = sum |psi|^2 (1 - 2 bit_p).
// Blocks walk whole 2^kZBits-amplitude chunks: inside a chunk, bits 0..7 are fixed per thread,
// bits 8..11 follow the thread's loop counter and the bits above are constant.
constexpr int kZBits = 12;

__global__ __launch_bounds__(kThreads) void sz_partial(const double2* __restrict__ psi, int L,
                                                       double2* __restrict__ part, int part_ld) {
    __shared__ double lds[kWaves * 32];
    const int64_t D = int64_t(1) << L;
    const int cb = L < kZBits ? L : kZBits;
    const int64_t csize = int64_t(1) << cb;
    const int64_t nchunk = D >> cb;
    const int t = threadIdx.x;
    double acc[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) acc[i] = 0.0;
    for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
        double ct = 0.0;
        double cbits[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t i = t; i < csize; i += kThreads) {
            const double2 y = psi[(ch << cb) + i];
            const double q = fma(y.x, y.x, y.y * y.y);
            ct += q;
#pragma unroll
            for (int p = 8; p < 12; ++p) cbits[p - 8] += ((i >> p) & 1) ? -q : q;
        }
        acc[0] += ct;
#pragma unroll
        for (int p = 8; p < 12; ++p)
            if (p < cb) acc[1 + p] += cbits[p - 8];
#pragma unroll
        for (int p = 12; p < 31; ++p)
            if (p < L) acc[1 + p] += (((ch << cb) >> p) & 1) ? -ct : ct;
    }
#pragma unroll
    for (int p = 0; p < 8; ++p) acc[1 + p] = (p < cb) ? (((t >> p) & 1) ? -acc[0] : acc[0]) : 0.0;
    block_sum<32>(acc, lds);
    if (t < L + 1) part[int64_t(blockIdx.x) * part_ld + t] = make_double2(acc[0], 0.0);
}

// ---------------------------------------------------------------- scaled-basis kernels
// A Krylov basis is kept as (u_i, c_i) with v_i = c_i u_i, so normalising a new vector is a host
// scalar instead of a pass over the state. Vectors come as pointer lists (u_0 may be the caller's
// state itself).
struct VecPtrs {
    const double2* p[kDotGroup];
};
struct Scales {
    double s[kDotGroup];
};

// part[b][i] = sum_x conj(u_i[x]) w[x] over block b's chunk, i < n <= kDotGroup
template <int NG>
__global__ __launch_bounds__(kThreads) void dot_partial_ptr(VecPtrs U, int n, const double2* __restrict__ w,
                                                            int64_t D, double2* __restrict__ part, int part_ld) {
    __shared__ double lds[kWaves * 2 * NG];
    double a[2 * NG];
#pragma unroll
    for (int i = 0; i < 2 * NG; ++i) a[i] = 0.0;
    const int64_t chunk = (D + gridDim.x - 1) / gridDim.x;
    const int64_t lo = int64_t(blockIdx.x) * chunk;
    const int64_t hi = lo + chunk < D ? lo + chunk : D;
    for (int64_t x = lo + threadIdx.x; x < hi; x += kThreads) {
        const double2 y = w[x];
#pragma unroll
        for (int i = 0; i < NG; ++i) {
            if (i < n) {
                const double2 v = U.p[i][x];
                a[2 * i] = fma(v.x, y.x, fma(v.y, y.y, a[2 * i]));
                a[2 * i + 1] = fma(v.x, y.y, fma(-v.y, y.x, a[2 * i + 1]));
            }
        }
    }
    block_sum<2 * NG>(a, lds);
    if (threadIdx.x < 2 * n) {
        double* p = reinterpret_cast<double*>(part + int64_t(blockIdx.x) * part_ld);
        p[threadIdx.x] = a[0];
    }
}

// One sweep of w against up to kChunk basis vectors: w -= sum_i (s_i coef[i]) u_i (coef device,
// s host). Every element of w is read and written once whatever n is; the vectors are loaded 8
// at a time with all loads of a group issued before use. NORM: part[b][0] = sum |w_new|^2 over
// block b's chunk. KEEP (> 0): the values of the first KEEP vectors stay in registers and
// part[b][i] = sum conj(u_i) w_new over the chunk for i < min(n, KEEP): the dots of the next
// Gram-Schmidt pass, taken in the same sweep.
struct ChunkArgs {
    const double2* p[kChunk];
    double s[kChunk];
};

template <bool NORM, int KEEP>
__global__ __launch_bounds__(kThreads) void sub_sweep(ChunkArgs U, int n, const double2* __restrict__ coef,
                                                      double2* __restrict__ w, int64_t D,
                                                      double2* __restrict__ part, int part_ld) {
    constexpr int G = 8;
    constexpr int ND = 2 * KEEP;                       // dot components, then the norm
    constexpr int NA = ND + (NORM ? 1 : 0) > 0 ? ND + (NORM ? 1 : 0) : 1;
    __shared__ double2 cl[kChunk];
    __shared__ double lds[kWaves * NA];
    for (int i = threadIdx.x; i < n; i += kThreads) {
        const double2 k = coef[i];
        cl[i] = make_double2(U.s[i] * k.x, U.s[i] * k.y);
    }
    __syncthreads();
    double a[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) a[i] = 0.0;
    const int64_t chunk = (D + gridDim.x - 1) / gridDim.x;
    const int64_t lo = int64_t(blockIdx.x) * chunk;
    const int64_t hi = lo + chunk < D ? lo + chunk : D;
    for (int64_t x = lo + threadIdx.x; x < hi; x += kThreads) {
        double2 acc = w[x];
        double2 keep[KEEP > 0 ? KEEP : 1];
        int i0 = 0;
        if constexpr (KEEP > 0) {
#pragma unroll
            for (int i = 0; i < KEEP; ++i) keep[i] = U.p[i < n ? i : 0][x];
#pragma unroll
            for (int i = 0; i < KEEP; ++i) {
                if (i < n) {
                    acc.x -= cl[i].x * keep[i].x - cl[i].y * keep[i].y;
                    acc.y -= cl[i].x * keep[i].y + cl[i].y * keep[i].x;
                }
            }
            i0 = KEEP;
        }
        for (; i0 < n; i0 += G) {
            double2 v[G];
#pragma unroll
            for (int i = 0; i < G; ++i) v[i] = U.p[i0 + i < n ? i0 + i : i0][x];
#pragma unroll
            for (int i = 0; i < G; ++i) {
                if (i0 + i < n) {
                    const double2 c = cl[i0 + i];
                    acc.x -= c.x * v[i].x - c.y * v[i].y;
                    acc.y -= c.x * v[i].y + c.y * v[i].x;
                }
            }
        }
        w[x] = acc;
        if constexpr (KEEP > 0) {
#pragma unroll
            for (int i = 0; i < KEEP; ++i) {
                if (i < n) {
                    a[2 * i] = fma(keep[i].x, acc.x, fma(keep[i].y, acc.y, a[2 * i]));
                    a[2 * i + 1] = fma(keep[i].x, acc.y, fma(-keep[i].y, acc.x, a[2 * i + 1]));
                }
            }
        }
        if constexpr (NORM) a[ND] = fma(acc.x, acc.x, fma(acc.y, acc.y, a[ND]));
    }
    // block row: the dots of the first min(n, KEEP) vectors at entries 0.., the norm at entry KEEP
    if constexpr (KEEP > 0 || NORM) {
        block_sum<NA>(a, lds);
        const int nk = n < KEEP ? n : KEEP;
        double* p = reinterpret_cast<double*>(part + int64_t(blockIdx.x) * part_ld);
        if (threadIdx.x < 2 * nk) p[threadIdx.x] = a[0];
        if (NORM && threadIdx.x == ND) {
            p[ND] = a[0];
            p[ND + 1] = 0.0;
        }
    }
}

// out[x] = sum_i c_i u_i[x] (+ out[x] when accumulate); in place on out == u_0 is safe (each
// element is read before it is written by the same thread)
struct CombPtrs {
    const double2* p[kMaxComb];
    double2 c[kMaxComb];
};

__global__ __launch_bounds__(kThreads) void combine_ptr(CombPtrs cp, int n, double2* out, int64_t D, int accumulate) {
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t x = int64_t(blockIdx.x) * kThreads + threadIdx.x; x < D; x += stride) {
        double2 acc = accumulate ? out[x] : make_double2(0.0, 0.0);
        for (int i = 0; i < n; ++i) {
            const double2 v = cp.p[i][x];
            acc.x = fma(cp.c[i].x, v.x, fma(-cp.c[i].y, v.y, acc.x));
            acc.y = fma(cp.c[i].x, v.y, fma(cp.c[i].y, v.x, acc.y));
        }
        out[x] = acc;
    }
}

// out_o[x] = sum_i C[i * n_out + o] u_i[x] for o < n_out (real coefficients in device memory, staged
// in LDS). Every thread reads all inputs at its x before it writes its outputs at x, so the
// outputs may be any of the inputs (the pointers carry no restrict).
struct MultiPtrs {
    const double2* in[kMultiIn];
    double2* out[kMultiOut];
};

__global__ __launch_bounds__(kThreads) void combine_multi_kernel(MultiPtrs P, int n_in, int n_out,
                                                                 const double* __restrict__ C, int64_t D) {
    __shared__ double cs[kMultiIn * kMultiOut];
    for (int i = threadIdx.x; i < n_in * n_out; i += kThreads) cs[i] = C[i];
    __syncthreads();
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t x = int64_t(blockIdx.x) * kThreads + threadIdx.x; x < D; x += stride) {
        double2 acc[kMultiOut];
#pragma unroll
        for (int o = 0; o < kMultiOut; ++o) acc[o] = make_double2(0.0, 0.0);
        for (int i = 0; i < n_in; ++i) {
            const double2 v = P.in[i][x];
#pragma unroll
            for (int o = 0; o < kMultiOut; ++o) {
                if (o < n_out) {
                    const double c = cs[i * n_out + o];
                    acc[o].x = fma(c, v.x, acc[o].x);
                    acc[o].y = fma(c, v.y, acc[o].y);
                }
            }
        }
#pragma unroll
        for (int o = 0; o < kMultiOut; ++o)
            if (o < n_out) P.out[o][x] = acc[o];
    }
}

// dst[x] = src[x], one amplitude per thread, with streaming (non-temporal) stores: the plain device
// copy that sets the box's practical HBM streaming rate for the calibration of the benchmarks.
__global__ __launch_bounds__(kThreads) void stream_copy_kernel(const double2* __restrict__ src,
                                                               double2* __restrict__ dst, int64_t n) {
    const int64_t x = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (x < n) {
        const double2 v = src[x];
        double* o = reinterpret_cast<double*>(dst + x);
        __builtin_nontemporal_store(v.x, o);
        __builtin_nontemporal_store(v.y, o + 1);
    }
}

inline int grid_for(int64_t D) {
    int64_t g = D / (kThreads * 4);
    if (g < 1) g = 1;
    if (g > kRedBlocks) g = kRedBlocks;
    return int(g);
}

}  // namespace

int reduction_blocks(int64_t D) { return grid_for(D); }

hipError_t dots(const double2* V, int64_t ldv, int n, const double2* w, int64_t D, double2* out,
                double2* part, hipStream_t s) {
    const int G = grid_for(D);
    for (int i0 = 0; i0 < n; i0 += kDotGroup) {
        const int nn = n - i0 < kDotGroup ? n - i0 : kDotGroup;
        if (nn <= 4) {
            hipLaunchKernelGGL((dot_partial<4>), dim3(G), dim3(kThreads), 0, s, V + int64_t(i0) * ldv, ldv, nn, w, D, part, kPartLd);
        } else {
            hipLaunchKernelGGL((dot_partial<kDotGroup>), dim3(G), dim3(kThreads), 0, s, V + int64_t(i0) * ldv, ldv, nn, w, D, part, kPartLd);
        }
        hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kThreads), 0, s, part, kPartLd, G, nn, out + i0, 0);
    }
    return hipGetLastError();
}

hipError_t axpy_multi(const double2* V, int64_t ldv, int n, const double2* coef, double sign, double2* w,
                      int64_t D, hipStream_t s) {
    const int G = grid_for(D);
    for (int i0 = 0; i0 < n; i0 += kDotGroup) {
        const int nn = n - i0 < kDotGroup ? n - i0 : kDotGroup;
        if (nn <= 4) {
            hipLaunchKernelGGL((multi_axpy<4>), dim3(G), dim3(kThreads), 0, s, V + int64_t(i0) * ldv, ldv, nn, coef + i0, sign, w, D);
        } else {
            hipLaunchKernelGGL((multi_axpy<kDotGroup>), dim3(G), dim3(kThreads), 0, s, V + int64_t(i0) * ldv, ldv, nn, coef + i0, sign, w, D);
        }
    }
    return hipGetLastError();
}

hipError_t reduce_partial_rows(const double2* part, int nblk, int n, double2* out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kThreads), 0, s, part, kPartLd, nblk, n, out, 0);
    return hipGetLastError();
}

hipError_t norm2(const double2* w, int64_t D, double2* out, double2* part, hipStream_t s) {
    const int G = grid_for(D);
    hipLaunchKernelGGL(norm2_partial, dim3(G), dim3(kThreads), 0, s, w, D, part, kPartLd);
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kThreads), 0, s, part, kPartLd, G, 1, out, 0);
    return hipGetLastError();
}

hipError_t normalize(const double2* src, double2* dst, const double2* nrm2_dev, int64_t D, hipStream_t s) {
    hipLaunchKernelGGL(scale_by_invnorm, dim3(grid_for(D)), dim3(kThreads), 0, s, src, dst, nrm2_dev, D);
    return hipGetLastError();
}

hipError_t scale(const double2* src, double2* dst, double2 a, int64_t D, hipStream_t s) {
    hipLaunchKernelGGL(scale_copy, dim3(grid_for(D)), dim3(kThreads), 0, s, src, dst, a, D);
    return hipGetLastError();
}

hipError_t combination(const double2* V, int64_t ldv, int n, const double2* c, double2* out, int64_t D,
                       hipStream_t s) {
    for (int i0 = 0; i0 < n || i0 == 0; i0 += kMaxComb) {
        const int nn = n - i0 < kMaxComb ? n - i0 : kMaxComb;
        CombArgs ca;
        for (int i = 0; i < kMaxComb; ++i) ca.c[i] = i < nn ? c[i0 + i] : make_double2(0.0, 0.0);
        hipLaunchKernelGGL(combine, dim3(grid_for(D)), dim3(kThreads), 0, s, V + int64_t(i0) * ldv, ldv, nn, ca,
                           out, D, i0 > 0 ? 1 : 0);
        if (n == 0) break;
    }
    return hipGetLastError();
}

hipError_t axpby(const double2* x, double2* y, double2 a, double2 b, int64_t D, hipStream_t s) {
    hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(D)), dim3(kThreads), 0, s, x, y, a, b, D);
    return hipGetLastError();
}

hipError_t sz_all(const double2* psi, int L, double2* out, double2* part, hipStream_t s) {
    const int64_t D = int64_t(1) << L;
    const int cb = L < kZBits ? L : kZBits;
    int64_t nchunk = D >> cb;
    int G = int(nchunk < kSzBlocks ? nchunk : kSzBlocks);
    hipLaunchKernelGGL(sz_partial, dim3(G), dim3(kThreads), 0, s, psi, L, part, kPartLd);
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kThreads), 0, s, part, kPartLd, G, L + 1, out, 0);
    return hipGetLastError();
}

}  // namespace ed

namespace ed {

hipError_t sum_partials(const double2* part, int64_t n, double2* out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kThreads), 0, s, part, 1, int(n), 1, out, 0);
    return hipGetLastError();
}

hipError_t set_scalar(double2* dst, double2 v, hipStream_t s) {
    hipLaunchKernelGGL(set_value, dim3(1), dim3(64), 0, s, dst, v);
    return hipGetLastError();
}

hipError_t dots_ptr(const double2* const* U, int n, const double2* w, int64_t D, double2* out, double2* part,
                    hipStream_t s) {
    const int G = grid_for(D);
    for (int i0 = 0; i0 < n; i0 += kDotGroup) {
        const int nn = n - i0 < kDotGroup ? n - i0 : kDotGroup;
        VecPtrs vp;
        for (int i = 0; i < kDotGroup; ++i) vp.p[i] = i < nn ? U[i0 + i] : nullptr;
        if (nn <= 4) {
            hipLaunchKernelGGL((dot_partial_ptr<4>), dim3(G), dim3(kThreads), 0, s, vp, nn, w, D, part, kPartLd);
        } else {
            hipLaunchKernelGGL((dot_partial_ptr<kDotGroup>), dim3(G), dim3(kThreads), 0, s, vp, nn, w, D, part, kPartLd);
        }
        hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kThreads), 0, s, part, kPartLd, G, nn, out + i0, 0);
    }
    return hipGetLastError();
}

hipError_t axpy_norm_ptr(const double2* const* U, int n, const double2* coef, const double* scale, double2* w,
                         int64_t D, double2* nrm_out, double2* part, hipStream_t s) {
    const int G = grid_for(D);
    for (int i0 = 0; i0 < n || i0 == 0; i0 += kChunk) {
        const int nn = n - i0 < kChunk ? n - i0 : kChunk;
        const bool last = i0 + kChunk >= n;
        ChunkArgs ca;
        for (int i = 0; i < kChunk; ++i) {
            ca.p[i] = i < nn ? U[i0 + i] : nullptr;
            ca.s[i] = i < nn ? scale[i0 + i] : 0.0;
        }
        if (last) {
            hipLaunchKernelGGL((sub_sweep<true, 0>), dim3(G), dim3(kThreads), 0, s, ca, nn, coef + i0, w, D, part,
                               kPartLd);
            hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kThreads), 0, s, part, kPartLd, G, 1, nrm_out, 0);
        } else {
            hipLaunchKernelGGL((sub_sweep<false, 0>), dim3(G), dim3(kThreads), 0, s, ca, nn, coef + i0, w, D, part,
                               kPartLd);
        }
        if (n == 0) break;
    }
    return hipGetLastError();
}

hipError_t axpy_dots_ptr(const double2* const* U, int n, const double2* coef, const double* scale, double2* w,
                         int64_t D, double2* dots_out, double2* part, hipStream_t s) {
    if (n > kChunk) {
        // the subtraction takes several sweeps: dots afterwards, in their own sweeps
        for (int i0 = 0; i0 < n; i0 += kChunk) {
            const int nn = n - i0 < kChunk ? n - i0 : kChunk;
            ChunkArgs ca;
            for (int i = 0; i < kChunk; ++i) {
                ca.p[i] = i < nn ? U[i0 + i] : nullptr;
                ca.s[i] = i < nn ? scale[i0 + i] : 0.0;
            }
            hipLaunchKernelGGL((sub_sweep<false, 0>), dim3(grid_for(D)), dim3(kThreads), 0, s, ca, nn, coef + i0, w,
                               D, part, kPartLd);
        }
        return dots_ptr(U, n, w, D, dots_out, part, s);
    }
    const int G = grid_for(D);
    ChunkArgs ca;
    for (int i = 0; i < kChunk; ++i) {
        ca.p[i] = i < n ? U[i] : nullptr;
        ca.s[i] = i < n ? scale[i] : 0.0;
    }
    hipLaunchKernelGGL((sub_sweep<false, kKeepDots>), dim3(G), dim3(kThreads), 0, s, ca, n, coef, w, D, part,
                       kPartLd);
    const int nk = n < kKeepDots ? n : kKeepDots;
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kThreads), 0, s, part, kPartLd, G, nk, dots_out, 0);
    if (n > kKeepDots) return dots_ptr(U + kKeepDots, n - kKeepDots, w, D, dots_out + kKeepDots, part, s);
    return hipGetLastError();
}

hipError_t axpy_dots_norm_ptr(const double2* const* U, int n, const double2* coef, const double* scale, double2* w,
                              int64_t D, double2* dots_out, double2* nrm_out, int* ndots, double2* part,
                              hipStream_t s) {
    if (n > kChunk) {
        *ndots = 0;
        return axpy_norm_ptr(U, n, coef, scale, w, D, nrm_out, part, s);
    }
    const int G = grid_for(D);
    ChunkArgs ca;
    for (int i = 0; i < kChunk; ++i) {
        ca.p[i] = i < n ? U[i] : nullptr;
        ca.s[i] = i < n ? scale[i] : 0.0;
    }
    hipLaunchKernelGGL((sub_sweep<true, kKeepDots>), dim3(G), dim3(kThreads), 0, s, ca, n, coef, w, D, part, kPartLd);
    const int nk = n < kKeepDots ? n : kKeepDots;
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kThreads), 0, s, part, kPartLd, G, nk, dots_out, 0);
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kThreads), 0, s, part + kKeepDots, kPartLd, G, 1, nrm_out, 0);
    *ndots = nk;
    return hipGetLastError();
}

hipError_t combination_multi(const double2* const* U, int n_in, const double* C, double2* const* out, int n_out,
                             int64_t D, hipStream_t s) {
    if (n_in < 1 || n_in > kMultiIn || n_out < 1 || n_out > kMultiOut) return hipErrorInvalidValue;
    MultiPtrs P;
    for (int i = 0; i < kMultiIn; ++i) P.in[i] = i < n_in ? U[i] : nullptr;
    for (int o = 0; o < kMultiOut; ++o) P.out[o] = o < n_out ? out[o] : nullptr;
    hipLaunchKernelGGL(combine_multi_kernel, dim3(grid_for(D)), dim3(kThreads), 0, s, P, n_in, n_out, C, D);
    return hipGetLastError();
}

hipError_t combination_ptr(const double2* const* U, int n, const double2* c, double2* out, int64_t D, hipStream_t s) {
    // out may alias U[0] only when n <= kMaxComb (a single pass)
    for (int i0 = 0; i0 < n || i0 == 0; i0 += kMaxComb) {
        const int nn = n - i0 < kMaxComb ? n - i0 : kMaxComb;
        CombPtrs cp;
        for (int i = 0; i < kMaxComb; ++i) {
            cp.p[i] = i < nn ? U[i0 + i] : nullptr;
            cp.c[i] = i < nn ? c[i0 + i] : make_double2(0.0, 0.0);
        }
        hipLaunchKernelGGL(combine_ptr, dim3(grid_for(D)), dim3(kThreads), 0, s, cp, nn, out, D, i0 > 0 ? 1 : 0);
        if (n == 0) break;
    }
    return hipGetLastError();
}

}  // namespace ed

extern "C" ed_status ed_stream_copy(const ed_c64* src, ed_c64* dst, int64_t n, void* stream) {
    if (!src || !dst || n < 0) return ed::fail(ED_ERR_ARG, "bad argument (null pointer or n < 0)");
    if (n == 0) return ED_OK;
    const int64_t blocks = (n + ed::kThreads - 1) / ed::kThreads;
    if (blocks > int64_t(0x7fffffff)) return ed::fail(ED_ERR_ARG, "n too large for one launch");
    hipLaunchKernelGGL(ed::stream_copy_kernel, dim3(unsigned(blocks)), dim3(ed::kThreads), 0,
                       static_cast<hipStream_t>(stream), reinterpret_cast<const double2*>(src),
                       reinterpret_cast<double2*>(dst), n);
    ED_HIP_TRY(hipGetLastError());
    return ED_OK;
}
