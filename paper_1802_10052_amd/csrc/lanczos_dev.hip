// Device-resident Lanczos ground state for short chains (Sec. ed:sec:statics, by the Lanczos recurrence
// of Sec. ed:sec:krylov): with full reorthogonalisation and no restart, the whole recurrence runs in
// one cooperative launch instead of a dozen launches and a host round trip per product.
//
// G workgroups of kLT threads own consecutive slices of the state, one amplitude per thread. A
// product w = H v_j takes every term per amplitude (partners read from the whole of v_j), then
// classical Gram-Schmidt runs twice against v_0..v_j: each workgroup writes its partial dot
// products, and after a grid barrier every workgroup sums all of them in the same order (so all
// hold identical coefficients). beta_j = |w| comes the same way and v_{j+1} = w / beta_j. Every
// kLCheck products workgroup 0 tests convergence on T_m (the lowest eigenvalue by multisection on
// Sturm counts, the last component of its eigenvector by inverse iteration); the decision is
// written before the next barrier and read by every workgroup after it, so all stop together.
// The barrier is a monotone counter with a bounded wait: a workgroup that waits too long flags an
// error and every workgroup leaves, so the launch always ends.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <vector>

#include "ed_vec.h"
#include "hpsi_device.h"
#include "krylov_core.h"

namespace ed {
namespace {

constexpr int kLT = 256;                    // threads per workgroup
constexpr int kLCheck = 8;                  // products between convergence tests
constexpr unsigned kSpinLimit = 1u << 26;   // barrier polls before giving up
constexpr int kDevMaxVec = 512;             // basis vectors the kernel's LDS coefficients hold

struct DevLzArgs {
    const double2* site;
    const double2* bond;
    int L;
    int64_t D;
    double2* V;     // basis slots 0..nmax (slot 0 holds the normalised start vector)
    int nmax;       // at most nmax products
    double2* p1;    // partial dots of the first pass [G][pld]
    double2* p2;    // partial dots of the second pass [G][pld]
    int pld;
    double* pn;     // partial squared norms [G]
    double* alpha;  // [nmax]
    double* beta;   // [nmax]
    unsigned* bar;  // barrier counter, zero at launch
    int* ctl;       // [0] error flag, [1] basis size at convergence (0: not yet), [2] products done
    double tol;
};

__device__ __forceinline__ int ld_ctl(int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier number gen + 1: the counter reaches (gen + 1) G once every workgroup has arrived.
// Returns false (and flags the error) when the wait exceeds the limit or another workgroup failed.
__device__ bool grid_sync(const DevLzArgs& a, unsigned& gen, int* bad) {
    __syncthreads();
    if (threadIdx.x == 0) {
        *bad = 0;
        __threadfence();
        atomicAdd(a.bar, 1u);
        const unsigned target = (gen + 1) * gridDim.x;
        unsigned spins = 0;
        while (__hip_atomic_load(a.bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (ld_ctl(a.ctl) != 0 || ++spins > kSpinLimit) {
                atomicExch(a.ctl, 1);
                *bad = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
    }
    ++gen;
    __syncthreads();
    return *bad == 0;
}

// part[i] (i < n) = sum over the workgroup's amplitudes of conj(V_i[x]) w, in groups of 16 vectors:
// each wave forms the 16 sums with one transposing butterfly (a lane keeps half of its values at
// each exchange), then the 4 waves are added in order.
__device__ void block_dots(const double2* V, int64_t D, int n, int64_t x, bool xok, double2 w, double2* part,
                           double2 (*red)[16]) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int i0 = 0; i0 < n; i0 += 16) {
        double2 r[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            r[q] = make_double2(0.0, 0.0);
            if (xok && i0 + q < n) {
                const double2 v = V[int64_t(i0 + q) * D + x];
                r[q] = make_double2(v.x * w.x + v.y * w.y, v.x * w.y - v.y * w.x);
            }
        }
#pragma unroll
        for (int h = 8, o = 32; h >= 1; h >>= 1, o >>= 1) {
            const bool up = (lane & o) != 0;
#pragma unroll
            for (int q = 0; q < h; ++q) {
                const double2 keep = up ? r[q + h] : r[q];
                const double2 send = up ? r[q] : r[q + h];
                r[q].x = keep.x + __shfl_xor(send.x, o, 64);
                r[q].y = keep.y + __shfl_xor(send.y, o, 64);
            }
        }
#pragma unroll
        for (int o = 2; o >= 1; o >>= 1) {
            r[0].x += __shfl_xor(r[0].x, o, 64);
            r[0].y += __shfl_xor(r[0].y, o, 64);
        }
        if ((lane & 3) == 0) red[wv][(lane >> 2) & 15] = r[0];
        __syncthreads();
        if (t < 16 && i0 + t < n) {
            double2 s = red[0][t];
            for (int k = 1; k < kLT / 64; ++k) {
                s.x += red[k][t].x;
                s.y += red[k][t].y;
            }
            part[i0 + t] = s;
        }
        __syncthreads();
    }
}

// coef[i] (LDS, i < n) = sum over the G workgroups of part[b][i], the same sum on every workgroup:
// four lanes per coefficient take the rows b = k, k + 4, ... (their loads issued in groups of 8),
// and the four sums are added in lane order.
__device__ void sum_partials(const double2* part, int pld, int G, int n, double2* coef) {
    const int t = threadIdx.x, k = t & 3;
    for (int i0 = 0; i0 < n; i0 += kLT / 4) {
        const int i = i0 + (t >> 2);
        double2 s = make_double2(0.0, 0.0);
        if (i < n) {
            for (int b0 = k; b0 < G; b0 += 32) {
                double2 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int b = b0 + 4 * u;
                    v[u] = b < G ? part[int64_t(b) * pld + i] : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    s.x += v[u].x;
                    s.y += v[u].y;
                }
            }
        }
        // lanes 4q .. 4q + 3 of a wave hold coefficient i's four sums: add them in lane order
        const double2 s1 = make_double2(__shfl(s.x, (t & 63) & ~3 | 1, 64), __shfl(s.y, (t & 63) & ~3 | 1, 64));
        const double2 s2 = make_double2(__shfl(s.x, (t & 63) & ~3 | 2, 64), __shfl(s.y, (t & 63) & ~3 | 2, 64));
        const double2 s3 = make_double2(__shfl(s.x, (t & 63) & ~3 | 3, 64), __shfl(s.y, (t & 63) & ~3 | 3, 64));
        if (k == 0 && i < n) coef[i] = make_double2(((s.x + s1.x) + s2.x) + s3.x, ((s.y + s1.y) + s2.y) + s3.y);
    }
    __syncthreads();
}

// w -= sum_{i < n} coef[i] V_i[x], the vectors in groups of 16 whose loads are issued together
__device__ void subtract(const double2* V, int64_t D, int n, int64_t x, const double2* coef, double2& w) {
    for (int i0 = 0; i0 < n; i0 += 16) {
        double2 v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = i0 + q < n ? V[int64_t(i0 + q) * D + x] : make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if (i0 + q < n) {
                const double2 c = coef[i0 + q];
                w.x -= c.x * v[q].x - c.y * v[q].y;
                w.y -= c.x * v[q].y + c.y * v[q].x;
            }
        }
    }
}

// Number of eigenvalues of the tridiagonal (d, e2 = squared off-diagonal) below x: negative
// pivots of LDL^T(T - x I), a pivot smaller in magnitude than pivmin taken as -pivmin.
__device__ int sturm_below(const double* d, const double* e2, int m, double x, double pivmin) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int c = q < 0.0;
#pragma unroll 4
    for (int i = 1; i < m; ++i) {
        q = (d[i] - x) - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
    }
    return c;
}

// Workgroup 0's convergence test on T_m (diagonal al, off-diagonal be), the lowest Ritz value
// being at most hi0 (the previous test's, by interlacing; +inf at the first). theta = the lowest
// eigenvalue by multisection (kLT points per round); then y = (T - theta I)^{-1} applied twice to
// ones by elimination with partial pivoting (one thread), s_last = y[m-1] / |y|. Returns |s_last|
// (the residual estimate is beta_{m-1} |s_last|) and theta in *theta.
__device__ double ritz_last(const double* al, const double* be, int m, double hi0, double* sd, double* se,
                            double* se2, double* lu, int* first, double* theta) {
    const int t = threadIdx.x;
    for (int i = t; i < m; i += kLT) {
        sd[i] = al[i];
        se[i] = i + 1 < m ? be[i] : 0.0;
        se2[i] = se[i] * se[i];
    }
    __syncthreads();
    __shared__ double lo, hi, pivmin, slast;
    if (t == 0) {
        double l = HUGE_VAL, h = -HUGE_VAL, emax = 0.0;
        for (int i = 0; i < m; ++i) {
            const double r = (i > 0 ? fabs(se[i - 1]) : 0.0) + (i + 1 < m ? fabs(se[i]) : 0.0);
            l = fmin(l, sd[i] - r);
            h = fmax(h, sd[i] + r);
            if (i + 1 < m) emax = fmax(emax, se2[i]);
        }
        const double tn = fmax(fabs(l), fabs(h));
        pivmin = DBL_MIN * fmax(1.0, emax);
        const double pad = 2.1 * DBL_EPSILON * tn * m + 4.2 * pivmin;
        lo = l - pad;
        hi = fmin(h, hi0) + pad;
    }
    __syncthreads();
    for (int round = 0; round < 12; ++round) {
        const double l0 = lo, h0 = hi;
        if (!(h0 - l0 > 2.0 * DBL_EPSILON * fmax(fabs(l0), fabs(h0)) + pivmin)) break;
        const double step = (h0 - l0) / (kLT + 1);
        if (t == 0) *first = kLT;
        __syncthreads();
        if (sturm_below(sd, se2, m, l0 + (t + 1) * step, pivmin) >= 1) atomicMin(first, t);
        __syncthreads();
        if (t == 0) {
            const int f = *first;
            lo = f == 0 ? l0 : l0 + f * step;
            hi = f == kLT ? h0 : l0 + (f + 1) * step;
        }
        __syncthreads();
    }
    if (t == 0) {
        const double th = lo + 0.5 * (hi - lo);
        // rows of T - theta I: sub-diagonal se[i-1], diagonal c[i], super-diagonal u[i]; with row
        // swaps the eliminated rows keep at most two super-diagonals (u, u2)
        double* c = lu;
        double* u = lu + m;
        double* u2 = lu + 2 * m;
        double* y = lu + 3 * m;
        const double tiny = DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin;
        for (int i = 0; i < m; ++i) y[i] = 1.0;
        for (int it = 0; it < 2; ++it) {
            for (int i = 0; i < m; ++i) {
                c[i] = sd[i] - th;
                u[i] = se[i];
                u2[i] = 0.0;
            }
            for (int i = 0; i + 1 < m; ++i) {
                const double b = se[i];  // entry (i+1, i)
                if (fabs(b) > fabs(c[i])) {
                    // swap rows i and i+1, then eliminate the old row i below the new pivot
                    const double ci = c[i], ui = u[i];
                    c[i] = b;
                    u[i] = c[i + 1];
                    u2[i] = u[i + 1];
                    const double ty = y[i];
                    y[i] = y[i + 1];
                    y[i + 1] = ty;
                    const double f = ci / b;
                    c[i + 1] = ui - f * u[i];
                    u[i + 1] = -f * u2[i];
                    y[i + 1] -= f * y[i];
                } else {
                    const double piv = c[i] != 0.0 ? c[i] : tiny;
                    c[i] = piv;
                    const double f = b / piv;
                    c[i + 1] -= f * u[i];
                    y[i + 1] -= f * y[i];
                }
            }
            if (c[m - 1] == 0.0) c[m - 1] = tiny;
            for (int i = m - 1; i >= 0; --i) {
                double r = y[i];
                if (i + 1 < m) r -= u[i] * y[i + 1];
                if (i + 2 < m) r -= u2[i] * y[i + 2];
                y[i] = r / c[i];
            }
            double nrm = 0.0;
            for (int i = 0; i < m; ++i) nrm = fmax(nrm, fabs(y[i]));
            for (int i = 0; i < m; ++i) y[i] /= nrm;
        }
        double n2 = 0.0;
        for (int i = 0; i < m; ++i) n2 += y[i] * y[i];
        slast = fabs(y[m - 1]) / sqrt(n2);
        *theta = th;
    }
    __syncthreads();
    return slast;
}

template <unsigned CLS>
__global__ __launch_bounds__(kLT) void lanczos_dev_kernel(DevLzArgs a) {
    __shared__ double2 h1[kDevMaxVec], h2[kDevMaxVec];
    __shared__ double2 red[kLT / 64][16];
    __shared__ double nred[kLT / 64];
    __shared__ double sd[kDevMaxVec], se[kDevMaxVec], se2[kDevMaxVec], lu[4 * kDevMaxVec];
    __shared__ int bad, first;
    __shared__ double theta_prev;  // workgroup 0: the last test's lowest Ritz value
    const int t = threadIdx.x, g = blockIdx.x, G = gridDim.x;
    if (t == 0) theta_prev = HUGE_VAL;  // read after the first grid barrier
    const int64_t x = int64_t(g) * kLT + t;
    const bool xok = x < a.D;
    unsigned gen = 0;
    for (int j = 0; j < a.nmax; ++j) {
        const int n = j + 1;
        double2 w = make_double2(0.0, 0.0);
        if (xok) w = small_entry<CLS>(a.V + int64_t(j) * a.D, a.site, a.bond, a.L, x);
        block_dots(a.V, a.D, n, x, xok, w, a.p1 + int64_t(g) * a.pld, red);
        if (!grid_sync(a, gen, &bad)) return;
        // first pass: h1_i = <v_i|w>, w -= sum_i h1_i v_i
        sum_partials(a.p1, a.pld, G, n, h1);
        if (xok) subtract(a.V, a.D, n, x, h1, w);
        block_dots(a.V, a.D, n, x, xok, w, a.p2 + int64_t(g) * a.pld, red);
        if (!grid_sync(a, gen, &bad)) return;
        // second pass, and the partial squared norm of the result
        sum_partials(a.p2, a.pld, G, n, h2);
        double nn = 0.0;
        if (xok) {
            subtract(a.V, a.D, n, x, h2, w);
            nn = w.x * w.x + w.y * w.y;
        }
        for (int o = 32; o > 0; o >>= 1) nn += __shfl_xor(nn, o, 64);
        if ((t & 63) == 0) nred[t >> 6] = nn;
        __syncthreads();
        if (t == 0) {
            double s = nred[0];
            for (int k = 1; k < kLT / 64; ++k) s += nred[k];
            a.pn[g] = s;
        }
        if (g == 0 && t == 0) a.alpha[j] = h1[j].x + h2[j].x;
        if (!grid_sync(a, gen, &bad)) return;
        // beta_j from every workgroup's partial norm, the same sum on every workgroup: lane l of each
        // wave loads rows l, l + 64, ..., and the wave sum follows a fixed butterfly
        double b2 = 0.0;
        for (int b = t & 63; b < G; b += 64) b2 += a.pn[b];
        for (int o = 32; o > 0; o >>= 1) b2 += __shfl_xor(b2, o, 64);
        const double beta = sqrt(b2);
        double hmax = 0.0;
        for (int i = 0; i < n; ++i) {
            const double2 c = make_double2(h1[i].x + h2[i].x, h1[i].y + h2[i].y);
            hmax = fmax(hmax, sqrt(c.x * c.x + c.y * c.y));
        }
        const bool brk = beta <= 1e-14 * fmax(hmax, 1e-300) || beta == 0.0;
        if (xok && !brk) a.V[int64_t(n) * a.D + x] = make_double2(w.x / beta, w.y / beta);
        if (g == 0) {
            if (t == 0) {
                a.beta[j] = beta;
                a.ctl[2] = n;
            }
            bool done = brk;
            if (!done && (n % kLCheck == 0 || n == a.nmax)) {
                __syncthreads();  // alpha[j] and beta[j] written by thread 0
                double th = 0.0;
                done = beta * ritz_last(a.alpha, a.beta, n, theta_prev, sd, se, se2, lu, &first, &th) <= a.tol;
                if (t == 0) theta_prev = th;
            }
            if (t == 0 && done) a.ctl[1] = n;
        }
        if (!grid_sync(a, gen, &bad)) return;
        if (ld_ctl(a.ctl + 1) != 0) return;
    }
}

template <unsigned CLS>
hipError_t launch_dev(const DevLzArgs& a, int G, hipStream_t s) {
    DevLzArgs args = a;
    void* params[] = {&args};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&lanczos_dev_kernel<CLS>), dim3(G), dim3(kLT),
                                      params, 0, s);
}

template <int I>
hipError_t dispatch_dev(unsigned cls, const DevLzArgs& a, int G, hipStream_t s) {
    if constexpr (I >= kNumVariants) {
        return hipErrorInvalidValue;
    } else {
        if (variant_fits(kVariants[I], cls)) return launch_dev<kVariants[I]>(a, G, s);
        return dispatch_dev<I + 1>(cls, a, G, s);
    }
}

__global__ void clear_ints(int* p, int n) {
    const int i = int(threadIdx.x);
    if (i < n) p[i] = 0;
}

}  // namespace

bool lanczos_device_fits(const ed_model* m, int max_iter) {
    if (m->L > kDevLanczosMaxL || m->lr || m->lv_L > 0 || !m->far.empty()) return false;
    if (max_iter < 1 || max_iter > kDevMaxVec - 1) return false;
    const int64_t D = int64_t(1) << m->L;
    const int64_t G = (D + kLT - 1) / kLT;
    return 2 * G * int64_t(max_iter + 1) * int64_t(sizeof(double2)) <= int64_t(kPartBytes);
}

ed_status lanczos_device(const ed_model* m, const Workspace& w, int max_iter, double tol, int* m_out,
                         int* products, bool* converged, std::vector<double>* alpha, std::vector<double>* beta,
                         hipStream_t s) {
    const int64_t D = w.D;
    const int G = int((D + kLT - 1) / kLT);
    DevLzArgs a;
    a.site = m->d_site;
    a.bond = m->d_bond;
    a.L = m->L;
    a.D = D;
    a.V = w.V;
    a.nmax = max_iter;
    a.pld = max_iter + 1;
    a.p1 = w.part;
    a.p2 = w.part + int64_t(G) * a.pld;
    // device scalars after the ones the step kernels use: pn[G], alpha, beta, barrier and control
    double* sc = reinterpret_cast<double*>(w.scal + kObs);
    static_assert(kScalars - kObs >= 8, "scalar area");
    double* base = reinterpret_cast<double*>(w.scal + 1);  // the h1/h2 area is free on this path
    a.pn = base;
    a.alpha = base + G;
    a.beta = a.alpha + max_iter;
    unsigned* bar = reinterpret_cast<unsigned*>(sc);
    a.bar = bar;
    a.ctl = reinterpret_cast<int*>(sc) + 4;
    a.tol = tol;
    if (size_t(G + 2 * max_iter) * sizeof(double) > size_t(2 * kMaxProj) * sizeof(double2))
        return fail(ED_ERR_UNSUPPORTED, "device Lanczos: too many scalars");
    hipLaunchKernelGGL(clear_ints, dim3(1), dim3(64), 0, s, reinterpret_cast<int*>(sc), 8);
    hipError_t e = dispatch_dev<0>(m->op_class, a, G, s);
    if (e == hipErrorCooperativeLaunchTooLarge) {
        // the workgroups cannot all be resident now: the caller runs the host-driven recurrence
        (void)hipGetLastError();
        *products = 0;
        return ED_ERR_UNSUPPORTED;
    }
    if (e != hipSuccess) return fail(ED_ERR_HIP, std::string("device Lanczos launch: ") + hipGetErrorString(e));
    int ctl[3] = {0, 0, 0};
    ED_HIP_TRY(hipMemcpyAsync(ctl, a.ctl, sizeof(ctl), hipMemcpyDeviceToHost, s));
    ED_HIP_TRY(hipStreamSynchronize(s));
    if (ctl[0] != 0) return fail(ED_ERR_HIP, "device Lanczos: a grid barrier timed out");
    const int done = ctl[2];
    *products = done;
    *converged = ctl[1] != 0;
    *m_out = ctl[1] != 0 ? ctl[1] : done;
    alpha->assign(size_t(*m_out), 0.0);
    beta->assign(size_t(*m_out), 0.0);
    if (*m_out > 0) {
        ED_HIP_TRY(hipMemcpy(alpha->data(), a.alpha, sizeof(double) * size_t(*m_out), hipMemcpyDeviceToHost));
        ED_HIP_TRY(hipMemcpy(beta->data(), a.beta, sizeof(double) * size_t(*m_out), hipMemcpyDeviceToHost));
    }
    return ED_OK;
}

}  // namespace ed
