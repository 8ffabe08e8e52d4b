// Quantum trajectories for the Lindblad equation (Sec. ed:sec:QT). Per trajectory, with
// H_eff = H - (i/2) sum_nu L_nu^dagger L_nu and L_nu = sqrt(rate_nu) J on site nu:
//   1. draw r; evolve the unnormalised state under H_eff until |psi|^2 drops to r;
//   2. draw r_kappa; p_nu = <psi|L_nu^dagger L_nu|psi>, P_nu the normalised cumulative sum;
//   3. apply L_kappa with P_{kappa-1} < r_kappa <= P_kappa, renormalise, go back to 1.
// The evolution uses Krylov steps (the paper notes quantum trajectories work with any of its
// three propagators); H_eff is not Hermitian, so the basis comes from Arnoldi and the projected
// matrix is upper Hessenberg (Sec. ed:sec:Liouville). The step's basis gives psi(t + tau) for every tau in the
// step, so the time at which |psi|^2 reaches r is solved in the small space, without extra H psi.
//
// Batched path: one persistent launch. Each workgroup runs its own list of trajectories, dealt on
// the host by longest processing time first (each trajectory, heaviest first, goes to the
// workgroup with the least work so far; the work of a trajectory is taken proportional to its
// state size plus a fixed per-step overhead), keeps the state and Krylov basis in its own slice of
// the workspace, runs H psi
// tile by tile through LDS, and does every reduction, the small exponential, the root search,
// the Philox draws and the jumps itself, so a trajectory never returns to the host.
// Plain path: the same algorithm one trajectory at a time from the host, on the library's
// stream-level kernels (the per-instance baseline).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "dense.h"
#include "ed_vec.h"
#include "hpsi_device.h"
#include "krylov_core.h"

namespace ed {

ed_status create_model(const ed_model_desc* desc, ed_model** out);
void destroy_model(ed_model* m);

namespace {

constexpr int kTT = 256;       // threads per trajectory workgroup
constexpr int kTMax = 24;      // max Krylov dimension per step (basis holds kTMax + 1 vectors)
constexpr int kMaxL = 20;
constexpr int kMaxHalvings = 10;       // exp(-i tau H_m) e_1: at most 2^10 scaled Taylor sums
constexpr int kMaxEventsPerStep = 256;  // jumps resolved inside one time step before giving up

// ---------------------------------------------------------------------------- Philox4x64-10
// Salmon et al. (SC'11): two 64x64 -> 128 multiplies per round, key bumped by Weyl constants.
__device__ __host__ inline void philox4x64_10(const uint64_t c_in[4], uint64_t k0, uint64_t k1, uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t x0 = c_in[0], x1 = c_in[1], x2 = c_in[2], x3 = c_in[3];
    for (int r = 0; r < 10; ++r) {
#ifdef __HIP_DEVICE_COMPILE__
        const uint64_t hi0 = __umul64hi(M0, x0), hi1 = __umul64hi(M1, x2);
#else
        const uint64_t hi0 = uint64_t((unsigned __int128)M0 * x0 >> 64);
        const uint64_t hi1 = uint64_t((unsigned __int128)M1 * x2 >> 64);
#endif
        const uint64_t lo0 = M0 * x0, lo1 = M1 * x2;
        const uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

// Word n of the stream of key (seed, id): counter block n/4 + 1, word n%4.
__device__ __host__ inline uint64_t philox_word(uint64_t seed, uint64_t id, uint64_t n) {
    const uint64_t c[4] = {n / 4 + 1, 0, 0, 0};
    uint64_t o[4];
    philox4x64_10(c, seed, id, o);
    return o[n % 4];
}

__device__ __host__ inline double to_unit(uint64_t w) { return double((w >> 11) + 1) * 0x1.0p-53; }

// ---------------------------------------------------------------------------- descriptors
struct TrajModel {
    ModelTables tb;
    const double2* psi0;
    double rate[kMaxL];
    int L;
    unsigned cls;
};

struct TrajArgs {
    const TrajModel* models;
    const int* order;        // trajectories, heaviest first: the queue the workgroups take them from
    const int* model_of;
    int n_traj;
    double dt;
    int n_steps;
    int out_stride;
    int n_out;
    uint64_t seed;
    int m_max;
    double tol;
    int max_jumps;
    double2 J[4];
    double jdj_up, jdj_dn;
    int Lmax;
    double* sz_out;
    int* n_jumps;
    double* jump_t;
    int* jump_site;
    int* m_total;
    int* unconverged;    // per trajectory: Krylov steps that stopped at m_max with the error above tol
    double2* scratch;
    int64_t scratch_stride;
    int* counter;     // counter[0]: the queue's next position (zero at launch)
    long long* busy;  // per workgroup: wall-clock ticks from its start to the end of its last trajectory
};

struct Shared {
    double2 H[(kTMax + 1) * (kTMax + 1)];
    double2 u[kTMax + 1], term[kTMax + 1], acc[kTMax + 1], h[kTMax + 1], h2[kTMax + 1], coef[kTMax + 1];
    double cs[kTMax + 1];  // basis vector i of the step is v_i = cs[i] u_i (u_i stored)
    double red[kTT / 64][2 * (kTMax + 1)];
    double pop[kMaxL + 1];
    double scal[8];
};

// ---------------------------------------------------------------------------- WG reductions
// Sum NA per-thread doubles over the workgroup; every thread receives all NA totals in out[].
template <int NA>
__device__ void wg_sum(double (&a)[NA], Shared& sh, double* out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        double v = a[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) sh.red[wv][i] = v;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kTT / 64; ++w) s += sh.red[w][i];
        out[i] = s;
    }
    __syncthreads();
}

// The loops below take 4 elements (or a group of basis vectors) per iteration and issue all of
// their loads before using any, so every wave keeps several loads in flight; a workgroup's state
// has N = 2^L >= 256 = kTT elements, a multiple of kTT.
__device__ double wg_norm2(const double2* x, int64_t N, Shared& sh) {
    double a[1] = {0.0};
    #pragma unroll 1
    for (int64_t i = threadIdx.x; i < N; i += 4 * kTT) {
        double2 y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) y[u] = x[i + u * kTT < N ? i + u * kTT : i];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * kTT < N) a[0] = fma(y[u].x, y[u].x, fma(y[u].y, y[u].y, a[0]));
    }
    double o[1];
    wg_sum<1>(a, sh, o);
    return o[0];
}

__device__ void wg_scale(double2* x, int64_t N, double s) {
    #pragma unroll 1
    for (int64_t i = threadIdx.x; i < N; i += 4 * kTT) {
        double2 y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) y[u] = x[i + u * kTT < N ? i + u * kTT : i];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * kTT < N) x[i + u * kTT] = make_double2(y[u].x * s, y[u].y * s);
    }
    __syncthreads();
}

// out[i] (into sh.h) = <V_i|w>, i < n; vectors taken in groups of 8 to bound register use
__device__ void wg_dots(const double2* V, int64_t ld, int n, const double2* w, int64_t N, Shared& sh) {
    constexpr int G = 8;
    for (int i0 = 0; i0 < n; i0 += G) {
        double a[2 * G];
#pragma unroll
        for (int i = 0; i < 2 * G; ++i) a[i] = 0.0;
        #pragma unroll 1
        for (int64_t x = threadIdx.x; x < N; x += kTT) {
            const double2 y = w[x];
            double2 v[G];
#pragma unroll
            for (int i = 0; i < G; ++i) v[i] = V[(i0 + i < n ? i0 + i : i0) * ld + x];
#pragma unroll
            for (int i = 0; i < G; ++i) {
                if (i0 + i < n) {
                    a[2 * i] = fma(v[i].x, y.x, fma(v[i].y, y.y, a[2 * i]));
                    a[2 * i + 1] = fma(v[i].x, y.y, fma(-v[i].y, y.x, a[2 * i + 1]));
                }
            }
        }
        double o[2 * G];
        wg_sum<2 * G>(a, sh, o);
        if (threadIdx.x < G && i0 + threadIdx.x < n)
            sh.h[i0 + threadIdx.x] = make_double2(o[2 * threadIdx.x], o[2 * threadIdx.x + 1]);
    }
    __syncthreads();
}

// w -= sum_i c_i V_i with c in shared memory
__device__ void wg_sub(const double2* V, int64_t ld, int n, const double2* c, double2* w, int64_t N) {
    constexpr int G = 8;
    #pragma unroll 1
    for (int64_t x = threadIdx.x; x < N; x += kTT) {
        double2 acc = w[x];
        for (int i0 = 0; i0 < n; i0 += G) {
            double2 v[G];
#pragma unroll
            for (int i = 0; i < G; ++i) v[i] = V[(i0 + i < n ? i0 + i : i0) * ld + x];
#pragma unroll
            for (int i = 0; i < G; ++i) {
                if (i0 + i < n) {
                    const double2 ci = c[i0 + i];
                    acc.x -= ci.x * v[i].x - ci.y * v[i].y;
                    acc.y -= ci.x * v[i].y + ci.y * v[i].x;
                }
            }
        }
        w[x] = acc;
    }
    __syncthreads();
}

// out = scale * sum_i c_i V_i
__device__ void wg_combine(const double2* V, int64_t ld, int n, const double2* c, double scale, double2* out,
                           int64_t N) {
    constexpr int G = 8;
    #pragma unroll 1
    for (int64_t x = threadIdx.x; x < N; x += kTT) {
        double2 acc = make_double2(0.0, 0.0);
        for (int i0 = 0; i0 < n; i0 += G) {
            double2 v[G];
#pragma unroll
            for (int i = 0; i < G; ++i) v[i] = V[(i0 + i < n ? i0 + i : i0) * ld + x];
#pragma unroll
            for (int i = 0; i < G; ++i) {
                if (i0 + i < n) {
                    const double2 ci = c[i0 + i];
                    acc.x += ci.x * v[i].x - ci.y * v[i].y;
                    acc.y += ci.x * v[i].y + ci.y * v[i].x;
                }
            }
        }
        out[x] = make_double2(scale * acc.x, scale * acc.y);
    }
    __syncthreads();
}

// Scaled-basis Gram-Schmidt pieces (v_i = cs[i] u_i). sweep B: w -= sum_i coef_i u_i over all n
// vectors and, in the same pass, h2[i] = cs[i] <u_i|w_new> for the first kSubKeep of them (their
// values are still in registers) and |w_new|^2, which it returns; wg_more_dots takes the dots of
// any further vectors, in an extra pass.
constexpr int kSubKeep = 8;
__device__ double wg_sub_dots(const double2* V, int64_t ld, int n, double2* w, int64_t N, Shared& sh) {
    constexpr int G = kSubKeep;
    double a[2 * G + 1];
#pragma unroll
    for (int i = 0; i < 2 * G + 1; ++i) a[i] = 0.0;
    #pragma unroll 1
    for (int64_t x = threadIdx.x; x < N; x += kTT) {
        double2 acc = w[x];
        double2 keep[G];
#pragma unroll
        for (int i = 0; i < G; ++i) keep[i] = V[(i < n ? i : 0) * ld + x];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            if (i < n) {
                const double2 ci = sh.coef[i];
                acc.x -= ci.x * keep[i].x - ci.y * keep[i].y;
                acc.y -= ci.x * keep[i].y + ci.y * keep[i].x;
            }
        }
        for (int i0 = G; i0 < n; i0 += G) {
            double2 v[G];
#pragma unroll
            for (int i = 0; i < G; ++i) v[i] = V[(i0 + i < n ? i0 + i : i0) * ld + x];
#pragma unroll
            for (int i = 0; i < G; ++i) {
                if (i0 + i < n) {
                    const double2 ci = sh.coef[i0 + i];
                    acc.x -= ci.x * v[i].x - ci.y * v[i].y;
                    acc.y -= ci.x * v[i].y + ci.y * v[i].x;
                }
            }
        }
        w[x] = acc;
#pragma unroll
        for (int i = 0; i < G; ++i) {
            if (i < n) {
                a[2 * i] = fma(keep[i].x, acc.x, fma(keep[i].y, acc.y, a[2 * i]));
                a[2 * i + 1] = fma(keep[i].x, acc.y, fma(-keep[i].y, acc.x, a[2 * i + 1]));
            }
        }
        a[2 * G] = fma(acc.x, acc.x, fma(acc.y, acc.y, a[2 * G]));
    }
    double o[2 * G + 1];
    wg_sum<2 * G + 1>(a, sh, o);
    if (threadIdx.x < G && threadIdx.x < n)
        sh.h2[threadIdx.x] = make_double2(sh.cs[threadIdx.x] * o[2 * threadIdx.x], sh.cs[threadIdx.x] * o[2 * threadIdx.x + 1]);
    __syncthreads();
    return o[2 * G];
}

// h2[i] = cs[i] <u_i|w> for kSubKeep <= i < n (the second pass's dots beyond those of sweep B)
__device__ void wg_more_dots(const double2* V, int64_t ld, int n, const double2* w, int64_t N, Shared& sh) {
    constexpr int G = kSubKeep;
    if (n <= G) return;
    wg_dots(V + G * ld, ld, n - G, w, N, sh);
    if (threadIdx.x < n - G) {
        const double c = sh.cs[G + threadIdx.x];
        sh.h2[G + threadIdx.x] = make_double2(c * sh.h[threadIdx.x].x, c * sh.h[threadIdx.x].y);
    }
    __syncthreads();
}

// sweep C: w -= sum_i coef_i u_i; returns |w_new|^2
__device__ double wg_sub_norm(const double2* V, int64_t ld, int n, double2* w, int64_t N, Shared& sh) {
    constexpr int G = 8;
    double a[1] = {0.0};
    #pragma unroll 1
    for (int64_t x = threadIdx.x; x < N; x += kTT) {
        double2 acc = w[x];
        for (int i0 = 0; i0 < n; i0 += G) {
            double2 v[G];
#pragma unroll
            for (int i = 0; i < G; ++i) v[i] = V[(i0 + i < n ? i0 + i : i0) * ld + x];
#pragma unroll
            for (int i = 0; i < G; ++i) {
                if (i0 + i < n) {
                    const double2 ci = sh.coef[i0 + i];
                    acc.x -= ci.x * v[i].x - ci.y * v[i].y;
                    acc.y -= ci.x * v[i].y + ci.y * v[i].x;
                }
            }
        }
        w[x] = acc;
        a[0] = fma(acc.x, acc.x, fma(acc.y, acc.y, a[0]));
    }
    double o[1];
    wg_sum<1>(a, sh, o);
    return o[0];
}

// Per-site populations: pop[p] = sum_{bit p of x = 0} |psi_x|^2 (p = bit), pop[L] = total.
__device__ void wg_pops(const double2* psi, int L, Shared& sh) {
    double a[kMaxL + 1];
#pragma unroll
    for (int i = 0; i <= kMaxL; ++i) a[i] = 0.0;
    const int64_t N = int64_t(1) << L;
    #pragma unroll 1
    for (int64_t x = threadIdx.x; x < N; x += kTT) {
        const double2 y = psi[x];
        const double q = fma(y.x, y.x, y.y * y.y);
        a[kMaxL] += q;
#pragma unroll
        for (int p = 0; p < kMaxL; ++p)
            if (p < L && !((x >> p) & 1)) a[p] += q;
    }
    double o[kMaxL + 1];
    wg_sum<kMaxL + 1>(a, sh, o);
    if (threadIdx.x == 0) {
        for (int p = 0; p < L; ++p) sh.pop[p] = o[p];
        sh.pop[kMaxL] = o[kMaxL];
    }
    __syncthreads();
}

// dst = H_eff src for the whole small state of this workgroup; partner amplitudes are read from
// global memory (the state of one trajectory is at most 1 MiB).
template <unsigned CLS>
__device__ void wg_apply(const TrajModel& md, const double2* src, double scale, double2* dst, Shared& sh) {
    const int L = md.L;
    const int64_t N = int64_t(1) << L;
    #pragma unroll 1
    for (int64_t x = threadIdx.x; x < N; x += kTT) {
        const double2 y = small_entry<CLS>(src, md.tb.site, md.tb.bond, L, x);
        dst[x] = make_double2(scale * y.x, scale * y.y);
    }
    __syncthreads();
}

// u = exp(-i tau H_m) e_1 for the m x m Hessenberg in sh.H (leading dimension kTMax + 1), by
// scaling the matrix to norm <= 1/2 and summing the Taylor series of the vector 2^s times.
__device__ void wg_expv(int m, double tau, Shared& sh) {
    constexpr int LD = kTMax + 1;
    double nrm = 0.0;
    for (int j = 0; j < m; ++j) {
        double cs = 0.0;
        for (int i = 0; i < m; ++i) {
            const double2 h = sh.H[i * LD + j];
            cs += sqrt(h.x * h.x + h.y * h.y);
        }
        nrm = fmax(nrm, cs);
    }
    nrm *= fabs(tau);
    int sq = 0;
    while (nrm > 0.5 && sq < kMaxHalvings) {
        nrm *= 0.5;
        ++sq;
    }
    const double sc = tau * ldexp(1.0, -sq);  // A = -i sc H
    const int t = threadIdx.x;
    if (t < m) sh.u[t] = make_double2(t == 0 ? 1.0 : 0.0, 0.0);
    __syncthreads();
    const long reps = 1L << sq;
    for (long rep = 0; rep < reps; ++rep) {
        if (t < m) {
            sh.term[t] = sh.u[t];
            sh.acc[t] = sh.u[t];
        }
        __syncthreads();
        for (int k = 1; k <= 40; ++k) {
            double2 nt = make_double2(0.0, 0.0);
            if (t < m) {
                for (int j = 0; j < m; ++j) {
                    const double2 h = sh.H[t * LD + j], v = sh.term[j];
                    nt.x += h.x * v.x - h.y * v.y;
                    nt.y += h.x * v.y + h.y * v.x;
                }
                // multiply by -i sc / k
                const double f = sc / k;
                nt = make_double2(f * nt.y, -f * nt.x);
            }
            __syncthreads();
            if (t < m) {
                sh.term[t] = nt;
                sh.acc[t].x += nt.x;
                sh.acc[t].y += nt.y;
            }
            __syncthreads();
            double tn = 0.0, an = 0.0;
            for (int j = 0; j < m; ++j) {
                tn = fmax(tn, fabs(sh.term[j].x) + fabs(sh.term[j].y));
                an = fmax(an, fabs(sh.acc[j].x) + fabs(sh.acc[j].y));
            }
            __syncthreads();
            if (tn <= 1e-18 * an) break;
        }
        if (t < m) sh.u[t] = sh.acc[t];
        __syncthreads();
    }
}

__device__ double unorm2(int m, Shared& sh) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += sh.u[i].x * sh.u[i].x + sh.u[i].y * sh.u[i].y;
    return s;
}

template <unsigned CLS>
__device__ void run_trajectory(const TrajArgs& a, int tr, double2* base, Shared& sh) {
    constexpr int LD = kTMax + 1;
    const TrajModel& md = a.models[a.model_of[tr]];
    const int L = md.L;
    const int64_t N = int64_t(1) << L;
    const int64_t ldv = int64_t(1) << a.Lmax;
    // the step's basis u_0 .. u_m sits at base + i * ldv, and u_0 is the state itself
    double2* psi = base;
    double2* V = base;
    const int t = threadIdx.x;
    uint64_t ndraw = 0;
    auto draw = [&]() -> double {
        const double u = to_unit(philox_word(a.seed, uint64_t(tr), ndraw));
        ++ndraw;
        return u;
    };
    for (int64_t x = t; x < N; x += kTT) psi[x] = md.psi0[x];
    __syncthreads();
    {
        const double n2 = wg_norm2(psi, N, sh);
        wg_scale(psi, N, 1.0 / sqrt(n2));
    }
    double r = draw();
    int njump = 0, mtot = 0, nunconv = 0;
    double* szo = a.sz_out + int64_t(tr) * a.n_out * a.Lmax;
    auto record = [&](int slot) {
        wg_pops(psi, L, sh);
        const double tot = sh.pop[kMaxL];
        if (t < L) {
            const int p = L - 1 - t;  // site k = t+1 sits at bit L-1-t
            const double up = sh.pop[p];
            szo[int64_t(slot) * a.Lmax + t] = (2.0 * up - tot) / tot;
        }
        __syncthreads();
    };
    record(0);
    bool failed = false;
    for (int step = 0; step < a.n_steps && !failed; ++step) {
        double tau_left = a.dt;
        for (int ev = 0; tau_left > 0.0; ++ev) {
            // Krylov basis of the current state
            const double n2 = wg_norm2(psi, N, sh);
            const double nrm = sqrt(n2);
            if (!(n2 > 0.0) || !isfinite(n2) || ev >= kMaxEventsPerStep) {
                failed = true;  // uniform: every thread sees the same n2 and ev
                break;
            }
            // v_0 = psi / |psi|: u_0 is psi itself, scaled by cs[0]
            if (t == 0) sh.cs[0] = 1.0 / nrm;
            if (t < LD * LD) {
                for (int e = t; e < LD * LD; e += kTT) sh.H[e] = make_double2(0.0, 0.0);
            }
            __syncthreads();
            int m = 0;
            double beta = 0.0;
            bool unconv = false;
            for (int j = 0; j < a.m_max; ++j) {
                double2* Vj = V + j * ldv;
                double2* Wn = V + (j + 1) * ldv;
                // w = H v_j = cs[j] H u_j, then classical Gram-Schmidt: dots, subtraction (with the
                // second pass's dots and the new norm), and the second subtraction only when the first
                // removed more than half of the squared norm (the DGKS test, eta = 1/sqrt(2))
                wg_apply<CLS>(md, Vj, sh.cs[j], Wn, sh);
                wg_dots(V, ldv, j + 1, Wn, N, sh);  // sh.h = <u_i|w>
                if (t <= j) {
                    const double c = sh.cs[t];
                    const double2 g = make_double2(c * sh.h[t].x, c * sh.h[t].y);  // <v_i|w>
                    sh.H[t * LD + j] = g;
                    sh.coef[t] = make_double2(c * g.x, c * g.y);  // w -= <v_i|w> v_i = (c_i <v_i|w>) u_i
                }
                __syncthreads();
                const double nw2 = wg_sub_dots(V, ldv, j + 1, Wn, N, sh);  // sh.h2 = <v_i|w'>, |w'|^2
                // |w|^2 = |w'|^2 + sum_i |<v_i|w>|^2: the same sum on every thread, in the same order
                double removed = 0.0;
                for (int i = 0; i <= j; ++i)
                    removed += sh.H[i * LD + j].x * sh.H[i * LD + j].x + sh.H[i * LD + j].y * sh.H[i * LD + j].y;
                double b2 = nw2;
                if (!(nw2 >= removed)) {
                    wg_more_dots(V, ldv, j + 1, Wn, N, sh);
                    if (t <= j) {
                        const double c = sh.cs[t];
                        sh.H[t * LD + j].x += sh.h2[t].x;
                        sh.H[t * LD + j].y += sh.h2[t].y;
                        sh.coef[t] = make_double2(c * sh.h2[t].x, c * sh.h2[t].y);
                    }
                    __syncthreads();
                    b2 = wg_sub_norm(V, ldv, j + 1, Wn, N, sh);
                }
                beta = sqrt(b2);
                m = j + 1;
                double hs = 0.0;
                for (int i = 0; i <= j; ++i) hs = fmax(hs, sqrt(sh.H[i * LD + j].x * sh.H[i * LD + j].x + sh.H[i * LD + j].y * sh.H[i * LD + j].y));
                const bool brk = beta <= 1e-14 * fmax(hs, 1e-300) || beta == 0.0;
                wg_expv(m, tau_left, sh);
                const double err = brk ? 0.0 : nrm * beta * sqrt(sh.u[m - 1].x * sh.u[m - 1].x + sh.u[m - 1].y * sh.u[m - 1].y);
                if (brk || err <= a.tol || m >= a.m_max) {
                    unconv = !brk && err > a.tol;
                    break;
                }
                // u_{j+1} = w'' unnormalised, v_{j+1} = w'' / beta
                if (t == 0) {
                    sh.H[(j + 1) * LD + j] = make_double2(beta, 0.0);
                    sh.cs[j + 1] = 1.0 / beta;
                }
                __syncthreads();
            }
            mtot += m;
            nunconv += unconv ? 1 : 0;
            // sh.u = exp(-i tau_left H_m) e_1
            const double lr = log(r);
            const double f_end = log(n2 * unorm2(m, sh)) - lr;
            // psi(tau) = nrm sum_i u_i(tau) v_i = sum_i (nrm cs[i] u_i(tau)) u_i, written over u_0 = psi
            // (each thread reads its element of every u_i before writing it)
            if (f_end > 0.0) {
                if (t < m) sh.acc[t] = make_double2(nrm * sh.cs[t] * sh.u[t].x, nrm * sh.cs[t] * sh.u[t].y);
                __syncthreads();
                wg_combine(V, ldv, m, sh.acc, 1.0, psi, N);
                tau_left = 0.0;
                break;
            }
            // crossing inside (0, tau_left]: f(tau) = log(|psi(tau)|^2) - log r is decreasing
            double lo = 0.0, hi = tau_left;
            double flo = log(n2) - lr, fhi = f_end;
            double tau = hi;
            if (flo <= 0.0) {
                tau = 0.0;
            } else {
                int side = 0;
                for (int it = 0; it < 200; ++it) {
                    double c = hi - fhi * (hi - lo) / (fhi - flo);
                    if (!(c > lo && c < hi)) c = 0.5 * (lo + hi);
                    wg_expv(m, c, sh);
                    const double fc = log(n2 * unorm2(m, sh)) - lr;
                    if (fc > 0.0) {
                        lo = c;
                        flo = fc;
                        if (side == -1) fhi *= 0.5;
                        side = -1;
                    } else {
                        hi = c;
                        fhi = fc;
                        if (side == 1) flo *= 0.5;
                        side = 1;
                    }
                    tau = hi;
                    if (fc == 0.0 || hi - lo <= 1e-15 * a.dt) {
                        tau = (fc == 0.0) ? c : hi;
                        break;
                    }
                }
            }
            wg_expv(m, tau, sh);
            if (t < m) sh.acc[t] = make_double2(nrm * sh.cs[t] * sh.u[t].x, nrm * sh.cs[t] * sh.u[t].y);
            __syncthreads();
            wg_combine(V, ldv, m, sh.acc, 1.0, psi, N);
            const double t_abs = step * a.dt + (a.dt - tau_left) + tau;
            // jump probabilities p_nu = rate_nu <psi| J^dag J |psi>_nu (J^dag J diagonal)
            wg_pops(psi, L, sh);
            const double tot = sh.pop[kMaxL];
            const double rk = draw();
            int kappa = L - 1;
            {
                double ptot = 0.0;
                for (int nu = 0; nu < L; ++nu) {
                    const double up = sh.pop[L - 1 - nu];
                    ptot += md.rate[nu] * (a.jdj_up * up + a.jdj_dn * (tot - up));
                }
                double cum = 0.0;
                for (int nu = 0; nu < L; ++nu) {
                    const double up = sh.pop[L - 1 - nu];
                    cum += md.rate[nu] * (a.jdj_up * up + a.jdj_dn * (tot - up));
                    if (rk <= cum / ptot) {
                        kappa = nu;
                        break;
                    }
                }
            }
            // psi <- J on site kappa (bit L-1-kappa), then renormalise
            {
                const int p = L - 1 - kappa;
                const int64_t half = N >> 1;
                for (int64_t q = t; q < half; q += kTT) {
                    const int64_t lowm = (int64_t(1) << p) - 1;
                    const int64_t x0 = ((q & ~lowm) << 1) | (q & lowm);
                    const int64_t x1 = x0 | (int64_t(1) << p);
                    const double2 a0 = psi[x0], a1 = psi[x1];
                    const double2 n0 = make_double2(a.J[0].x * a0.x - a.J[0].y * a0.y + a.J[1].x * a1.x - a.J[1].y * a1.y,
                                                    a.J[0].x * a0.y + a.J[0].y * a0.x + a.J[1].x * a1.y + a.J[1].y * a1.x);
                    const double2 n1 = make_double2(a.J[2].x * a0.x - a.J[2].y * a0.y + a.J[3].x * a1.x - a.J[3].y * a1.y,
                                                    a.J[2].x * a0.y + a.J[2].y * a0.x + a.J[3].x * a1.y + a.J[3].y * a1.x);
                    psi[x0] = n0;
                    psi[x1] = n1;
                }
                __syncthreads();
                const double jn2 = wg_norm2(psi, N, sh);
                wg_scale(psi, N, 1.0 / sqrt(jn2));
            }
            if (t == 0 && njump < a.max_jumps) {
                a.jump_t[int64_t(tr) * a.max_jumps + njump] = t_abs;
                a.jump_site[int64_t(tr) * a.max_jumps + njump] = kappa;
            }
            ++njump;
            r = draw();
            tau_left -= tau;
            if (tau_left <= 1e-15 * a.dt) tau_left = 0.0;
        }
        if ((step + 1) % a.out_stride == 0) record((step + 1) / a.out_stride);
    }
    if (t == 0) {
        a.n_jumps[tr] = failed ? -1 : njump;
        a.m_total[tr] = mtot;
        a.unconverged[tr] = nunconv;
    }
    __syncthreads();
}

// Persistent launch: the workgroups take the trajectories of order[] (heaviest first) one at a
// time from a queue (an atomic counter); every loop below is bounded.
template <unsigned CLS>
__global__ __launch_bounds__(kTT) __attribute__((amdgpu_waves_per_eu(2))) void traj_kernel(TrajArgs a) {
    __shared__ Shared sh;
    double2* base = a.scratch + int64_t(blockIdx.x) * a.scratch_stride;
    __shared__ int qnext;
    const unsigned long long t0 = wall_clock64();
    // each workgroup takes the next trajectory of the queue until it is empty (no workgroup waits
    // for another; the results do not depend on which workgroup runs a trajectory)
    for (;;) {
        if (threadIdx.x == 0) qnext = atomicAdd(a.counter, 1);
        __syncthreads();
        const int q = qnext;
        __syncthreads();
        if (q >= a.n_traj) break;
        run_trajectory<CLS>(a, a.order[q], base, sh);
    }
    if (threadIdx.x == 0) a.busy[blockIdx.x] = static_cast<long long>(wall_clock64() - t0);
}

__global__ void zero_ints(int* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void zero_doubles(double* p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

template <int I>
hipError_t launch_traj(unsigned cls, dim3 grid, size_t shm, hipStream_t s, const TrajArgs& a) {
    if constexpr (I >= kNumVariants) {
        return hipErrorInvalidValue;
    } else {
        if (variant_fits(kVariants[I], cls)) {
            hipLaunchKernelGGL((traj_kernel<kVariants[I]>), grid, dim3(kTT), 0, s, a);
            return hipGetLastError();
        }
        return launch_traj<I + 1>(cls, grid, shm, s, a);
    }
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// ----------------------------------------------------------------------------- shared setup
struct TrajSetup {
    std::vector<std::shared_ptr<ed_model>> heff;  // from the cache below
    int Lmax = 0;
    int n_out = 0;
    unsigned cls = 0;
    double jdj_up = 0.0, jdj_dn = 0.0;
};

// Effective Hamiltonians are kept between calls, keyed by their full description and the device:
// a call with descriptions seen before allocates nothing, a new one builds (and allocates) once.
// At most kHeffCacheMax are kept (the oldest is dropped, and freed once no call holds it). The
// cache lives until the process ends and is never destroyed, so no device memory is freed after
// the runtime has shut down.
constexpr size_t kHeffCacheMax = 64;
struct HeffCache {
    std::mutex mu;
    std::deque<std::pair<std::string, std::shared_ptr<ed_model>>> entries;  // oldest first
};
static HeffCache& heff_cache() {
    static HeffCache* c = new HeffCache;
    return *c;
}

static std::string heff_key(const ed_model_desc& md, int dev) {
    std::string k;
    auto put = [&](const void* p, size_t n) { k.append(static_cast<const char*>(p), n); };
    put(&dev, sizeof(dev));
    put(&md.L, sizeof(md.L));
    put(&md.d, sizeof(md.d));
    put(&md.n_site, sizeof(md.n_site));
    put(&md.n_bond, sizeof(md.n_bond));
    put(md.site_op, sizeof(ed_c64) * 4 * size_t(md.n_site));
    put(md.site_coef, sizeof(double) * size_t(md.n_site) * md.L);
    put(md.bond_op, sizeof(ed_c64) * 16 * size_t(md.n_bond));
    put(md.bond_coef, sizeof(double) * size_t(md.n_bond) * (md.L - 1));
    return k;  // (no long-range rules: H_eff descriptions never carry any)
}

static ed_status heff_model(const ed_model_desc& md, std::shared_ptr<ed_model>* out) {
    int dev = 0;
    ED_HIP_TRY(hipGetDevice(&dev));
    const std::string key = heff_key(md, dev);
    HeffCache& c = heff_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    for (const auto& e : c.entries)
        if (e.first == key) {
            *out = e.second;
            return ED_OK;
        }
    ed_model* h = nullptr;
    ED_TRY(create_model(&md, &h));
    std::shared_ptr<ed_model> sp(h, destroy_model);
    c.entries.emplace_back(key, sp);
    if (c.entries.size() > kHeffCacheMax) c.entries.pop_front();
    *out = sp;
    return ED_OK;
}

static double heff_bound(const ed_model* m);

static ed_status validate_traj(const ed_traj_desc* d, const ed_traj_params* p) {
    if (!d || !p) return fail(ED_ERR_ARG, "null argument");
    if (d->n_models < 1 || !d->models || !d->jump_op || !d->rates || !d->psi0 || !d->model_of_traj)
        return fail(ED_ERR_ARG, "incomplete trajectory description");
    if (d->n_traj < 0) return fail(ED_ERR_ARG, "n_traj must be >= 0");
    if (!(d->dt > 0.0) || d->n_steps < 0 || d->out_stride < 1) return fail(ED_ERR_ARG, "bad time grid");
    if (p->m_max < 1 || p->m_max > kTMax) return fail(ED_ERR_ARG, "m_max must be in [1, 24]");
    if (!(p->tol > 0.0)) return fail(ED_ERR_ARG, "tol must be > 0");
    if (p->max_jumps < 0) return fail(ED_ERR_ARG, "max_jumps must be >= 0");
    for (int i = 0; i < d->n_models; ++i) {
        if (!d->models[i] || !d->rates[i] || !d->psi0[i]) return fail(ED_ERR_ARG, "null model entry");
        if (d->models[i]->L > 16) return fail(ED_ERR_UNSUPPORTED, "trajectory chains are limited to L <= 16");
        if (d->models[i]->lr) return fail(ED_ERR_UNSUPPORTED, "trajectories do not take long-range (InfiniteFunc) terms");
        if (d->models[i]->lv_L > 0) return fail(ED_ERR_UNSUPPORTED, "trajectories take Hamiltonians, not Liouvillians");
    }
    for (int t = 0; t < d->n_traj; ++t)
        if (d->model_of_traj[t] < 0 || d->model_of_traj[t] >= d->n_models) return fail(ED_ERR_ARG, "model_of_traj out of range");
    // J^dag J must be diagonal (true for lowering, raising, number and dephasing operators)
    const ed_c64* J = d->jump_op;
    const double o_re = J[0].re * J[1].re + J[0].im * J[1].im + J[2].re * J[3].re + J[2].im * J[3].im;
    const double o_im = J[0].re * J[1].im - J[0].im * J[1].re + J[2].re * J[3].im - J[2].im * J[3].re;
    if (std::fabs(o_re) > 0.0 || std::fabs(o_im) > 0.0)
        return fail(ED_ERR_UNSUPPORTED, "jump operators with off-diagonal J^dagger J are not supported");
    return ED_OK;
}

// H_eff = H - (i/2) sum_k rate_k J^dag J on site k, built as a copy of each model's terms plus one
// site rule with the operator -(i/2) J^dag J and coefficients rate_k.
static ed_status build_setup(const ed_traj_desc* d, TrajSetup* st) {
    const ed_c64* J = d->jump_op;
    st->jdj_up = J[0].re * J[0].re + J[0].im * J[0].im + J[2].re * J[2].re + J[2].im * J[2].im;
    st->jdj_dn = J[1].re * J[1].re + J[1].im * J[1].im + J[3].re * J[3].re + J[3].im * J[3].im;
    st->n_out = d->n_steps / d->out_stride + 1;
    for (int i = 0; i < d->n_models; ++i) {
        const ed_model* m = d->models[i];
        const int L = m->L;
        st->Lmax = std::max(st->Lmax, L);
        // site ops: the folded per-site operators of H (one rule per site) + the decay rule
        std::vector<ed_c64> sop(4 * (L + 1));
        std::vector<double> scoef(size_t(L + 1) * L, 0.0);
        for (int k = 1; k <= L; ++k) {
            const int p = L - k;
            for (int e = 0; e < 4; ++e) sop[4 * (k - 1) + e] = ed_c64{m->site[4 * p + e].x, m->site[4 * p + e].y};
            scoef[size_t(k - 1) * L + (k - 1)] = 1.0;
        }
        sop[4 * L + 0] = ed_c64{0.0, -0.5 * st->jdj_up};
        sop[4 * L + 1] = ed_c64{0.0, 0.0};
        sop[4 * L + 2] = ed_c64{0.0, 0.0};
        sop[4 * L + 3] = ed_c64{0.0, -0.5 * st->jdj_dn};
        for (int k = 0; k < L; ++k) scoef[size_t(L) * L + k] = d->rates[i][k];
        std::vector<ed_c64> bop(16 * (L - 1));
        std::vector<double> bcoef(size_t(L - 1) * (L - 1), 0.0);
        for (int k = 1; k <= L - 1; ++k) {
            const int p = L - k - 1;
            for (int e = 0; e < 16; ++e) bop[16 * (k - 1) + e] = ed_c64{m->bond[16 * p + e].x, m->bond[16 * p + e].y};
            bcoef[size_t(k - 1) * (L - 1) + (k - 1)] = 1.0;
        }
        ed_model_desc md{L, 2, L + 1, sop.data(), scoef.data(), L - 1, bop.data(), bcoef.data()};
        std::shared_ptr<ed_model> h;
        ED_TRY(heff_model(md, &h));
        st->cls |= h->op_class & kWork;
        st->heff.push_back(std::move(h));
    }
    for (const auto& h : st->heff)
        if (d->dt * heff_bound(h.get()) > 50.0)
            return fail(ED_ERR_UNSUPPORTED, "dt * |H_eff| > 50: use a smaller trajectory time step");
    // real flags: only if every model has them
    unsigned real = kOffReal | kDiagReal;
    for (const auto& h : st->heff) real &= h->op_class;
    st->cls |= real;
    return ED_OK;
}

// Upper bound of |H_eff| (sum over terms of the largest absolute row sum of each local operator):
// dt times it must stay moderate so that the scaled Taylor series of each step is short.
static double heff_bound(const ed_model* m) {
    double b = 0.0;
    for (int p = 0; p < m->L; ++p) {
        double r = 0.0;
        for (int row = 0; row < 2; ++row) {
            double rs = 0.0;
            for (int c = 0; c < 2; ++c) rs += std::hypot(m->site[4 * p + 2 * row + c].x, m->site[4 * p + 2 * row + c].y);
            r = std::max(r, rs);
        }
        b += r;
    }
    for (int p = 0; p + 1 < m->L; ++p) {
        double r = 0.0;
        for (int row = 0; row < 4; ++row) {
            double rs = 0.0;
            for (int c = 0; c < 4; ++c) rs += std::hypot(m->bond[16 * p + 4 * row + c].x, m->bond[16 * p + 4 * row + c].y);
            r = std::max(r, rs);
        }
        b += r;
    }
    return b;
}

// Workgroups of the persistent launch: as many as can be resident at once for the kernel variant
// (the deal is static, so a workgroup that had to wait for a free slot would finish late), at
// most one per trajectory, and at most what a 32 GiB scratch budget holds (each workgroup keeps a
// state and its Krylov basis: (m_max + 2) 2^Lmax amplitudes). variant < 0: the largest count over
// the variants (used to size the workspace).
template <int I>
static int resident_per_cu(int variant) {
    if constexpr (I >= kNumVariants) {
        return 1;
    } else {
        if (I == variant) {
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, traj_kernel<kVariants[I]>, kTT, 0) != hipSuccess)
                nb = 1;
            return std::max(nb, 1);
        }
        return resident_per_cu<I + 1>(variant);
    }
}

static int persistent_blocks(int n_traj, int Lmax, int m_max, int variant) {
    int dev = 0, cu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t pr;
        if (hipGetDeviceProperties(&pr, dev) == hipSuccess) cu = pr.multiProcessorCount;
    }
    int per_cu = 1;
    if (variant >= 0) {
        per_cu = resident_per_cu<0>(variant);
    } else {
        for (int v = 0; v < kNumVariants; ++v) per_cu = std::max(per_cu, resident_per_cu<0>(v));
    }
    const double per_bytes = double(m_max + 2) * double(int64_t(1) << Lmax) * sizeof(double2);
    const int64_t by_mem = std::max<int64_t>(1, int64_t((double(int64_t(32) << 30)) / per_bytes));
    return int(std::max<int64_t>(1, std::min<int64_t>({int64_t(n_traj), int64_t(per_cu) * cu, by_mem})));
}

// Executable graph of the batched launch, one per (device, stream); kept until the process ends
// (a stream's graph is reused by the next call on that stream).
static std::mutex g_traj_graph_mu;
static std::map<std::pair<int, hipStream_t>, hipGraphExec_t> g_traj_graph;

// The queue of the batched launch: trajectories by decreasing cost, a trajectory's cost being
// 2^L + kStepOverhead amplitude-equivalents per step (its products and sweeps stream the state; a
// step also has a fixed cost of reductions and barriers). Workgroups take them in this order as
// they finish (longest processing time first, list scheduling), so the heavy ones start early
// and the light ones fill the end.
static void queue_order(const ed_traj_desc* d, std::vector<int>* ord) {
    constexpr double kStepOverhead = 2048.0;
    const int nt = d->n_traj;
    ord->resize(nt);
    for (int i = 0; i < nt; ++i) (*ord)[i] = i;
    auto cost = [&](int t) { return double(int64_t(1) << d->models[d->model_of_traj[t]]->L) + kStepOverhead; };
    std::stable_sort(ord->begin(), ord->end(), [&](int x, int y) { return cost(x) > cost(y); });
}

static size_t traj_bytes(const ed_traj_desc* d, const ed_traj_params* p, int Lmax, int n_out, int G) {
    const size_t per = size_t(p->m_max + 2) << Lmax;
    return al256(size_t(G) * per * sizeof(double2)) + al256(size_t(d->n_models) * sizeof(TrajModel)) +
           3 * al256(size_t(d->n_traj) * sizeof(int)) +
           al256(size_t(d->n_traj) * n_out * Lmax * sizeof(double)) +
           al256(size_t(d->n_traj) * std::max(p->max_jumps, 1) * (sizeof(double) + sizeof(int))) + al256(sizeof(int) * 4) +
           2 * al256(size_t(d->n_traj) * sizeof(int)) + al256(size_t(G) * sizeof(long long));
}

}  // namespace ed

using namespace ed;

extern "C" ed_status ed_trajectories_workspace(const ed_traj_desc* d, const ed_traj_params* p, size_t* bytes) {
    if (!bytes) return fail(ED_ERR_ARG, "bytes is null");
    ED_TRY(validate_traj(d, p));
    int Lmax = 0;
    for (int i = 0; i < d->n_models; ++i) Lmax = std::max(Lmax, d->models[i]->L);
    const int n_out = d->n_steps / d->out_stride + 1;
    *bytes = traj_bytes(d, p, Lmax, n_out, persistent_blocks(std::max(d->n_traj, 1), Lmax, p->m_max, -1));
    return ED_OK;
}

extern "C" ed_status ed_trajectories_batch(const ed_traj_desc* d, const ed_traj_params* p, const ed_traj_out* out,
                                           ed_traj_info* info, void* ws, size_t ws_bytes, void* stream) {
    ED_TRY(validate_traj(d, p));
    if (!out || !out->sz) return fail(ED_ERR_ARG, "output sz is null");
    size_t need = 0;
    ED_TRY(ed_trajectories_workspace(d, p, &need));
    if (!ws) return fail(ED_ERR_ARG, "workspace is null");
    if (ws_bytes < need) return fail(ED_ERR_WORKSPACE, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    TrajSetup st;
    ED_TRY(build_setup(d, &st));
    const int G = persistent_blocks(std::max(d->n_traj, 1), st.Lmax, p->m_max, pick_variant(st.cls));
    const int Lmax = st.Lmax, n_out = st.n_out, nt = d->n_traj;
    // carve
    char* c = static_cast<char*>(ws);
    auto take = [&](size_t bytes) {
        char* r = c;
        c += al256(bytes);
        return r;
    };
    const size_t per = size_t(p->m_max + 2) << Lmax;
    double2* scratch = reinterpret_cast<double2*>(take(size_t(G) * per * sizeof(double2)));
    TrajModel* dmod = reinterpret_cast<TrajModel*>(take(size_t(d->n_models) * sizeof(TrajModel)));
    int* order = reinterpret_cast<int*>(take(size_t(nt) * sizeof(int)));
    int* model_of = reinterpret_cast<int*>(take(size_t(nt) * sizeof(int)));
    int* njumps = reinterpret_cast<int*>(take(size_t(nt) * sizeof(int)));
    double* sz = reinterpret_cast<double*>(take(size_t(nt) * n_out * Lmax * sizeof(double)));
    const int mj = std::max(p->max_jumps, 1);
    char* jbuf = take(size_t(nt) * mj * (sizeof(double) + sizeof(int)));
    double* jt = reinterpret_cast<double*>(jbuf);
    int* js = reinterpret_cast<int*>(jbuf + size_t(nt) * mj * sizeof(double));
    int* counter = reinterpret_cast<int*>(take(sizeof(int) * 4));
    int* mtot = reinterpret_cast<int*>(take(size_t(nt) * sizeof(int)));
    int* unconv = reinterpret_cast<int*>(take(size_t(nt) * sizeof(int)));
    long long* busy = reinterpret_cast<long long*>(take(size_t(G) * sizeof(long long)));
    // host-side descriptors
    std::vector<TrajModel> hm(d->n_models);
    for (int i = 0; i < d->n_models; ++i) {
        std::memset(&hm[i], 0, sizeof(TrajModel));
        hm[i].tb = tables_of(st.heff[i].get());
        hm[i].psi0 = reinterpret_cast<const double2*>(d->psi0[i]);
        hm[i].L = st.heff[i]->L;
        hm[i].cls = st.heff[i]->op_class;
        for (int k = 0; k < hm[i].L; ++k) hm[i].rate[k] = d->rates[i][k];
    }
    std::vector<int> mo(d->model_of_traj, d->model_of_traj + nt);
    std::vector<int> ord;
    queue_order(d, &ord);
    ED_HIP_TRY(hipMemcpyAsync(dmod, hm.data(), sizeof(TrajModel) * hm.size(), hipMemcpyHostToDevice, s));
    if (nt > 0) {
        ED_HIP_TRY(hipMemcpyAsync(order, ord.data(), sizeof(int) * nt, hipMemcpyHostToDevice, s));
        ED_HIP_TRY(hipMemcpyAsync(model_of, mo.data(), sizeof(int) * nt, hipMemcpyHostToDevice, s));
    }
    TrajArgs a;
    std::memset(&a, 0, sizeof(a));
    a.models = dmod;
    a.order = order;
    a.model_of = model_of;
    a.n_traj = nt;
    a.dt = d->dt;
    a.n_steps = d->n_steps;
    a.out_stride = d->out_stride;
    a.n_out = n_out;
    a.seed = d->seed;
    a.m_max = p->m_max;
    a.tol = p->tol;
    a.max_jumps = p->max_jumps;
    for (int e = 0; e < 4; ++e) a.J[e] = make_double2(d->jump_op[e].re, d->jump_op[e].im);
    a.jdj_up = st.jdj_up;
    a.jdj_dn = st.jdj_dn;
    a.Lmax = Lmax;
    a.sz_out = sz;
    a.n_jumps = njumps;
    a.jump_t = jt;
    a.jump_site = js;
    a.m_total = mtot;
    a.unconverged = unconv;
    a.scratch = scratch;
    a.scratch_stride = int64_t(per);
    a.counter = counter;
    a.busy = busy;
    // clear the counters and the outputs with fill kernels, then the persistent launch; on a
    // non-null stream the three launches are captured as a hipGraph and run through the stream's
    // executable graph, which a later call updates in place (new arguments, same topology) and
    // replays instead of instantiating again
    auto enqueue = [&]() -> hipError_t {
        hipLaunchKernelGGL(zero_ints, dim3(1), dim3(64), 0, s, counter, 4);
        if (nt == 0) return hipGetLastError();
        const int64_t nz = int64_t(nt) * n_out * Lmax;
        hipLaunchKernelGGL(zero_doubles, dim3(unsigned((nz + 255) / 256)), dim3(256), 0, s, sz, nz);
        return launch_traj<0>(st.cls, dim3(G), 0, s, a);
    };
    if (s == nullptr) {
        hipError_t e = enqueue();
        if (e != hipSuccess) return fail(ED_ERR_HIP, std::string("trajectory launch: ") + hipGetErrorString(e));
        ED_HIP_TRY(hipStreamSynchronize(s));
    } else {
        hipGraph_t graph = nullptr;
        ED_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue();
        hipError_t ce = hipStreamEndCapture(s, &graph);
        if (e != hipSuccess || ce != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(ED_ERR_HIP, std::string("trajectory capture: ") + hipGetErrorString(e != hipSuccess ? e : ce));
        }
        std::lock_guard<std::mutex> lock(g_traj_graph_mu);
        int dev = 0;
        (void)hipGetDevice(&dev);
        hipGraphExec_t& exec = g_traj_graph[{dev, s}];
        bool updated = false;
        if (exec) {
            hipGraphNode_t err_node = nullptr;
            hipGraphExecUpdateResult ur = hipGraphExecUpdateError;
            updated = hipGraphExecUpdate(exec, graph, &err_node, &ur) == hipSuccess && ur == hipGraphExecUpdateSuccess;
            if (!updated) {
                (void)hipGetLastError();
                (void)hipGraphExecDestroy(exec);
                exec = nullptr;
            }
        }
        if (!exec) {
            hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (ie != hipSuccess) {
                exec = nullptr;
                (void)hipGraphDestroy(graph);
                return fail(ED_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
            }
        }
        (void)hipGraphDestroy(graph);
        hipError_t le = hipGraphLaunch(exec, s);
        hipError_t se = hipStreamSynchronize(s);
        if (le != hipSuccess) return fail(ED_ERR_HIP, std::string("graph launch: ") + hipGetErrorString(le));
        if (se != hipSuccess) return fail(ED_ERR_HIP, std::string("trajectory kernel: ") + hipGetErrorString(se));
        if (info) info->graph_replayed = updated ? 1 : 0;
    }
    // outputs to the host
    std::vector<double> hsz(size_t(nt) * n_out * Lmax);
    std::vector<int> hnj(nt), hmt(nt), hun(nt);
    if (nt > 0) {
        ED_HIP_TRY(hipMemcpy(hsz.data(), sz, sizeof(double) * hsz.size(), hipMemcpyDeviceToHost));
        ED_HIP_TRY(hipMemcpy(hnj.data(), njumps, sizeof(int) * nt, hipMemcpyDeviceToHost));
        ED_HIP_TRY(hipMemcpy(hmt.data(), mtot, sizeof(int) * nt, hipMemcpyDeviceToHost));
        ED_HIP_TRY(hipMemcpy(hun.data(), unconv, sizeof(int) * nt, hipMemcpyDeviceToHost));
    }
    std::memcpy(out->sz, hsz.data(), sizeof(double) * hsz.size());
    if (out->n_jumps) std::memcpy(out->n_jumps, hnj.data(), sizeof(int) * nt);
    if ((out->jump_t || out->jump_site) && p->max_jumps > 0 && nt > 0) {
        std::vector<double> hjt(size_t(nt) * mj);
        std::vector<int> hjs(size_t(nt) * mj);
        ED_HIP_TRY(hipMemcpy(hjt.data(), jt, sizeof(double) * hjt.size(), hipMemcpyDeviceToHost));
        ED_HIP_TRY(hipMemcpy(hjs.data(), js, sizeof(int) * hjs.size(), hipMemcpyDeviceToHost));
        if (out->jump_t) std::memcpy(out->jump_t, hjt.data(), sizeof(double) * hjt.size());
        if (out->jump_site) std::memcpy(out->jump_site, hjs.data(), sizeof(int) * hjs.size());
    }
    for (int i = 0; i < nt; ++i)
        if (hnj[i] < 0) return fail(ED_ERR_NUMERIC, "trajectory " + std::to_string(i) + " hit a non-finite norm or too many jumps in one step");
    if (info) {
        long long tj = 0, tm = 0, tu = 0;
        for (int i = 0; i < nt; ++i) {
            tj += hnj[i];
            tm += hmt[i];
            tu += hun[i];
        }
        info->total_jumps = tj;
        info->total_krylov = tm;
        info->blocks = G;
        info->unconverged_steps = tu;
        if (s == nullptr) info->graph_replayed = 0;
        // per-workgroup busy time (the balance of the dealt lists)
        std::vector<long long> hb(G);
        ED_HIP_TRY(hipMemcpy(hb.data(), busy, sizeof(long long) * G, hipMemcpyDeviceToHost));
        int dev = 0, khz = 0;
        ED_HIP_TRY(hipGetDevice(&dev));
        ED_HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        double mx = 0.0, mn = 0.0, sum = 0.0;
        for (int g = 0; g < G; ++g) {
            const double ms = khz > 0 ? double(hb[g]) / double(khz) : 0.0;
            mx = g == 0 ? ms : std::max(mx, ms);
            mn = g == 0 ? ms : std::min(mn, ms);
            sum += ms;
        }
        info->busy_max_ms = mx;
        info->busy_min_ms = mn;
        info->busy_mean_ms = G > 0 ? sum / G : 0.0;
    }
    return ED_OK;
}

// ----------------------------------------------------------------------------- plain path
// One trajectory at a time from the host: the Arnoldi basis from the stream-level kernels, the
// small exponential, root search and jump choice on the host, the jump itself by a kernel.
namespace ed {
namespace {
__global__ void apply_site_op(double2* psi, int L, int p, double2 j0, double2 j1, double2 j2, double2 j3) {
    const int64_t half = int64_t(1) << (L - 1);
    const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= half) return;
    const int64_t lowm = (int64_t(1) << p) - 1;
    const int64_t x0 = ((q & ~lowm) << 1) | (q & lowm);
    const int64_t x1 = x0 | (int64_t(1) << p);
    const double2 a0 = psi[x0], a1 = psi[x1];
    psi[x0] = make_double2(j0.x * a0.x - j0.y * a0.y + j1.x * a1.x - j1.y * a1.y, j0.x * a0.y + j0.y * a0.x + j1.x * a1.y + j1.y * a1.x);
    psi[x1] = make_double2(j2.x * a0.x - j2.y * a0.y + j3.x * a1.x - j3.y * a1.y, j2.x * a0.y + j2.y * a0.x + j3.x * a1.y + j3.y * a1.x);
}
}  // namespace
}  // namespace ed

extern "C" ed_status ed_trajectories_plain_workspace(const ed_traj_desc* d, const ed_traj_params* p, size_t* bytes) {
    if (!bytes) return fail(ED_ERR_ARG, "bytes is null");
    ED_TRY(validate_traj(d, p));
    int Lmax = 0;
    for (int i = 0; i < d->n_models; ++i) Lmax = std::max(Lmax, d->models[i]->L);
    *bytes = core_scratch_bytes() + al256(size_t(p->m_max + 2) * (size_t(1) << Lmax) * sizeof(double2));
    return ED_OK;
}

extern "C" ed_status ed_trajectories_plain(const ed_traj_desc* d, const ed_traj_params* p, const ed_traj_out* out,
                                           ed_traj_info* info, void* ws, size_t ws_bytes, void* stream) {
    ED_TRY(validate_traj(d, p));
    if (!out || !out->sz) return fail(ED_ERR_ARG, "output sz is null");
    size_t need = 0;
    ED_TRY(ed_trajectories_plain_workspace(d, p, &need));
    if (!ws) return fail(ED_ERR_ARG, "workspace is null");
    if (ws_bytes < need) return fail(ED_ERR_WORKSPACE, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    TrajSetup st;
    ED_TRY(build_setup(d, &st));
    const int Lmax = st.Lmax, n_out = st.n_out, nt = d->n_traj;
    const int mj = std::max(p->max_jumps, 1);
    std::fill(out->sz, out->sz + size_t(nt) * n_out * Lmax, 0.0);
    long long tot_j = 0, tot_m = 0, tot_unconv = 0;
    for (int tr = 0; tr < nt; ++tr) {
        const int mi = d->model_of_traj[tr];
        const ed_model* hm = st.heff[mi].get();
        const int L = hm->L;
        const int64_t D = int64_t(1) << L;
        Workspace w;
        ED_TRY(carve(ws, ws_bytes, D, p->m_max + 2, &w));
        double2* psi = w.V + int64_t(p->m_max + 1) * D;  // the state lives after the basis
        ED_HIP_TRY(hipMemcpyAsync(psi, d->psi0[mi], sizeof(double2) * D, hipMemcpyDeviceToDevice, s));
        double n0 = 0.0;
        ED_TRY(start_vector(w, psi, &n0, s));
        ED_HIP_TRY(hipMemcpyAsync(psi, w.V, sizeof(double2) * D, hipMemcpyDeviceToDevice, s));
        uint64_t ndraw = 0;
        auto draw = [&]() {
            const double u = to_unit(philox_word(d->seed, uint64_t(tr), ndraw));
            ++ndraw;
            return u;
        };
        double r = draw();
        int njump = 0;
        double* szo = out->sz + size_t(tr) * n_out * Lmax;
        auto record = [&](int slot) -> ed_status {
            std::vector<double> szv(L);
            ED_TRY(measure_state(psi, L, w, szv.data(), nullptr, s));
            for (int k = 0; k < L; ++k) szo[size_t(slot) * Lmax + k] = szv[k];
            return ED_OK;
        };
        ED_TRY(record(0));
        for (int step = 0; step < d->n_steps; ++step) {
            double tau_left = d->dt;
            while (tau_left > 0.0) {
                double nrm = 0.0;
                ED_TRY(start_vector(w, psi, &nrm, s));
                const double n2 = nrm * nrm;
                const int mmax = p->m_max;
                std::vector<cplx> T(size_t(mmax + 1) * (mmax + 1), 0.0), h(mmax + 1), u(mmax + 1);
                int m = 0;
                auto expv = [&](int mm, double tau, std::vector<cplx>& uu) {
                    std::vector<cplx> A(size_t(mm) * mm), E(size_t(mm) * mm);
                    for (int r2 = 0; r2 < mm; ++r2)
                        for (int c2 = 0; c2 < mm; ++c2) A[size_t(r2) * mm + c2] = cplx(0.0, -tau) * T[size_t(r2) * (mmax + 1) + c2];
                    expm_complex(mm, A.data(), E.data());
                    for (int r2 = 0; r2 < mm; ++r2) uu[r2] = E[size_t(r2) * mm];
                };
                for (int j = 0; j < mmax; ++j) {
                    double beta = 0.0;
                    bool brk = false;
                    ED_TRY(krylov_step(hm, w, j, 0, 2, 1e-14, h.data(), &beta, &brk, s));
                    for (int i = 0; i <= j; ++i) T[size_t(i) * (mmax + 1) + j] = h[i];
                    m = j + 1;
                    expv(m, tau_left, u);
                    const double err = brk ? 0.0 : nrm * beta * std::abs(u[m - 1]);
                    if (brk || err <= p->tol || m >= mmax) {
                        if (!brk && err > p->tol) ++tot_unconv;
                        break;
                    }
                    T[size_t(j + 1) * (mmax + 1) + j] = beta;
                }
                tot_m += m;
                auto lnorm = [&](const std::vector<cplx>& uu) {
                    double q = 0.0;
                    for (int i = 0; i < m; ++i) q += std::norm(uu[i]);
                    return std::log(n2 * q);
                };
                const double lr = std::log(r);
                const double f_end = lnorm(u) - lr;
                auto combine = [&](const std::vector<cplx>& uu) -> ed_status {
                    std::vector<double2> c(m);
                    for (int i = 0; i < m; ++i) c[i] = make_double2(nrm * uu[i].real(), nrm * uu[i].imag());
                    return combine_basis(w, m, c.data(), psi, s);
                };
                if (f_end > 0.0) {
                    ED_TRY(combine(u));
                    tau_left = 0.0;
                    break;
                }
                double lo = 0.0, hi = tau_left, flo = std::log(n2) - lr, fhi = f_end, tau = hi;
                if (flo <= 0.0) {
                    tau = 0.0;
                } else {
                    int side = 0;
                    for (int it = 0; it < 200; ++it) {
                        double c = hi - fhi * (hi - lo) / (fhi - flo);
                        if (!(c > lo && c < hi)) c = 0.5 * (lo + hi);
                        expv(m, c, u);
                        const double fc = lnorm(u) - lr;
                        if (fc > 0.0) {
                            lo = c;
                            flo = fc;
                            if (side == -1) fhi *= 0.5;
                            side = -1;
                        } else {
                            hi = c;
                            fhi = fc;
                            if (side == 1) flo *= 0.5;
                            side = 1;
                        }
                        tau = hi;
                        if (fc == 0.0 || hi - lo <= 1e-15 * d->dt) {
                            tau = (fc == 0.0) ? c : hi;
                            break;
                        }
                    }
                }
                expv(m, tau, u);
                ED_TRY(combine(u));
                const double t_abs = step * d->dt + (d->dt - tau_left) + tau;
                std::vector<double> szv(L);
                double nn = 0.0;
                ED_TRY(measure_state(psi, L, w, szv.data(), &nn, s));
                const double rk = draw();
                int kappa = L - 1;
                double ptot = 0.0;
                std::vector<double> pk(L);
                for (int nu = 0; nu < L; ++nu) {
                    const double up = 0.5 * (1.0 + szv[nu]) * nn * nn;
                    pk[nu] = d->rates[mi][nu] * (st.jdj_up * up + st.jdj_dn * (nn * nn - up));
                    ptot += pk[nu];
                }
                double cum = 0.0;
                for (int nu = 0; nu < L; ++nu) {
                    cum += pk[nu];
                    if (rk <= cum / ptot) {
                        kappa = nu;
                        break;
                    }
                }
                const ed_c64* J = d->jump_op;
                const int64_t half = D / 2;
                hipLaunchKernelGGL(apply_site_op, dim3(unsigned((half + 255) / 256)), dim3(256), 0, s, psi, L, L - 1 - kappa,
                                   make_double2(J[0].re, J[0].im), make_double2(J[1].re, J[1].im),
                                   make_double2(J[2].re, J[2].im), make_double2(J[3].re, J[3].im));
                ED_HIP_TRY(hipGetLastError());
                ED_TRY(start_vector(w, psi, &nn, s));
                ED_HIP_TRY(hipMemcpyAsync(psi, w.V, sizeof(double2) * D, hipMemcpyDeviceToDevice, s));
                if (njump < p->max_jumps) {
                    if (out->jump_t) out->jump_t[size_t(tr) * mj + njump] = t_abs;
                    if (out->jump_site) out->jump_site[size_t(tr) * mj + njump] = kappa;
                }
                ++njump;
                r = draw();
                tau_left -= tau;
                if (tau_left <= 1e-15 * d->dt) tau_left = 0.0;
            }
            if ((step + 1) % d->out_stride == 0) ED_TRY(record((step + 1) / d->out_stride));
        }
        if (out->n_jumps) out->n_jumps[tr] = njump;
        tot_j += njump;
    }
    ED_HIP_TRY(hipStreamSynchronize(s));
    if (info) {
        info->total_jumps = tot_j;
        info->total_krylov = tot_m;
        info->blocks = 1;
        info->unconverged_steps = tot_unconv;
        info->graph_replayed = 0;
        info->busy_max_ms = info->busy_min_ms = info->busy_mean_ms = 0.0;
    }
    return ED_OK;
}

// Raw Philox words as the trajectories draw them (for checking the generator against its
// published definition): out[i] = word i of the stream of key (seed, id).
namespace ed {
namespace {
__global__ void philox_words_kernel(uint64_t seed, uint64_t id, uint64_t* out, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = philox_word(seed, id, uint64_t(i));
}
}  // namespace
}  // namespace ed

extern "C" ed_status ed_philox_words(uint64_t seed, uint64_t id, uint64_t* out, int64_t n, void* stream) {
    if (!out || n < 0) return fail(ED_ERR_ARG, "bad argument");
    if (n == 0) return ED_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(philox_words_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, seed, id, out, n);
    ED_HIP_TRY(hipGetLastError());
    return ED_OK;
}
