// out = H psi for a site + bond rule set on a dense complex128 state (Sec. III.C: the rule set
// applied to the state without storing H, cost L(2 n_b + n_s) O(d^(L+1)), Eq. ed:eq:OKrylov).
//
// The paper contracts each rule with the rank-L tensor (tensordot + permutation per rule and
// site). Here the state streams through HBM in a few passes. Each pass stages a 2^12-amplitude
// tile in LDS; the tile spans either the 12 low bits (first pass: it also adds the diagonal of
// every term) or 3 low bits (128-byte runs) times a 9-bit window of high bits (later passes,
// which accumulate into out). Every site and bond term is assigned to exactly one pass, so a
// term whose bits both lie in the tile is evaluated entirely on chip: the partner amplitude
// psi[x ^ flip] comes from LDS, or from the thread's own registers when the flipped bits map to
// the register dimension of the tile.
#include "ed_internal.h"

namespace ed {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <bool REAL>
__device__ __forceinline__ void cfma(double2& acc, double2 c, double2 v) {
    if (REAL) {
        acc.x = fma(c.x, v.x, acc.x);
        acc.y = fma(c.x, v.y, acc.y);
    } else {
        acc.x = fma(c.x, v.x, acc.x);
        acc.x = fma(-c.y, v.y, acc.x);
        acc.y = fma(c.x, v.y, acc.y);
        acc.y = fma(c.y, v.x, acc.y);
    }
}

__device__ __forceinline__ double2 sel2(int b, double2 a0, double2 a1) {
    return b ? a1 : a0;
}

__device__ __forceinline__ double2 sel4(int l, double2 a0, double2 a1, double2 a2, double2 a3) {
    double2 lo = (l & 1) ? a1 : a0;
    double2 hi = (l & 1) ? a3 : a2;
    return (l & 2) ? hi : lo;
}

// -------------------------------------------------------------------------------------------
// Small-L kernel: one thread per output amplitude, partners read from global memory (the whole
// state is cache resident for L < 12).
template <unsigned CLS>
__global__ __launch_bounds__(256) void hpsi_small(const double2* __restrict__ psi,
                                                  double2* __restrict__ out,
                                                  const double2* __restrict__ site,
                                                  const double2* __restrict__ bond, int L) {
    constexpr bool OFFR = CLS & kOffReal;
    const int64_t D = int64_t(1) << L;
    const int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (x >= D) return;
    double2 v = psi[x];
    double2 diag = make_double2(0.0, 0.0);
    double2 acc = make_double2(0.0, 0.0);
    for (int p = 0; p < L; ++p) {
        const int b = (x >> p) & 1;
        const double2* S = site + 4 * p;
        diag.x += S[3 * b].x;
        diag.y += S[3 * b].y;
        if (CLS & kSiteOff) cfma<OFFR>(acc, S[b ? 2 : 1], psi[x ^ (int64_t(1) << p)]);
    }
    for (int p = 0; p + 1 < L; ++p) {
        const int l = (x >> p) & 3;
        const double2* B = bond + 16 * p;
        diag.x += B[5 * l].x;
        diag.y += B[5 * l].y;
        if (CLS & kBondSingle) {
            cfma<OFFR>(acc, B[4 * l + (l ^ 1)], psi[x ^ (int64_t(1) << p)]);
            cfma<OFFR>(acc, B[4 * l + (l ^ 2)], psi[x ^ (int64_t(2) << p)]);
        }
        if (CLS & kBondDouble) cfma<OFFR>(acc, B[4 * l + (l ^ 3)], psi[x ^ (int64_t(3) << p)]);
    }
    double2 dv = cmul(diag, v);
    out[x] = make_double2(acc.x + dv.x, acc.y + dv.y);
}

// -------------------------------------------------------------------------------------------
// Tiled pass. Tile-local index i = t + 256 k (t = thread, k = register slot 0..15): local bits
// 0..7 run across the threads, local bits 8..11 across the 16 registers of a thread.
constexpr int kSlots = (1 << kTileBits) / kTileThreads;  // 16

struct PassArgs {
    int c, h0, first;
    uint32_t site_mask, bond_mask;
    int bit_of[kTileBits];
};

template <unsigned CLS, bool FIRST>
__global__ __launch_bounds__(kTileThreads) void hpsi_tile(const double2* __restrict__ psi,
                                                          double2* __restrict__ out,
                                                          const double2* __restrict__ site,
                                                          const double2* __restrict__ bond,
                                                          const double2* __restrict__ dlo,
                                                          const double2* __restrict__ dmid,
                                                          const double2* __restrict__ dhi,
                                                          PassArgs pa) {
    constexpr bool OFFR = CLS & kOffReal;
    constexpr bool DIAGR = CLS & kDiagReal;
    __shared__ double2 s[1 << kTileBits];

    const int t = threadIdx.x;
    const int64_t n = blockIdx.x;
    // global index of tile-local index i
    int64_t base;
    if (FIRST) {
        base = n << kTileBits;
    } else {
        const int lo_bits = pa.h0 - pa.c;  // fixed bits between the low run and the window
        const int64_t nlo = n & ((int64_t(1) << lo_bits) - 1);
        const int64_t nhi = n >> lo_bits;
        base = (nlo << pa.c) | (nhi << (pa.h0 + kTileBits - pa.c));
    }
    auto gidx = [&](int i) -> int64_t {
        if (FIRST) return base + i;
        const int lowmask = (1 << pa.c) - 1;
        return base | int64_t(i & lowmask) | (int64_t(i >> pa.c) << pa.h0);
    };

    double2 v[kSlots];
    double2 acc[kSlots];
#pragma unroll
    for (int k = 0; k < kSlots; ++k) v[k] = psi[gidx(t + kTileThreads * k)];
    if (!FIRST) {
#pragma unroll
        for (int k = 0; k < kSlots; ++k) acc[k] = out[gidx(t + kTileThreads * k)];
    }
#pragma unroll
    for (int k = 0; k < kSlots; ++k) s[t + kTileThreads * k] = v[k];

    if (FIRST) {
        // diagonal of every term: low table (bits 0..7) + middle (bits 7..11) + high (bits 11..)
        const double2 dl = dlo[t & 255];
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            const int i = t + kTileThreads * k;
            const double2 dm = dmid[(i >> 7) & 31];
            const double2 dh = dhi[(n << 1) | ((i >> 11) & 1)];
            double2 dd = make_double2(dl.x + dm.x + dh.x, dl.y + dm.y + dh.y);
            if (DIAGR) {
                acc[k] = make_double2(dd.x * v[k].x, dd.x * v[k].y);
            } else {
                acc[k] = cmul(dd, v[k]);
            }
        }
    }
    __syncthreads();

#pragma unroll
    for (int q = 0; q < kTileBits; ++q) {
        const int p = pa.bit_of[q];
        if ((CLS & kSiteOff) && ((pa.site_mask >> q) & 1)) {
            const double2 c01 = site[4 * p + 1];
            const double2 c10 = site[4 * p + 2];
#pragma unroll
            for (int k = 0; k < kSlots; ++k) {
                const int i = t + kTileThreads * k;
                const int b = (i >> q) & 1;
                double2 w;
                if (q >= 8) {
                    w = v[k ^ (1 << (q >= 8 ? q - 8 : 0))];
                } else {
                    w = s[i ^ (1 << q)];
                }
                cfma<OFFR>(acc[k], sel2(b, c01, c10), w);
            }
        }
        if ((CLS & (kBondSingle | kBondDouble)) && q + 1 < kTileBits && ((pa.bond_mask >> q) & 1)) {
            const double2* B = bond + 16 * p;
            if (CLS & kBondSingle) {
#pragma unroll
                for (int m = 1; m <= 2; ++m) {
                    const double2 b0 = B[0 * 4 + (0 ^ m)], b1 = B[1 * 4 + (1 ^ m)];
                    const double2 b2 = B[2 * 4 + (2 ^ m)], b3 = B[3 * 4 + (3 ^ m)];
#pragma unroll
                    for (int k = 0; k < kSlots; ++k) {
                        const int i = t + kTileThreads * k;
                        const int l = (i >> q) & 3;
                        double2 w;
                        if (q >= 8) {
                            w = v[k ^ (m << (q >= 8 ? q - 8 : 0))];
                        } else {
                            w = s[i ^ (m << q)];
                        }
                        cfma<OFFR>(acc[k], sel4(l, b0, b1, b2, b3), w);
                    }
                }
            }
            if (CLS & kBondDouble) {
                const double2 b0 = B[0 * 4 + 3], b1 = B[1 * 4 + 2];
                const double2 b2 = B[2 * 4 + 1], b3 = B[3 * 4 + 0];
#pragma unroll
                for (int k = 0; k < kSlots; ++k) {
                    const int i = t + kTileThreads * k;
                    const int l = (i >> q) & 3;
                    double2 w;
                    if (q >= 8) {
                        w = v[k ^ (3 << (q >= 8 ? q - 8 : 0))];
                    } else {
                        w = s[i ^ (3 << q)];
                    }
                    cfma<OFFR>(acc[k], sel4(l, b0, b1, b2, b3), w);
                }
            }
        }
    }

#pragma unroll
    for (int k = 0; k < kSlots; ++k) out[gidx(t + kTileThreads * k)] = acc[k];
}

// Kernel variants: a model runs on the first variant whose work flags cover its own and whose
// "real" flags it satisfies.
constexpr unsigned kWork = kSiteOff | kBondSingle | kBondDouble;
constexpr unsigned kVariants[] = {
    kSiteOff | kOffReal | kDiagReal,                 // transverse-field Ising
    kBondDouble | kOffReal | kDiagReal,              // XXZ
    kBondDouble | kOffReal,                          // XXZ with a decay term (H_eff)
    kSiteOff | kBondDouble | kOffReal | kDiagReal,   // XXZ with transverse fields
    kSiteOff | kBondDouble | kOffReal,
    kSiteOff | kBondSingle | kBondDouble,            // anything
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <unsigned CLS>
hipError_t launch_variant(const ed_model* m, const double2* psi, double2* out, hipStream_t s) {
    const int L = m->L;
    if (L < kTileBits) {
        const int64_t D = int64_t(1) << L;
        const int threads = 256;
        const int blocks = int((D + threads - 1) / threads);
        hipLaunchKernelGGL((hpsi_small<CLS>), dim3(blocks), dim3(threads), 0, s, psi, out,
                           m->d_site, m->d_bond, L);
        return hipGetLastError();
    }
    const int64_t tiles = int64_t(1) << (L - kTileBits);
    for (int ip = 0; ip < m->n_pass; ++ip) {
        const PassDesc& pd = m->pass[ip];
        PassArgs pa;
        pa.c = pd.c;
        pa.h0 = pd.h0;
        pa.first = pd.first;
        pa.site_mask = pd.site_mask;
        pa.bond_mask = pd.bond_mask;
        for (int q = 0; q < kTileBits; ++q) pa.bit_of[q] = pd.bit_of[q];
        if (pd.first) {
            hipLaunchKernelGGL((hpsi_tile<CLS, true>), dim3(unsigned(tiles)), dim3(kTileThreads), 0, s,
                               psi, out, m->d_site, m->d_bond, m->d_diag_lo, m->d_diag_mid,
                               m->d_diag_hi, pa);
        } else {
            hipLaunchKernelGGL((hpsi_tile<CLS, false>), dim3(unsigned(tiles)), dim3(kTileThreads), 0,
                               s, psi, out, m->d_site, m->d_bond, m->d_diag_lo, m->d_diag_mid,
                               m->d_diag_hi, pa);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int I>
hipError_t dispatch(const ed_model* m, const double2* psi, double2* out, hipStream_t s) {
    if constexpr (I >= kNumVariants) {
        return hipErrorInvalidValue;
    } else {
        constexpr unsigned V = kVariants[I];
        const unsigned mc = m->op_class;
        const bool work_ok = ((mc & kWork) & ~(V & kWork)) == 0;
        const bool real_ok = ((V & ~kWork) & ~(mc & ~kWork)) == 0;
        if (work_ok && real_ok) return launch_variant<V>(m, psi, out, s);
        return dispatch<I + 1>(m, psi, out, s);
    }
}

}  // namespace

ed_status launch_apply_H(const ed_model* m, const double2* psi, double2* out, hipStream_t s) {
    hipError_t e = dispatch<0>(m, psi, out, s);
    if (e != hipSuccess) return fail(ED_ERR_HIP, std::string("apply_H launch: ") + hipGetErrorString(e));
    return ED_OK;
}

}  // namespace ed
