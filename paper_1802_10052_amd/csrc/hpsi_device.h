// Device-side bodies of out = H psi (Sec. ed:sec:krylov, Eq. ed:eq:OKrylov), shared by the streaming
// kernels (one tile per workgroup) and by the trajectory kernel (one workgroup walks every tile of
// its own small state).
#pragma once
#include "ed_internal.h"

namespace ed {

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

__device__ __forceinline__ double2 sel2(int b, double2 a0, double2 a1) { return b ? a1 : a0; }

__device__ __forceinline__ double2 sel4(int l, double2 a0, double2 a1, double2 a2, double2 a3) {
    double2 lo = (l & 1) ? a1 : a0;
    double2 hi = (l & 1) ? a3 : a2;
    return (l & 2) ? hi : lo;
}

// Tile-local index i = t + 2^TB k: local bits 0..TB-1 across the threads of the workgroup,
// TB..11 across registers (TB = 8: 256 threads x 16 registers; TB = 10: 1024 threads x 4).
constexpr int kSlots = kTileSlots;  // 16, for TB = 8

struct PassArgs {
    int c, h0, first;
    uint32_t site_mask, bond_mask;
    int bit_of[kTileBits];
    int G, gb, gpos, gcross;
    const GatherJob* jobs;  // the pass's gathered terms (device), njobs of them
    int njobs;
    // long-range zz couplings (first pass only): lr_low[i] = pairs inside the tile's 12 bits,
    // lr_cross[p * L + q] = coupling of low bit p < 11 with high bit q >= 12
    int lr, L;
    const double2* lr_low;
    const double2* lr_cross;
    // last window pass with the product's projection on the input: dot_part[n] = the sum over
    // tile n of conj(psi[x]) out[x] (only the fused launch reads it)
    double2* dot_part;
};

// Operator tables of one model as the per-amplitude kernels see them.
struct ModelTables {
    const double2* site;
    const double2* bond;
    int L;
};

// First global index of tile n of a pass (the fixed bits of the tile).
__device__ __forceinline__ int64_t tile_base(const PassArgs& pa, bool first, int64_t n) {
    if (first) return n << kTileBits;
    const int lo_bits = pa.h0 - pa.c;
    const int64_t nlo = n & ((int64_t(1) << lo_bits) - 1);
    const int64_t nhi = n >> lo_bits;
    return (nlo << pa.c) | (nhi << (pa.h0 + kTileBits - pa.c));
}

__device__ __forceinline__ int64_t tile_index(const PassArgs& pa, bool first, int64_t base, int i) {
    if (first) return base + i;
    const int lowmask = (1 << pa.c) - 1;
    return base | int64_t(i & lowmask) | (int64_t(i >> pa.c) << pa.h0);
}

// Tile-local index t + 2^TB k sits at global index tile_index(t) + k * slot_step: the register
// slots only touch bits above the thread bits (c <= TB in window passes), so every slot of a
// thread is one uniform stride from the first and no per-slot 64-bit index is kept.
template <int TB = 8>
__device__ __forceinline__ int64_t slot_step(const PassArgs& pa, bool first) {
    return first ? (int64_t(1) << TB) : (int64_t((1 << TB) >> pa.c) << pa.h0);
}

// One tile of one pass (tile index n). s: 4096 double2 of LDS. FIRST: writes out including the
// diagonal; otherwise accumulates into out. GATHER: also evaluates the terms on the gathered bits
// above the tile (the pass's job list), reading partner amplitudes from the neighbouring tiles.
// PAIR: the workgroup holds two tiles, n and n ^ (tile-index bit gpos), one per half of its
// threads (t is the thread's index in its half, s its half's LDS tile, so the other half's
// tile); jobs whose partner is the other tile read it from LDS instead of global memory.
// TB: thread bits of the tile (8: 256 threads, 16 registers each; 10: 1024 threads, 4 each).
// Caller synchronises around reuse of s.
// DOT (last pass of the product, every thread of the workgroup calls with the same n layout):
// also writes pa.dot_part[n] = sum over the tile of conj(psi[x]) out[x], out being final here;
// sD holds one entry per wave of the tile. Contains a workgroup barrier.
// The load phase of a tile: thread t's amplitudes of psi (and, in later passes, of out, which is
// read once and not again by this pass: non-temporal, so that it does not evict the state tiles
// that neighbouring workgroups gather from L2).
template <bool FIRST, int TB>
__device__ __forceinline__ void tile_load(const double2* __restrict__ psi, const double2* __restrict__ out,
                                          const PassArgs& pa, int64_t n, int t, double2* v, double2* acc) {
    constexpr int kSl = 1 << (kTileBits - TB);
    const int64_t base = tile_base(pa, FIRST, n);
    const int64_t i0 = tile_index(pa, FIRST, base, t);
    const int64_t step = slot_step<TB>(pa, FIRST);
    const double2* __restrict__ pv = psi + i0;
#pragma unroll
    for (int k = 0; k < kSl; ++k) v[k] = pv[k * step];
    if (!FIRST) {
#pragma unroll
        for (int k = 0; k < kSl; ++k) {
            const double* o = reinterpret_cast<const double*>(out + i0 + k * step);
            acc[k].x = __builtin_nontemporal_load(o);
            acc[k].y = __builtin_nontemporal_load(o + 1);
        }
    }
}

// The rest of a tile, once tile_load has filled v (and acc in later passes): stage the tile in
// LDS, evaluate every term of the pass, store out. Contains a workgroup barrier (two with DOT).
// PF: the partners of the first PF gathered jobs are loaded right after the tile is staged, so
// that their L2 round trips overlap the in-tile terms' LDS work; halfway through the thread bits
// their terms are added and the next PF jobs' partners loaded into the same registers. Jobs
// beyond 2 PF (and all jobs when PF = 0) are loaded one by one after the in-tile terms.
template <unsigned CLS, bool FIRST, bool GATHER = false, bool PAIR = false, int TB = 8, bool DOT = false, int PF = 0>
__device__ __forceinline__ void tile_finish(double2* __restrict__ out,
                                            const double2* __restrict__ site, const double2* __restrict__ bond,
                                            const double2* __restrict__ dlo, const double2* __restrict__ dmid,
                                            const double2* __restrict__ dhi, const PassArgs& pa, int64_t n,
                                            double2* s, int t, const double2* so, double2* sF, double2* sD,
                                            const double2* __restrict__ psi, double2* v, double2* acc) {
    constexpr bool OFFR = CLS & kOffReal;
    constexpr bool DIAGR = CLS & kDiagReal;
    constexpr int kThr = 1 << TB;                  // threads of one tile
    constexpr int kSl = 1 << (kTileBits - TB);     // register slots per thread
    static_assert(TB >= 8 && TB < kTileBits, "the diagonal tables take bits 0..7 from the thread index");
    static_assert(!PAIR || TB == 8, "paired tiles use 256 threads per tile");
    static_assert(PF == 0 || (GATHER && !PAIR), "prefetched jobs are read from global memory");
    const int64_t base = tile_base(pa, FIRST, n);
    const int64_t i0 = tile_index(pa, FIRST, base, t);
    const int64_t step = slot_step<TB>(pa, FIRST);
    const double2* __restrict__ pv = psi + i0;
#pragma unroll
    for (int k = 0; k < kSl; ++k) s[t + kThr * k] = v[k];

    if (FIRST && pa.lr && t < kTileBits - 1) {
        // long-range field on low bit t from the tile's fixed high bits (z = +1 for bit 0)
        double2 f = make_double2(0.0, 0.0);
        for (int q = kTileBits; q < pa.L; ++q) {
            const double z = ((n >> (q - kTileBits)) & 1) ? -1.0 : 1.0;
            const double2 c = pa.lr_cross[t * pa.L + q];
            f.x += z * c.x;
            f.y += z * c.y;
        }
        sF[t] = f;
    }
    if (FIRST) {
        const double2 dl = dlo[t & 255];
#pragma unroll
        for (int k = 0; k < kSl; ++k) {
            const int i = t + kThr * k;
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
    double2 gv[PF > 0 ? PF : 1][kSl];
    // jobs j0 .. j0 + PF - 1: load their partners into gv, or add their terms from gv
    auto pf_load = [&](int j0) {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            if (j0 + j < pa.njobs) {
                const GatherJob& jb = pa.jobs[j0 + j];
                const int sx = jb.sx ? (kSl >> 1) : 0;
                const double2* __restrict__ pw = pv + (tile_base(pa, FIRST, n ^ jb.txor) - base);
#pragma unroll
                for (int k = 0; k < kSl; ++k) gv[j][k] = pw[(k ^ sx) * step];
            }
        }
    };
    auto pf_use = [&](int j0) {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            if (j0 + j < pa.njobs) {
                const GatherJob& jb = pa.jobs[j0 + j];
                const int p = int((n >> jb.shift) & 3);
                const double2 c0 = jb.coef[p][0], c1 = jb.coef[p][1];
#pragma unroll
                for (int k = 0; k < kSl; ++k) cfma<OFFR>(acc[k], k >= kSl / 2 ? c1 : c0, gv[j][k]);
            }
        }
    };
    if constexpr (PF > 0) pf_load(0);
    if (FIRST && pa.lr) {
        // long-range zz: pairs inside the tile (table) + sum over low bits p < 11 of z_p F_p
        // (bits 0..TB-1 are the thread's, TB..10 the slot's)
        double2 st = make_double2(0.0, 0.0);
#pragma unroll
        for (int p = 0; p < TB; ++p) {
            const double z = ((t >> p) & 1) ? -1.0 : 1.0;
            st.x += z * sF[p].x;
            st.y += z * sF[p].y;
        }
#pragma unroll
        for (int k = 0; k < kSl; ++k) {
            const int i = t + kThr * k;
            double2 e = pa.lr_low[i];
            e.x += st.x;
            e.y += st.y;
#pragma unroll
            for (int p = TB; p < kTileBits - 1; ++p) {
                const double z = ((k >> (p - TB)) & 1) ? -1.0 : 1.0;
                e.x += z * sF[p].x;
                e.y += z * sF[p].y;
            }
            if (DIAGR) {
                acc[k].x += e.x * v[k].x;
                acc[k].y += e.x * v[k].y;
            } else {
                const double2 ev = cmul(e, v[k]);
                acc[k].x += ev.x;
                acc[k].y += ev.y;
            }
        }
    }

#pragma unroll
    for (int q = 0; q < kTileBits; ++q) {
        const int p = pa.bit_of[q];
        if ((CLS & kSiteOff) && ((pa.site_mask >> q) & 1)) {
            const double2 c01 = site[4 * p + 1];
            const double2 c10 = site[4 * p + 2];
#pragma unroll
            for (int k = 0; k < kSl; ++k) {
                const int i = t + kThr * k;
                const int b = (i >> q) & 1;
                double2 w;
                if (q >= TB) {
                    w = v[k ^ (1 << (q >= TB ? q - TB : 0))];
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
                    for (int k = 0; k < kSl; ++k) {
                        const int i = t + kThr * k;
                        const int l = (i >> q) & 3;
                        double2 w;
                        if (q >= TB) {
                            w = v[k ^ (m << (q >= TB ? q - TB : 0))];
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
                for (int k = 0; k < kSl; ++k) {
                    const int i = t + kThr * k;
                    const int l = (i >> q) & 3;
                    double2 w;
                    if (q >= TB) {
                        w = v[k ^ (3 << (q >= TB ? q - TB : 0))];
                    } else {
                        w = s[i ^ (3 << q)];
                    }
                    cfma<OFFR>(acc[k], sel4(l, b0, b1, b2, b3), w);
                }
            }
        }
        if constexpr (PF > 0) {
            // halfway through the thread bits: add the first jobs, load the next ones
            if (q == TB / 2 - 1) {
                pf_use(0);
                pf_load(PF);
            }
        }
    }

    if constexpr (GATHER) {
        // the crossing bond (gb-1, gb) flipping only the tile-local top bit: partner in registers
        if ((CLS & kBondSingle) && pa.gcross) {
            const double2* B = bond + 16 * (pa.gb - 1);
            const int hb = int((n >> pa.gpos) & 1);
            const double2 c0 = B[4 * (2 * hb) + (2 * hb + 1)], c1 = B[4 * (2 * hb + 1) + (2 * hb)];
#pragma unroll
            for (int k = 0; k < kSl; ++k) cfma<OFFR>(acc[k], k >= kSl / 2 ? c1 : c0, v[k ^ (kSl >> 1)]);
        }
        // gathered terms: partner tile n ^ txor, register slot k ^ sx, coefficients by pattern.
        // The second round of jobs loaded ahead, then the rest one by one. (What pays is hiding
        // the partner reads behind the in-tile LDS work; loading several partners per round
        // trip at this point, after that work, was measured slower.)
        int j0 = 0;
        if constexpr (PF > 0) {
            pf_use(PF);
            j0 = 2 * PF;
        }
        for (int j = j0; j < pa.njobs; ++j) {
            const GatherJob& jb = pa.jobs[j];
            const int sx = jb.sx ? (kSl >> 1) : 0;  // jobs flip at most the tile's top bit
            const int p = int((n >> jb.shift) & 3);
            const double2 c0 = jb.coef[p][0], c1 = jb.coef[p][1];
            if (PAIR && jb.txor == (int64_t(1) << pa.gpos)) {
#pragma unroll
                for (int k = 0; k < kSl; ++k)
                    cfma<OFFR>(acc[k], k >= kSl / 2 ? c1 : c0, so[t + kThr * (k ^ sx)]);
            } else {
                const double2* __restrict__ pw = pv + (tile_base(pa, FIRST, n ^ jb.txor) - base);
#pragma unroll
                for (int k = 0; k < kSl; ++k) cfma<OFFR>(acc[k], k >= kSl / 2 ? c1 : c0, pw[(k ^ sx) * step]);
            }
        }
    }

    // streaming stores: out is not read again by this pass, so it should not evict the state tiles
    // that neighbouring workgroups gather from L2
#pragma unroll
    for (int k = 0; k < kSl; ++k) {
        double* o = reinterpret_cast<double*>(out + i0 + k * step);
        __builtin_nontemporal_store(acc[k].x, o);
        __builtin_nontemporal_store(acc[k].y, o + 1);
    }
    if constexpr (DOT) {
        // the tile of psi is still in LDS; fixed order: slots, wave butterfly, waves
        double dx = 0.0, dy = 0.0;
#pragma unroll
        for (int k = 0; k < kSl; ++k) {
            const double2 p = s[t + kThr * k];
            dx = fma(p.x, acc[k].x, fma(p.y, acc[k].y, dx));
            dy = fma(p.x, acc[k].y, fma(-p.y, acc[k].x, dy));
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            dx += __shfl_xor(dx, o);
            dy += __shfl_xor(dy, o);
        }
        if ((t & 63) == 0) sD[t >> 6] = make_double2(dx, dy);
        __syncthreads();
        if (t == 0) {
            double2 sum = sD[0];
#pragma unroll
            for (int w = 1; w < kThr / 64; ++w) {
                sum.x += sD[w].x;
                sum.y += sD[w].y;
            }
            pa.dot_part[n] = sum;
        }
    }
}

// One tile of one pass (tile index n): tile_load, then tile_finish (see there).
template <unsigned CLS, bool FIRST, bool GATHER = false, bool PAIR = false, int TB = 8, bool DOT = false, int PF = 0>
__device__ __forceinline__ void tile_body(const double2* __restrict__ psi, double2* __restrict__ out,
                                          const double2* __restrict__ site, const double2* __restrict__ bond,
                                          const double2* __restrict__ dlo, const double2* __restrict__ dmid,
                                          const double2* __restrict__ dhi, const PassArgs& pa, int64_t n,
                                          double2* s, int t = 0, const double2* so = nullptr,
                                          double2* sF = nullptr, double2* sD = nullptr) {
    constexpr int kSl = 1 << (kTileBits - TB);
    if (!PAIR) t = threadIdx.x;
    double2 v[kSl];
    double2 acc[kSl];
    tile_load<FIRST, TB>(psi, out, pa, n, t, v, acc);
    tile_finish<CLS, FIRST, GATHER, PAIR, TB, DOT, PF>(out, site, bond, dlo, dmid, dhi, pa, n, s, t, so, sF, sD, psi,
                                                       v, acc);
}

// Per-amplitude body for one x (small L, or one small state per workgroup): partners read from
// `src` (global memory or LDS). Sites are taken 4 at a time, and every load of a chunk (partner
// amplitudes and per-lane table entries) is issued before any is used; out-of-range sites load
// index 0 entries and add nothing. A wave so keeps a chunk's loads in flight instead of waiting
// on one partner per term.
template <unsigned CLS>
__device__ __forceinline__ double2 small_entry(const double2* src, const double2* __restrict__ site,
                                               const double2* __restrict__ bond, int L, int64_t x) {
    constexpr bool OFFR = CLS & kOffReal;
    constexpr int CH = 4;
    const double2 v = src[x];
    double2 diag = make_double2(0.0, 0.0);
    double2 acc = make_double2(0.0, 0.0);
    for (int p0 = 0; p0 < L; p0 += CH) {
        double2 ds[CH], db[CH], ws[CH], cs[CH], w1[CH], c1[CH], w2[CH], c2[CH], w3[CH], c3[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int p = p0 + k;
            const bool sok = p < L, bok = p + 1 < L;
            const int ps = sok ? p : 0, pb = bok ? p : 0;
            const int b = int((x >> ps) & 1);
            const int l = int((x >> pb) & 3);
            const double2* B = bond + 16 * pb;
            ds[k] = site[4 * ps + 3 * b];
            db[k] = B[5 * l];
            if (CLS & kSiteOff) {
                ws[k] = src[x ^ (int64_t(1) << ps)];
                cs[k] = site[4 * ps + (b ? 2 : 1)];
            }
            if (CLS & kBondSingle) {
                w1[k] = src[x ^ (int64_t(1) << pb)];
                c1[k] = B[4 * l + (l ^ 1)];
                w2[k] = src[x ^ (int64_t(2) << pb)];
                c2[k] = B[4 * l + (l ^ 2)];
            }
            if (CLS & kBondDouble) {
                w3[k] = src[x ^ (int64_t(3) << pb)];
                c3[k] = B[4 * l + (l ^ 3)];
            }
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int p = p0 + k;
            if (p < L) {
                diag.x += ds[k].x;
                diag.y += ds[k].y;
                if (CLS & kSiteOff) cfma<OFFR>(acc, cs[k], ws[k]);
            }
            if (p + 1 < L) {
                diag.x += db[k].x;
                diag.y += db[k].y;
                if (CLS & kBondSingle) {
                    cfma<OFFR>(acc, c1[k], w1[k]);
                    cfma<OFFR>(acc, c2[k], w2[k]);
                }
                if (CLS & kBondDouble) cfma<OFFR>(acc, c3[k], w3[k]);
            }
        }
    }
    const double2 dv = cmul(diag, v);
    return make_double2(acc.x + dv.x, acc.y + dv.y);
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

__host__ __device__ constexpr bool variant_fits(unsigned V, unsigned mc) {
    return (((mc & kWork) & ~(V & kWork)) == 0) && (((V & ~kWork) & ~(mc & ~kWork)) == 0);
}

inline int pick_variant(unsigned mc) {
    for (int i = 0; i < kNumVariants; ++i)
        if (variant_fits(kVariants[i], mc)) return i;
    return kNumVariants - 1;
}

inline PassArgs to_args(const PassDesc& pd, const GatherJob* jobs, int njobs) {
    PassArgs pa;
    pa.c = pd.c;
    pa.h0 = pd.h0;
    pa.first = pd.first;
    pa.site_mask = pd.site_mask;
    pa.bond_mask = pd.bond_mask;
    for (int q = 0; q < kTileBits; ++q) pa.bit_of[q] = pd.bit_of[q];
    pa.G = pd.G;
    pa.gb = pd.gb;
    pa.gpos = pd.gpos;
    pa.gcross = pd.gcross;
    pa.jobs = jobs;
    pa.njobs = njobs;
    pa.lr = 0;
    pa.L = 0;
    pa.lr_low = nullptr;
    pa.lr_cross = nullptr;
    pa.dot_part = nullptr;
    return pa;
}

inline ModelTables tables_of(const ed_model* m) {
    ModelTables tb;
    tb.site = m->d_site;
    tb.bond = m->d_bond;
    tb.L = m->L;
    return tb;
}

}  // namespace ed
