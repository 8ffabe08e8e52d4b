// Single-site and two-site reduced density matrices of a pure state (Sec. IV: rho of the kept
// sites is the sum over the traced indices of psi psi^*, arranged as the blocks [A][B] of the
// state with the kept legs in front; only one triangle is needed since rho is Hermitian), and
// the trace distance D = 1/2 Tr|rho - rho'| of the convergence study (Sec. V).
//
// rho_{k,j} for a pair of sites k < j (bits q = L-k > p = L-j) is, with u = bit q and v = bit p of
// the index, rho[2u+v][2u'+v'] = sum over the other bits of psi[.. u .. v ..] psi^*[.. u' .. v' ..].
// Every entry combines the four amplitudes of one "quad" {x, x|2^p, x|2^q, x|2^p|2^q} (x with both
// bits clear): 4 squared moduli and 6 conjugate products per quad and pair.
//
// The state is streamed in tiles of 2^T amplitudes (T = 12, 64 KiB of LDS) whose index bits are
// the 4 low bits (256-byte runs) plus 8 other bits; the quads of every pair of tile bits are then
// on chip. The high bits are cut into groups of 4; the tile of groups (a, b) holds every pair of
// bits inside low + G_a + G_b, so the C(m, 2) tiles cover all pairs (m = ceil((L-4)/4)). Each pair
// is evaluated in exactly one pass, the passes are balanced, and a pass holds at most 32 pairs
// (512 threads, 4 pairs per wave, each lane accumulating 16 doubles per pair over all of its
// tiles: 128 registers). One workgroup per CU is persistent over the tiles of a pass and loads
// the next tile into registers while it evaluates the current one from LDS; the reduction runs
// in a fixed order, so results are bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <vector>

#include "dense.h"
#include "ed_internal.h"

namespace ed {
namespace {

constexpr int kRdmThreads = 512;
constexpr int kThreadBits = 9;                                  // tile-local bits 0..8 = thread
constexpr int kSlots = 1 << (kTileBits - kThreadBits);          // amplitudes per thread (8)
constexpr int kWaves = kRdmThreads / 64;
constexpr int kRdmPairsPerWave = 4;
constexpr int kRdmMaxPairs = kWaves * kRdmPairsPerWave;  // pairs (work items) per pass
constexpr int kRdmLowBits = 4;
constexpr int kRdmMaxBlocks = 1024;  // workgroups per pass (one per CU)
constexpr int kRdmVals = 16;         // 4 real diagonal + 6 complex upper entries
constexpr int kRdmOff = 12;          // the 6 complex upper entries accumulated per work item
constexpr int kMaxComp = 30 - kTileBits;  // index bits outside a full tile (L <= 30)

struct RdmPass {
    int T;                         // tile bits
    int ncomp;                     // index bits outside the tile (L - T)
    int npairs;
    int nsplit;                    // work items per pair (each takes every nsplit-th run of 64 quads)
    int pos[kTileBits];            // global bit of tile-local bit i, ascending
    int comp[kMaxComp];            // global bits outside the tile, ascending
    int lp[kRdmMaxPairs];          // tile-local bits of each pair, lp < lq
    int lq[kRdmMaxPairs];
    int slot[kRdmMaxPairs];        // position of the pair in the lexicographic list of site pairs
};

// index of the site pair (k, j), 1 <= k < j <= L, in lexicographic order
__host__ __device__ inline int pair_slot(int k, int j, int L) { return (k - 1) * L - (k - 1) * k / 2 + (j - k - 1); }

// the six upper off-diagonal entries v_r conj(v_c), r < c, of one quad; the diagonal comes from
// the per-index probability sums
__device__ inline void quad_accumulate(double* a, double2 x0, double2 x1, double2 x2, double2 x3) {
    const double2 v[4] = {x0, x1, x2, x3};
    int o = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = r + 1; c < 4; ++c) {
            a[o] = fma(v[r].x, v[c].x, fma(v[r].y, v[c].y, a[o]));
            a[o + 1] = fma(v[r].y, v[c].x, fma(-v[r].x, v[c].y, a[o + 1]));
            o += 2;
        }
}

// insert a zero bit at position lo and one at position hi (lo < hi) into j
__host__ __device__ inline int insert_two(int j, int lo, int hi) {
    int x = ((j >> lo) << (lo + 1)) | (j & ((1 << lo) - 1));
    return ((x >> hi) << (hi + 1)) | (x & ((1 << hi) - 1));
}

// FULL: 2^12-amplitude tiles (L >= 12); otherwise the whole state (2^L < 4096) is one tile
template <bool FULL>
__global__ __launch_bounds__(kRdmThreads) void rdm_pass(const double2* __restrict__ psi, RdmPass pa, int64_t ntiles,
                                                        double* __restrict__ part, double* __restrict__ hist) {
    __shared__ double2 s[1 << kTileBits];
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);  // uniform: pair data in scalar registers
    const int tsize = FULL ? (1 << kTileBits) : (1 << pa.T);
    int64_t off_t = 0;
#pragma unroll
    for (int b = 0; b < kThreadBits; ++b)
        if ((FULL || b < pa.T) && ((t >> b) & 1)) off_t |= int64_t(1) << pa.pos[b];
    static_assert(kSlots == 8, "eight slot registers below");
    int64_t soff[kSlots];
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
        int64_t o = 0;
#pragma unroll
        for (int b = 0; b < kTileBits - kThreadBits; ++b)
            if ((FULL || kThreadBits + b < pa.T) && ((k >> b) & 1)) o |= int64_t(1) << pa.pos[kThreadBits + b];
        soff[k] = o;
    }
    // work item i = pair (i % npairs), part (i / npairs); wave w takes items w, w + 8, ...
    const int nitems = pa.npairs * pa.nsplit;
    double acc[kRdmPairsPerWave][kRdmOff];
#pragma unroll
    for (int w = 0; w < kRdmPairsPerWave; ++w)
#pragma unroll
        for (int e = 0; e < kRdmOff; ++e) acc[w][e] = 0.0;

    // the next tile is loaded into registers while the current one is evaluated from LDS; eight
    // named registers (an array that lives across the evaluation loop is placed in scratch memory)
    double2 v0, v1, v2, v3, v4, v5, v6, v7;
    // |psi|^2 of each of the thread's tile positions, summed over its tiles (the diagonal of every
    // pair's matrix is a marginal of these)
    double h0 = 0, h1 = 0, h2 = 0, h3 = 0, h4 = 0, h5 = 0, h6 = 0, h7 = 0;
#define ED_SLOT(k) (k == 0 ? v0 : k == 1 ? v1 : k == 2 ? v2 : k == 3 ? v3 : k == 4 ? v4 : k == 5 ? v5 : k == 6 ? v6 : v7)
#define ED_HIST(k) (k == 0 ? h0 : k == 1 ? h1 : k == 2 ? h2 : k == 3 ? h3 : k == 4 ? h4 : k == 5 ? h5 : k == 6 ? h6 : h7)
    int64_t n = blockIdx.x;
    if (n < ntiles) {
        int64_t base = off_t;
#pragma unroll
        for (int b = 0; b < kMaxComp; ++b)
            if (b < pa.ncomp && ((n >> b) & 1)) base |= int64_t(1) << pa.comp[b];
#pragma unroll
        for (int k = 0; k < kSlots; ++k)
            if (FULL || (k << kThreadBits) + t < tsize) ED_SLOT(k) = psi[base + soff[k]];
    }
    for (; n < ntiles; n += gridDim.x) {
        __syncthreads();  // the previous tile has been read
#pragma unroll
        for (int k = 0; k < kSlots; ++k)
            if (FULL || (k << kThreadBits) + t < tsize) {
                const double2 a = ED_SLOT(k);
                s[t + (k << kThreadBits)] = a;
                ED_HIST(k) = fma(a.x, a.x, fma(a.y, a.y, ED_HIST(k)));
            }
        __syncthreads();
        const int64_t nn = n + gridDim.x;
        if (nn < ntiles) {
            int64_t base = off_t;
#pragma unroll
            for (int b = 0; b < kMaxComp; ++b)
                if (b < pa.ncomp && ((nn >> b) & 1)) base |= int64_t(1) << pa.comp[b];
#pragma unroll
            for (int k = 0; k < kSlots; ++k) ED_SLOT(k) = psi[base + soff[k]];  // FULL only: ntiles > 1
        }
        const int rows = FULL ? (1 << (kTileBits - 2)) / 64 : ((tsize >> 2) + 63) / 64;  // runs of 64 quads
#pragma unroll
        for (int w = 0; w < kRdmPairsPerWave; ++w) {
            const int it = wave + kWaves * w;
            if (it < nitems) {  // uniform over the wave
                const int pi = it % pa.npairs, piece = it / pa.npairs;
                const int lp = pa.lp[pi], lq = pa.lq[pi];
                const int P = 1 << lp, Q = 1 << lq;
                // quad j = lane + 64 r: its base index is insert(lane) | insert(64 r) (disjoint bits)
                const int xl = insert_two(lane, lp, lq);
                int r = piece;
                if (FULL) {  // two quads per round: the second one's reads overlap the first one's FMAs
                    for (; r + pa.nsplit < rows; r += 2 * pa.nsplit) {
                        const double2* qa = s + (xl | insert_two(64 * r, lp, lq));
                        const double2* qb = s + (xl | insert_two(64 * (r + pa.nsplit), lp, lq));
                        const double2 a0 = qa[0], a1 = qa[P], a2 = qa[Q], a3 = qa[P + Q];
                        const double2 b0 = qb[0], b1 = qb[P], b2 = qb[Q], b3 = qb[P + Q];
                        quad_accumulate(acc[w], a0, a1, a2, a3);
                        quad_accumulate(acc[w], b0, b1, b2, b3);
                    }
                }
                for (; r < rows; r += pa.nsplit) {
                    if (!FULL && lane + 64 * r >= (tsize >> 2)) continue;
                    const double2* q = s + (xl | insert_two(64 * r, lp, lq));
                    quad_accumulate(acc[w], q[0], q[P], q[Q], q[P + Q]);
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kSlots; ++k)
        if (FULL || (k << kThreadBits) + t < tsize) hist[size_t(blockIdx.x) * (1 << kTileBits) + t + (k << kThreadBits)] = ED_HIST(k);
#undef ED_SLOT
#undef ED_HIST
    // fixed-order butterfly over the wave, then one row per (pair, workgroup)
#pragma unroll
    for (int w = 0; w < kRdmPairsPerWave; ++w) {
        const int it = wave + kWaves * w;
        if (it >= nitems) continue;
#pragma unroll
        for (int e = 0; e < kRdmOff; ++e) {
            double x = acc[w][e];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
            if (lane == 0) part[(size_t(it) * gridDim.x + blockIdx.x) * kRdmOff + e] = x;
        }
    }
}

// tile-position probabilities summed over the workgroups, in order
__global__ void rdm_hist_reduce(const double* __restrict__ hist, int nblocks, int tsize, double* __restrict__ H) {
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= tsize) return;
    double sum = 0.0;
#pragma unroll 8
    for (int g = 0; g < nblocks; ++g) sum += hist[size_t(g) * (1 << kTileBits) + y];
    H[y] = sum;
}

// one workgroup per pair of the pass: the table row's diagonal is the marginal of H over the
// pair's two tile bits (strided partial sums, then a fixed LDS tree); the upper entries are the
// sums of the per-workgroup rows of the pair's work items (parts, then workgroups, in order)
__global__ __launch_bounds__(256) void rdm_reduce(const double* __restrict__ part, int nblocks, RdmPass pa,
                                                  const double* __restrict__ H, double* __restrict__ table) {
    __shared__ double red[4][256];
    const int pi = blockIdx.x, t = threadIdx.x;
    const int lp = pa.lp[pi], lq = pa.lq[pi];
    const int nq = (1 << pa.T) >> 2;
    double d[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = t; j < nq; j += 256) {
        const int x = insert_two(j, lp, lq);
#pragma unroll
        for (int e = 0; e < 4; ++e) d[e] += H[x | ((e >> 1) << lq) | ((e & 1) << lp)];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) red[e][t] = d[e];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
#pragma unroll
            for (int e = 0; e < 4; ++e) red[e][t] += red[e][t + h];
        __syncthreads();
    }
    double* row = table + size_t(pa.slot[pi]) * kRdmVals;
    if (t < 4) row[t] = red[t][0];
    if (t >= 4 && t < kRdmVals) {
        const int e = t - 4;
        double sum = 0.0;
        for (int pt = 0; pt < pa.nsplit; ++pt) {
            const size_t it = size_t(pt) * pa.npairs + pi;
#pragma unroll 8
            for (int g = 0; g < nblocks; ++g) sum += part[(it * nblocks + g) * kRdmOff + e];
        }
        row[t] = sum;
    }
}

__device__ inline double2 upper_entry(const double* r, int a, int b) {
    // (a < b): position of (a, b) among (0,1),(0,2),(0,3),(1,2),(1,3),(2,3)
    const int o = a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
    return make_double2(r[4 + 2 * o], r[5 + 2 * o]);
}

// full 4x4 rho_{k,j} of every pair, and rho_k as the partial trace of a bond pair:
// rho_k = Tr_{k+1} rho_{k,k+1} for k < L, rho_L = Tr_{L-1} rho_{L-1,L}
__global__ void rdm_expand(const double* __restrict__ table, int L, int npairs, double2* __restrict__ rho1,
                           double2* __restrict__ rho2) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (rho2 && idx < npairs) {
        const double* r = table + size_t(idx) * kRdmVals;
        double2* o = rho2 + size_t(idx) * 16;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                double2 v;
                if (a == b) {
                    v = make_double2(r[a], 0.0);
                } else if (a < b) {
                    v = upper_entry(r, a, b);
                } else {
                    const double2 u = upper_entry(r, b, a);
                    v = make_double2(u.x, -u.y);
                }
                o[4 * a + b] = v;
            }
    }
    if (rho1 && idx < L) {
        const int k = idx + 1;
        double2* o = rho1 + size_t(idx) * 4;
        double d0, d1;
        double2 c;
        if (k < L) {  // trace over the second site of (k, k+1): sum over v
            const double* r = table + size_t(pair_slot(k, k + 1, L)) * kRdmVals;
            d0 = r[0] + r[1];
            d1 = r[2] + r[3];
            const double2 e02 = upper_entry(r, 0, 2), e13 = upper_entry(r, 1, 3);
            c = make_double2(e02.x + e13.x, e02.y + e13.y);
        } else {  // trace over the first site of (L-1, L): sum over u
            const double* r = table + size_t(pair_slot(L - 1, L, L)) * kRdmVals;
            d0 = r[0] + r[2];
            d1 = r[1] + r[3];
            const double2 e01 = upper_entry(r, 0, 1), e23 = upper_entry(r, 2, 3);
            c = make_double2(e01.x + e23.x, e01.y + e23.y);
        }
        o[0] = make_double2(d0, 0.0);
        o[1] = c;
        o[2] = make_double2(c.x, -c.y);
        o[3] = make_double2(d1, 0.0);
    }
}

// ---------------------------------------------------------------------------- planning
// Tile bit sets and the pairs each pass evaluates. all_pairs: every pair of bits; otherwise the
// bonds (p, p+1) only, which is what the single-site matrices need.
std::vector<RdmPass> rdm_plan(int L, bool all_pairs) {
    const int T = std::min(L, kTileBits);
    const int c = std::min(kRdmLowBits, T);
    const int W = T - c;
    const int nH = L - c;
    std::vector<std::vector<int>> sets;
    std::vector<int> group(L, -1);
    int m = 0;
    const int g = W / 2;
    if (nH <= W) {
        std::vector<int> all(L);
        for (int b = 0; b < L; ++b) all[b] = b;
        sets.push_back(all);
    } else {
        m = (nH + g - 1) / g;
        for (int b = c; b < L; ++b) group[b] = (b - c) / g;
        for (int a = 0; a < m; ++a)
            for (int b2 = a + 1; b2 < m; ++b2) {
                std::vector<bool> in(L, false);
                for (int b = 0; b < c; ++b) in[b] = true;
                for (int b = c; b < L; ++b)
                    if (group[b] == a || group[b] == b2) in[b] = true;
                int cnt = 0;
                for (int b = 0; b < L; ++b) cnt += in[b];
                for (int b = c; b < L && cnt < T; ++b)  // fill a short last group with other bits
                    if (!in[b]) {
                        in[b] = true;
                        ++cnt;
                    }
                std::vector<int> S;
                for (int b = 0; b < L; ++b)
                    if (in[b]) S.push_back(b);
                sets.push_back(S);
            }
    }
    const int nsets = int(sets.size());
    auto set_index = [&](int a, int b2) {  // a < b2
        return a * m - a * (a + 1) / 2 + (b2 - a - 1);
    };
    struct Req {
        int p, q;
        std::vector<int> cand;
    };
    std::vector<Req> reqs;
    for (int p = 0; p < L; ++p)
        for (int q = p + 1; q < L; ++q) {
            if (!all_pairs && q != p + 1) continue;
            Req r{p, q, {}};
            if (nsets == 1) {
                r.cand.push_back(0);
            } else {
                const int ga = group[p], gb = group[q];
                if (ga >= 0 && gb >= 0 && ga != gb) {
                    r.cand.push_back(set_index(std::min(ga, gb), std::max(ga, gb)));
                } else {
                    const int gg = ga >= 0 ? ga : gb;  // the one group involved, or -1 (both low)
                    for (int a = 0; a < m; ++a)
                        for (int b2 = a + 1; b2 < m; ++b2)
                            if (gg < 0 || a == gg || b2 == gg) r.cand.push_back(set_index(a, b2));
                }
            }
            reqs.push_back(r);
        }
    std::stable_sort(reqs.begin(), reqs.end(),
                     [](const Req& x, const Req& y) { return x.cand.size() < y.cand.size(); });
    std::vector<std::vector<std::pair<int, int>>> members(nsets);
    for (const Req& r : reqs) {
        // all pairs: the least loaded candidate (balanced passes); bonds only: a candidate that is
        // already in use, so that as few tiles as possible are streamed
        int best = -1;
        for (int s : r.cand) {
            if (best < 0) {
                best = s;
                continue;
            }
            const bool s_used = !members[s].empty(), b_used = !members[best].empty();
            if (!all_pairs && s_used != b_used) {
                if (s_used) best = s;
                continue;
            }
            if (members[s].size() < members[best].size()) best = s;
        }
        members[best].push_back({r.p, r.q});
    }
    std::vector<RdmPass> passes;
    for (int si = 0; si < nsets; ++si) {
        auto& mem = members[si];
        if (mem.empty()) continue;
        std::sort(mem.begin(), mem.end());
        const std::vector<int>& S = sets[si];
        std::vector<int> local(L, -1);
        for (int i = 0; i < int(S.size()); ++i) local[S[i]] = i;
        const int npass = (int(mem.size()) + kRdmMaxPairs - 1) / kRdmMaxPairs;
        for (int ps = 0; ps < npass; ++ps) {
            const int lo = int(mem.size()) * ps / npass, hi = int(mem.size()) * (ps + 1) / npass;
            RdmPass pa{};
            pa.T = T;
            for (int i = 0; i < T; ++i) pa.pos[i] = S[i];
            pa.ncomp = 0;
            for (int b = 0; b < L; ++b)
                if (local[b] < 0) pa.comp[pa.ncomp++] = b;
            pa.npairs = hi - lo;
            // passes with few pairs split each pair's quads over several work items
            pa.nsplit = std::max(1, std::min(kRdmMaxPairs / pa.npairs, std::max(1, (1 << (T - 2)) / 64)));
            for (int i = lo; i < hi; ++i) {
                const int p = mem[i].first, q = mem[i].second;
                pa.lp[i - lo] = local[p];
                pa.lq[i - lo] = local[q];
                pa.slot[i - lo] = pair_slot(L - q, L - p, L);
            }
            passes.push_back(pa);
        }
    }
    return passes;
}

size_t table_bytes(int L) { return size_t(L) * (L - 1) / 2 * kRdmVals * sizeof(double); }
size_t part_bytes() { return size_t(kRdmMaxPairs) * kRdmMaxBlocks * kRdmOff * sizeof(double); }
size_t hist_bytes() { return (size_t(kRdmMaxBlocks) + 1) * (size_t(1) << kTileBits) * sizeof(double); }

int rdm_blocks(int64_t ntiles) {
    int dev = 0, cu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cu = v;
    }
    return int(std::min<int64_t>({ntiles, int64_t(cu), int64_t(kRdmMaxBlocks)}));
}

}  // namespace

}  // namespace ed

using namespace ed;

extern "C" int ed_rdm_plan_pairs(int L, int all_pairs, int* pairs, int max_pairs, int* pass_of) {
    if (L < 2 || L > 30) return -1;
    const std::vector<RdmPass> ps = rdm_plan(L, all_pairs != 0);
    int n = 0;
    for (int i = 0; i < int(ps.size()); ++i)
        for (int j = 0; j < ps[i].npairs; ++j) {
            if (n < max_pairs && pairs && pass_of) {
                pairs[2 * n] = ps[i].pos[ps[i].lp[j]];
                pairs[2 * n + 1] = ps[i].pos[ps[i].lq[j]];
                pass_of[n] = i;
            }
            ++n;
        }
    return n;
}

extern "C" ed_status ed_rdm_workspace(int L, size_t* bytes) {
    if (!bytes || L < 2 || L > 30) return fail(ED_ERR_ARG, "bad argument (2 <= L <= 30)");
    *bytes = table_bytes(L) + part_bytes() + hist_bytes();
    return ED_OK;
}

extern "C" ed_status ed_rdm(const ed_c64* psi, int L, ed_c64* rho1, ed_c64* rho2, void* ws, size_t ws_bytes,
                            void* stream) {
    if (!psi || L < 2 || L > 30) return fail(ED_ERR_ARG, "bad argument (psi null or L outside 2..30)");
    if (!rho1 && !rho2) return ED_OK;
    size_t need = 0;
    ED_TRY(ed_rdm_workspace(L, &need));
    if (!ws) return fail(ED_ERR_ARG, "workspace is null");
    if (ws_bytes < need) return fail(ED_ERR_WORKSPACE, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* table = static_cast<double*>(ws);
    double* part = reinterpret_cast<double*>(static_cast<char*>(ws) + table_bytes(L));
    double* hist = part + part_bytes() / sizeof(double);
    double* H = hist + size_t(kRdmMaxBlocks) * (size_t(1) << kTileBits);
    const std::vector<RdmPass> passes = rdm_plan(L, rho2 != nullptr);
    const double2* p = reinterpret_cast<const double2*>(psi);
    for (const RdmPass& pa : passes) {
        const int64_t ntiles = int64_t(1) << pa.ncomp;
        const int G = rdm_blocks(ntiles);
        if (pa.T == kTileBits) {
            hipLaunchKernelGGL(rdm_pass<true>, dim3(G), dim3(kRdmThreads), 0, s, p, pa, ntiles, part, hist);
        } else {
            hipLaunchKernelGGL(rdm_pass<false>, dim3(G), dim3(kRdmThreads), 0, s, p, pa, ntiles, part, hist);
        }
        ED_HIP_TRY(hipGetLastError());
        const int tsize = 1 << pa.T;
        hipLaunchKernelGGL(rdm_hist_reduce, dim3((tsize + 255) / 256), dim3(256), 0, s, hist, G, tsize, H);
        ED_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(rdm_reduce, dim3(pa.npairs), dim3(256), 0, s, part, G, pa, H, table);
        ED_HIP_TRY(hipGetLastError());
    }
    const int npairs = L * (L - 1) / 2;
    const int nt = std::max(npairs, L);
    hipLaunchKernelGGL(rdm_expand, dim3((nt + 255) / 256), dim3(256), 0, s, table, L, npairs,
                       reinterpret_cast<double2*>(rho1), reinterpret_cast<double2*>(rho2));
    ED_HIP_TRY(hipGetLastError());
    return ED_OK;
}

extern "C" ed_status ed_trace_distances(int n, int count, const ed_c64* a, const ed_c64* b, double* out) {
    if (n < 1 || n > 64 || count < 0) return fail(ED_ERR_ARG, "bad argument (1 <= n <= 64, count >= 0)");
    if (count > 0 && (!a || !b || !out)) return fail(ED_ERR_ARG, "null argument");
    // The Hermitian difference X + iY (X symmetric, Y antisymmetric) has the eigenvalues of the
    // real symmetric [[X, -Y], [Y, X]], each twice.
    const int n2 = 2 * n;
    std::vector<double> S(size_t(n2) * n2), w(n2), Z(size_t(n2) * n2);
    for (int m = 0; m < count; ++m) {
        const ed_c64* A = a + size_t(m) * n * n;
        const ed_c64* B = b + size_t(m) * n * n;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const size_t ij = size_t(i) * n + j, ji = size_t(j) * n + i;
                const double dre = A[ij].re - B[ij].re, dim = A[ij].im - B[ij].im;
                const double tre = A[ji].re - B[ji].re, tim = A[ji].im - B[ji].im;
                if (!std::isfinite(dre) || !std::isfinite(dim)) return fail(ED_ERR_NUMERIC, "non-finite entry");
                const double x = 0.5 * (dre + tre), y = 0.5 * (dim - tim);  // Hermitian part
                S[size_t(i) * n2 + j] = x;
                S[size_t(i + n) * n2 + (j + n)] = x;
                S[size_t(i) * n2 + (j + n)] = -y;
                S[size_t(i + n) * n2 + j] = y;
            }
        if (!sym_eig_jacobi(n2, S.data(), w.data(), Z.data()))
            return fail(ED_ERR_NOCONV, "Jacobi eigenvalue iteration did not converge");
        double sum = 0.0;
        for (double v : w) sum += std::fabs(v);
        out[m] = 0.25 * sum;
    }
    return ED_OK;
}
