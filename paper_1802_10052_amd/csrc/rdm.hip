// Single-site and two-site reduced density matrices of a pure state (Sec. ed:sec:meas: rho of the kept
// sites is the sum over the traced indices of psi psi^*, arranged as the blocks [A][B] of the
// state with the kept legs in front; only one triangle is needed since rho is Hermitian), and
// the trace distance D = 1/2 Tr|rho - rho'| of the convergence study (Sec. ed:sec:conv).
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
// (512 threads, 4 pairs per wave, each lane accumulating the 12 doubles of a pair's upper entries
// over all of its tiles). Pairs that share bits are evaluated together: the 8 amplitudes of three
// bits hold two quads of each of the three pairs among them, so a "triangle" of pairs reads 8
// amplitudes for 6 quads and a "star" of two pairs 8 for 4, where single pairs read 4 per quad.
// The single-site matrices alone take a path of their own (one 2x2 matrix per bit, every bit of the
// tile evaluated on chip, ceil((L-4)/8) passes).
// One workgroup per CU is persistent over the tiles of a pass and loads
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

// Wave programs. A wave keeps 4 accumulator slots (12 doubles each) and runs one of these
// layouts of items over the quads of its tile:
//   a "cube" item holds three tile bits (a, b, c) and the pairs (a,b), (a,c) (a "star") or also
//   (b,c) (a "triangle"): each base x (those bits clear) gives 8 amplitudes and 2 quads per pair,
//   8 LDS reads for up to 6 quads. A pair's quad is accumulated in the order (none, first bit of
//   the item, second, both); where the first bit is the higher one, the slot is marked swapped
//   and the reduction exchanges basis states 1 and 2;
//   a "one" item is a single pair: 4 LDS reads per quad.
enum RdmLayout { kLayNone = 0, kLayTriOne = 1, kLayCubeCube = 2, kLayCubeOneOne = 3, kLayOnes = 4 };

struct RdmPass {
    int T;                         // tile bits
    int ncomp;                     // index bits outside the tile (L - T)
    int npairs;
    int pos[kTileBits];            // global bit of tile-local bit i, ascending
    int comp[kMaxComp];            // global bits outside the tile, ascending
    int lp[kRdmMaxPairs];          // tile-local bits of each pair, lp < lq
    int lq[kRdmMaxPairs];
    int slot[kRdmMaxPairs];        // position of the pair in the lexicographic list of site pairs
    int layout[kWaves];            // RdmLayout of each wave
    int piece[kWaves];             // the wave takes runs r = piece, piece + nsplit, ... of its bases
    int nsplit[kWaves];
    int ib[kWaves][4][3];          // tile bits of the wave's items (cube: a, b, c; one: lp, lq)
    int wpair[kWaves][4];          // pair index held by each accumulator slot, -1 if none
    int wswap[kWaves][4];          // 1 if the slot's quads list the pair's higher bit first
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

// insert zero bits at positions a < b < c
__host__ __device__ inline int insert_three(int j, int a, int b, int c) {
    const int x = insert_two(j, a, b);
    return ((x >> c) << (c + 1)) | (x & ((1 << c) - 1));
}

// One pair (bits lp < lq) into accumulator slot S over the quads of rows r = piece, piece + ns, ...
// (quad j = lane + 64 r; its base is insert(lane) | insert(64 r), disjoint bits).
template <int S, bool FULL>
__device__ __forceinline__ void run_one(double (&acc)[kRdmPairsPerWave][kRdmOff], const double2* s, int lane,
                                        int lp, int lq, int piece, int ns, int nq) {
    const int P = 1 << lp, Q = 1 << lq;
    const int rows = FULL ? (1 << (kTileBits - 2)) / 64 : (nq + 63) / 64;
    const int xl = insert_two(lane, lp, lq);
    int r = piece;
    if (FULL) {  // two quads per round: the second one's reads overlap the first one's FMAs
        for (; r + ns < rows; r += 2 * ns) {
            const double2* qa = s + (xl | insert_two(64 * r, lp, lq));
            const double2* qb = s + (xl | insert_two(64 * (r + ns), lp, lq));
            const double2 a0 = qa[0], a1 = qa[P], a2 = qa[Q], a3 = qa[P + Q];
            const double2 b0 = qb[0], b1 = qb[P], b2 = qb[Q], b3 = qb[P + Q];
            quad_accumulate(acc[S], a0, a1, a2, a3);
            quad_accumulate(acc[S], b0, b1, b2, b3);
        }
    }
    for (; r < rows; r += ns) {
        if (!FULL && lane + 64 * r >= nq) continue;
        const double2* q = s + (xl | insert_two(64 * r, lp, lq));
        quad_accumulate(acc[S], q[0], q[P], q[Q], q[P + Q]);
    }
}

// The pairs (a,b), (a,c) and, if TRI, (b,c) of the item bits a, b, c (distinct, in any order) into
// slots S0, S0 + 1, S0 + 2 (full tiles: 512 bases, 8 rows of 64). y[k] = amplitude at
// base + (k & 1) A + ((k >> 1) & 1) B + (k >> 2) C.
template <bool TRI, int S0>
__device__ __forceinline__ void run_cube(double (&acc)[kRdmPairsPerWave][kRdmOff], const double2* s, int lane,
                                         const int* bits, int piece, int ns) {
    const int a = bits[0], b = bits[1], c = bits[2];
    const int lo = min(a, min(b, c)), hi = max(a, max(b, c)), mid = a + b + c - lo - hi;
    const int A = 1 << a, B = 1 << b, C = 1 << c;
    const int xl = insert_three(lane, lo, mid, hi);
    for (int r = piece; r < (1 << (kTileBits - 3)) / 64; r += ns) {
        const double2* q = s + (xl | insert_three(64 * r, lo, mid, hi));
        const double2 y0 = q[0], y1 = q[A], y2 = q[B], y3 = q[A + B];
        const double2 y4 = q[C], y5 = q[A + C], y6 = q[B + C], y7 = q[A + B + C];
        quad_accumulate(acc[S0], y0, y1, y2, y3);
        quad_accumulate(acc[S0], y4, y5, y6, y7);
        quad_accumulate(acc[S0 + 1], y0, y1, y4, y5);
        quad_accumulate(acc[S0 + 1], y2, y3, y6, y7);
        if (TRI) {
            quad_accumulate(acc[S0 + 2], y0, y2, y4, y6);
            quad_accumulate(acc[S0 + 2], y1, y3, y5, y7);
        }
    }
}

// The tile loop of one wave program. All waves stream the same tiles and meet at the same
// barriers; each runs the copy of the loop specialised to its layout, so that the registers of the
// other layouts are not held through it. Two LDS buffers: while tile n is evaluated from one, the
// thread stores tile n + G (already in its registers) into the other and loads tile n + 2G into
// registers (G = gridDim.x); one barrier per tile.
template <bool FULL, int LAY>
__device__ __forceinline__ void tile_loop(const double2* __restrict__ psi, const RdmPass& pa, int64_t ntiles,
                                          double2 (*sb)[1 << kTileBits], double* sh, int t, int lane, int wave,
                                          int64_t off_t, const int64_t (&soff)[kSlots],
                                          double (&acc)[kRdmPairsPerWave][kRdmOff]) {
    const int tsize = FULL ? (1 << kTileBits) : (1 << pa.T);
    const int piece = pa.piece[wave], ns = pa.nsplit[wave];
    const int64_t G = gridDim.x;
    // eight named registers (an array that lives across the evaluation loop is placed in scratch)
    double2 v0, v1, v2, v3, v4, v5, v6, v7;
#define ED_SLOT(k) (k == 0 ? v0 : k == 1 ? v1 : k == 2 ? v2 : k == 3 ? v3 : k == 4 ? v4 : k == 5 ? v5 : k == 6 ? v6 : v7)
    auto load = [&](int64_t n) {
        int64_t base = off_t;
#pragma unroll
        for (int b = 0; b < kMaxComp; ++b)
            if (b < pa.ncomp && ((n >> b) & 1)) base |= int64_t(1) << pa.comp[b];
#pragma unroll
        for (int k = 0; k < kSlots; ++k)
            if (FULL || (k << kThreadBits) + t < tsize) ED_SLOT(k) = psi[base + soff[k]];
    };
    auto store = [&](double2* s) {  // the registers' tile into s, and its |psi|^2 into the histogram
#pragma unroll
        for (int k = 0; k < kSlots; ++k)
            if (FULL || (k << kThreadBits) + t < tsize) {
                const double2 a = ED_SLOT(k);
                s[t + (k << kThreadBits)] = a;
                double& h = sh[t + (k << kThreadBits)];
                h = fma(a.x, a.x, fma(a.y, a.y, h));
            }
    };
    int64_t n = blockIdx.x;
    if (n < ntiles) {
        load(n);
        store(sb[0]);
        if (n + G < ntiles) load(n + G);
    }
    __syncthreads();
    for (int it = 0; n < ntiles; n += G, ++it) {  // n, G, ntiles uniform: every wave takes the same steps
        const double2* s = sb[it & 1];
        if (n + G < ntiles) {
            store(sb[(it + 1) & 1]);  // read by every wave in the previous step, before its barrier
            if (n + 2 * G < ntiles) load(n + 2 * G);
        }
        const int nq = tsize >> 2;  // quads of one pair in one tile
        const int(*ib)[3] = pa.ib[wave];
        if (LAY == kLayTriOne) {
            run_cube<true, 0>(acc, s, lane, ib[0], piece, ns);
            if (pa.wpair[wave][3] >= 0) run_one<3, FULL>(acc, s, lane, ib[1][0], ib[1][1], piece, ns, nq);
        } else if (LAY == kLayCubeCube) {
            run_cube<false, 0>(acc, s, lane, ib[0], piece, ns);
            if (pa.wpair[wave][2] >= 0) run_cube<false, 2>(acc, s, lane, ib[1], piece, ns);
        } else if (LAY == kLayCubeOneOne) {
            run_cube<false, 0>(acc, s, lane, ib[0], piece, ns);
            if (pa.wpair[wave][2] >= 0) run_one<2, FULL>(acc, s, lane, ib[1][0], ib[1][1], piece, ns, nq);
            if (pa.wpair[wave][3] >= 0) run_one<3, FULL>(acc, s, lane, ib[2][0], ib[2][1], piece, ns, nq);
        } else if (LAY == kLayOnes) {
            if (pa.wpair[wave][0] >= 0) run_one<0, FULL>(acc, s, lane, ib[0][0], ib[0][1], piece, ns, nq);
            if (pa.wpair[wave][1] >= 0) run_one<1, FULL>(acc, s, lane, ib[1][0], ib[1][1], piece, ns, nq);
            if (pa.wpair[wave][2] >= 0) run_one<2, FULL>(acc, s, lane, ib[2][0], ib[2][1], piece, ns, nq);
            if (pa.wpair[wave][3] >= 0) run_one<3, FULL>(acc, s, lane, ib[3][0], ib[3][1], piece, ns, nq);
        }
        __syncthreads();  // tile n has been read and tile n + G stored
    }
#undef ED_SLOT
}

// FULL: 2^12-amplitude tiles (L >= 12); otherwise the whole state (2^L < 4096) is one tile
template <bool FULL>
__global__ __launch_bounds__(kRdmThreads) void rdm_pass(const double2* __restrict__ psi, RdmPass pa, int64_t ntiles,
                                                        double* __restrict__ part, double* __restrict__ hist) {
    __shared__ double2 s[2][1 << kTileBits];  // two tile buffers: 128 KiB
    // |psi|^2 of each tile position, summed over the workgroup's tiles (the diagonal of every pair's
    // matrix is a marginal of these); position y is owned by thread y mod 512. 32 KiB: with the
    // tiles, the 160 KiB of LDS of a CU
    __shared__ double sh[1 << kTileBits];
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);  // uniform: pair data in scalar registers
    const int tsize = FULL ? (1 << kTileBits) : (1 << pa.T);
    int64_t off_t = 0;
#pragma unroll
    for (int b = 0; b < kThreadBits; ++b)
        if ((FULL || b < pa.T) && ((t >> b) & 1)) off_t |= int64_t(1) << pa.pos[b];
    static_assert(kSlots == 8, "eight slot registers in the tile loop");
    int64_t soff[kSlots];
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
        int64_t o = 0;
#pragma unroll
        for (int b = 0; b < kTileBits - kThreadBits; ++b)
            if ((FULL || kThreadBits + b < pa.T) && ((k >> b) & 1)) o |= int64_t(1) << pa.pos[kThreadBits + b];
        soff[k] = o;
    }
    double acc[kRdmPairsPerWave][kRdmOff];
#pragma unroll
    for (int w = 0; w < kRdmPairsPerWave; ++w)
#pragma unroll
        for (int e = 0; e < kRdmOff; ++e) acc[w][e] = 0.0;
#pragma unroll
    for (int k = 0; k < kSlots; ++k) sh[t + (k << kThreadBits)] = 0.0;

    const int layout = pa.layout[wave];  // uniform over the wave
    if (FULL && layout == kLayTriOne)
        tile_loop<FULL, kLayTriOne>(psi, pa, ntiles, s, sh, t, lane, wave, off_t, soff, acc);
    else if (FULL && layout == kLayCubeCube)
        tile_loop<FULL, kLayCubeCube>(psi, pa, ntiles, s, sh, t, lane, wave, off_t, soff, acc);
    else if (FULL && layout == kLayCubeOneOne)
        tile_loop<FULL, kLayCubeOneOne>(psi, pa, ntiles, s, sh, t, lane, wave, off_t, soff, acc);
    else if (layout == kLayOnes)
        tile_loop<FULL, kLayOnes>(psi, pa, ntiles, s, sh, t, lane, wave, off_t, soff, acc);
    else
        tile_loop<FULL, kLayNone>(psi, pa, ntiles, s, sh, t, lane, wave, off_t, soff, acc);
    __syncthreads();  // every thread's histogram entries are complete
#pragma unroll
    for (int k = 0; k < kSlots; ++k)
        if (FULL || (k << kThreadBits) + t < tsize)
            hist[size_t(blockIdx.x) * (1 << kTileBits) + t + (k << kThreadBits)] = sh[t + (k << kThreadBits)];
    // fixed-order butterfly over the wave, then one row per (pair, workgroup)
#pragma unroll
    for (int w = 0; w < kRdmPairsPerWave; ++w) {
        if (pa.wpair[wave][w] < 0) continue;
        const int it = wave * kRdmPairsPerWave + w;
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
// sums of the per-workgroup rows of the accumulator slots holding the pair (slots, then
// workgroups, in order)
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
        const int e = t - 4, o = e >> 1;
        // a swapped slot holds the entries in the basis with states 1 and 2 exchanged: entry
        // (0,1) is at (0,2), (0,2) at (0,1), (1,3) at (2,3), (2,3) at (1,3), and (1,2) is the
        // conjugate of the stored one
        constexpr int kSwapFrom[6] = {1, 0, 2, 3, 5, 4};
        const int e_sw = 2 * kSwapFrom[o] + (e & 1);
        const double sign_sw = (o == 3 && (e & 1)) ? -1.0 : 1.0;
        double sum = 0.0;
        for (int it = 0; it < kWaves * kRdmPairsPerWave; ++it) {  // the slots holding this pair, in order
            const int w = it / kRdmPairsPerWave, k = it % kRdmPairsPerWave;
            if (pa.wpair[w][k] != pi) continue;
            const bool sw = pa.wswap[w][k] != 0;
            const int src = sw ? e_sw : e;
            double acc = 0.0;
#pragma unroll 8
            for (int g = 0; g < nblocks; ++g) acc += part[(size_t(it) * nblocks + g) * kRdmOff + src];
            sum += sw ? sign_sw * acc : acc;
        }
        row[t] = sum;
    }
}

// ---------------------------------------------------------------------------- single sites
// rho_k alone: for the site at bit b, rho_k[0][0] = sum |psi(x)|^2, rho_k[1][1] = sum |psi(x|B)|^2
// and rho_k[0][1] = sum psi(x) psi^*(x|B) over the x with bit b clear (Sec. ed:sec:meas, one kept site).
// A pass evaluates the bits of its tile that no earlier pass has: the 4 low bits and 8 others in
// the first pass, 8 others in each later one (ceil((L - 4) / 8) passes).
constexpr int kRdm1Vals = 4;  // d0, d1, Re c, Im c

struct Rdm1Pass {
    int T, ncomp, nbits;
    int pos[kTileBits];
    int comp[kMaxComp];
    int lb[kTileBits];  // tile-local bits evaluated by the pass
    int gb[kTileBits];  // their global bits
};

__device__ __forceinline__ void site_accumulate(double* a, double2 x, double2 y) {
    a[0] = fma(x.x, x.x, fma(x.y, x.y, a[0]));
    a[1] = fma(y.x, y.x, fma(y.y, y.y, a[1]));
    a[2] = fma(x.x, y.x, fma(x.y, y.y, a[2]));
    a[3] = fma(x.y, y.x, fma(-x.x, y.y, a[3]));
}

// Thread t owns tile positions t + 512 k (k = 0..7). For a bit b >= 9 both amplitudes of a pair
// are the thread's own; for b < 9 the thread with bit b clear takes slots 0..3 and its partner
// thread slots 4..7, each reading the other amplitude from LDS. Smaller tiles (L < 12) take every
// pair from LDS in the thread that owns x.
template <bool FULL>
__global__ __launch_bounds__(kRdmThreads) void rdm1_pass(const double2* __restrict__ psi, Rdm1Pass pa, int64_t ntiles,
                                                         double* __restrict__ part) {
    __shared__ double2 s[1 << kTileBits];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int tsize = FULL ? (1 << kTileBits) : (1 << pa.T);
    int64_t off_t = 0;
#pragma unroll
    for (int b = 0; b < kThreadBits; ++b)
        if ((FULL || b < pa.T) && ((t >> b) & 1)) off_t |= int64_t(1) << pa.pos[b];
    int64_t soff[kSlots];
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
        int64_t o = 0;
#pragma unroll
        for (int b = 0; b < kTileBits - kThreadBits; ++b)
            if ((FULL || kThreadBits + b < pa.T) && ((k >> b) & 1)) o |= int64_t(1) << pa.pos[kThreadBits + b];
        soff[k] = o;
    }
    double acc[kTileBits][kRdm1Vals];
#pragma unroll
    for (int i = 0; i < kTileBits; ++i)
#pragma unroll
        for (int e = 0; e < kRdm1Vals; ++e) acc[i][e] = 0.0;
    double2 v0, v1, v2, v3, v4, v5, v6, v7;
#define ED_SLOT(k) (k == 0 ? v0 : k == 1 ? v1 : k == 2 ? v2 : k == 3 ? v3 : k == 4 ? v4 : k == 5 ? v5 : k == 6 ? v6 : v7)
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
        double2 own[kSlots];
#pragma unroll
        for (int k = 0; k < kSlots; ++k)
            if (FULL || (k << kThreadBits) + t < tsize) {
                own[k] = ED_SLOT(k);
                s[t + (k << kThreadBits)] = own[k];
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
#pragma unroll
        for (int i = 0; i < kTileBits; ++i) {
            if (i >= pa.nbits) continue;  // uniform; no break, so that acc stays in registers
            const int b = pa.lb[i], B = 1 << b;
            if (!FULL) {
#pragma unroll
                for (int k = 0; k < kSlots; ++k) {
                    const int y = t + (k << kThreadBits);
                    if (y < tsize && !(y & B)) site_accumulate(acc[i], s[y], s[y | B]);
                }
            } else if (b >= kThreadBits) {  // both amplitudes in the thread's registers
                const int kb = b - kThreadBits;
#pragma unroll
                for (int k = 0; k < kSlots; ++k) {
                    if (kb == 0 && !(k & 1)) site_accumulate(acc[i], own[k], own[k | 1]);
                    if (kb == 1 && !(k & 2)) site_accumulate(acc[i], own[k], own[k | 2]);
                    if (kb == 2 && !(k & 4)) site_accumulate(acc[i], own[k], own[k | 4]);
                }
            } else if (!(t & B)) {  // x is ours: slots 0..3
#pragma unroll
                for (int k = 0; k < kSlots / 2; ++k)
                    site_accumulate(acc[i], own[k], s[(t | B) + (k << kThreadBits)]);
            } else {  // x|B is ours: slots 4..7
#pragma unroll
                for (int k = kSlots / 2; k < kSlots; ++k)
                    site_accumulate(acc[i], s[(t ^ B) + (k << kThreadBits)], own[k]);
            }
        }
    }
#undef ED_SLOT
    // fixed-order butterfly over the wave, one row per (workgroup, wave, bit)
#pragma unroll
    for (int i = 0; i < kTileBits; ++i) {
        if (i >= pa.nbits) continue;
#pragma unroll
        for (int e = 0; e < kRdm1Vals; ++e) {
            double x = acc[i][e];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
            if (lane == 0) part[((size_t(blockIdx.x) * kWaves + wave) * kTileBits + i) * kRdm1Vals + e] = x;
        }
    }
}

// one workgroup per evaluated bit: strided partial sums over (workgroup, wave) rows and a fixed
// LDS tree, then rho_k of the bit's site k = L - b
__global__ __launch_bounds__(256) void rdm1_reduce(const double* __restrict__ part, int nrows, Rdm1Pass pa, int L,
                                                   double2* __restrict__ rho1) {
    __shared__ double red[kRdm1Vals][256];
    const int i = blockIdx.x, t = threadIdx.x;
    double d[kRdm1Vals] = {0.0, 0.0, 0.0, 0.0};
    for (int r = t; r < nrows; r += 256)
#pragma unroll
        for (int e = 0; e < kRdm1Vals; ++e) d[e] += part[(size_t(r) * kTileBits + i) * kRdm1Vals + e];
#pragma unroll
    for (int e = 0; e < kRdm1Vals; ++e) red[e][t] = d[e];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
#pragma unroll
            for (int e = 0; e < kRdm1Vals; ++e) red[e][t] += red[e][t + h];
        __syncthreads();
    }
    if (t == 0) {
        double2* o = rho1 + size_t(L - 1 - pa.gb[i]) * 4;
        o[0] = make_double2(red[0][0], 0.0);
        o[1] = make_double2(red[2][0], red[3][0]);
        o[2] = make_double2(red[2][0], -red[3][0]);
        o[3] = make_double2(red[1][0], 0.0);
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
// Items of one pass (pairs pa.lp/pa.lq): with full tiles, up to max_tri triangles (three pairs on
// three bits), then stars (two pairs sharing a bit, as a cube item with two pairs), then single
// pairs; packed into wave layouts, at most 4 accumulator slots per wave. A pass with few waves
// repeats them with the bases split between the copies. Returns false if more than kWaves waves
// would be needed.
bool pack_waves(RdmPass& pa, bool full, int max_tri) {
    const int n = pa.npairs;
    struct Item {
        int kind;     // 3 cube, 1 one
        int bits[3];  // cube: a, b, c (pairs (a,b), (a,c), (b,c)); one: lp, lq
        int pairs[3]; // pair indices in slot order
        int swap[3];  // slot lists the pair's higher bit first
        int npair;
    };
    auto find = [&](int a, int b, const std::vector<bool>& used) {
        if (a > b) std::swap(a, b);
        for (int i = 0; i < n; ++i)
            if (!used[i] && pa.lp[i] == a && pa.lq[i] == b) return i;
        return -1;
    };
    std::vector<bool> used(n, false);
    std::vector<Item> tris, stars, ones;
    // the pairs of a cube item on bits (x, y, z): (x,y), (x,z) and, for a triangle, (y,z)
    auto cube_of = [&](int x, int y, int z, const std::vector<int>& members) {
        Item it{};
        it.kind = 3;
        it.bits[0] = x;
        it.bits[1] = y;
        it.bits[2] = z;
        const int pr[3][2] = {{x, y}, {x, z}, {y, z}};
        for (int k = 0; k < int(members.size()); ++k) {
            const int u = pr[k][0], v = pr[k][1];
            int found = -1;
            for (int m : members)
                if (pa.lp[m] == std::min(u, v) && pa.lq[m] == std::max(u, v)) found = m;
            it.pairs[it.npair] = found;
            it.swap[it.npair++] = u > v;
        }
        return it;
    };
    if (full) {
        for (int i = 0; i < n && int(tris.size()) < max_tri; ++i) {
            if (used[i]) continue;
            for (int r = 0; r < pa.T; ++r) {
                if (r == pa.lp[i] || r == pa.lq[i]) continue;
                const int j = find(pa.lp[i], r, used), k = find(pa.lq[i], r, used);
                if (j < 0 || k < 0 || j == i || k == i) continue;
                used[i] = used[j] = used[k] = true;
                tris.push_back(cube_of(pa.lp[i], pa.lq[i], r, {i, j, k}));
                break;
            }
        }
    }
    if (full) {
        for (int i = 0; i < n; ++i) {
            if (used[i]) continue;
            for (int j = i + 1; j < n; ++j) {
                if (used[j]) continue;
                const int a = pa.lp[i], b = pa.lq[i], c = pa.lp[j], d = pa.lq[j];
                const int shared = (a == c) + (a == d) + (b == c) + (b == d);
                if (shared != 1) continue;
                const int shared_bit = (a == c || a == d) ? a : b;
                const int u = shared_bit == a ? b : a, v = (c == shared_bit) ? d : c;
                used[i] = used[j] = true;
                stars.push_back(cube_of(shared_bit, u, v, {i, j}));
                break;
            }
        }
    }
    for (int i = 0; i < n; ++i)
        if (!used[i]) {
            Item it{};
            it.kind = 1;
            it.bits[0] = pa.lp[i];
            it.bits[1] = pa.lq[i];
            it.pairs[0] = i;
            it.npair = 1;
            ones.push_back(it);
        }
    struct Wave {
        int layout;
        std::vector<Item> items;
    };
    std::vector<Wave> waves;
    for (const Item& t : tris) waves.push_back({kLayTriOne, {t}});
    for (size_t i = 0; i + 1 < stars.size(); i += 2) waves.push_back({kLayCubeCube, {stars[i], stars[i + 1]}});
    if (stars.size() % 2) waves.push_back({kLayCubeOneOne, {stars.back()}});
    size_t next = 0;
    for (Wave& w : waves) {
        const size_t room = w.layout == kLayTriOne ? 1 : (w.layout == kLayCubeOneOne ? 2 : 0);
        for (size_t k = 0; k < room && next < ones.size(); ++k) w.items.push_back(ones[next++]);
    }
    while (next < ones.size()) {
        Wave w{kLayOnes, {}};
        for (int k = 0; k < 4 && next < ones.size(); ++k) w.items.push_back(ones[next++]);
        waves.push_back(w);
    }
    if (int(waves.size()) > kWaves) return false;
    // wave programs: (wave, piece, nsplit). Few waves are repeated with their bases split between
    // the copies; otherwise the heaviest waves are split in two while waves are idle. The programs
    // are then placed so that the two waves of each SIMD (waves w and w + 4) carry similar loads.
    const int W = int(waves.size());
    auto load_of = [](const Wave& w) {
        int l = 0;
        for (const Item& it : w.items) l += it.kind == 1 ? 16 : 16 * it.npair;  // quads per lane and tile
        return l;
    };
    struct Prog {
        int w, piece, nsplit;
        double load;
    };
    std::vector<Prog> progs;
    if (W > 0 && W <= kWaves / 2) {
        const int copies = kWaves / W;
        for (int c = 0; c < copies; ++c)
            for (int w = 0; w < W; ++w) progs.push_back({w, c, copies, double(load_of(waves[w])) / copies});
    } else {
        for (int w = 0; w < W; ++w) progs.push_back({w, 0, 1, double(load_of(waves[w]))});
        while (int(progs.size()) < kWaves) {
            int h = -1;
            for (int i = 0; i < int(progs.size()); ++i)
                if (progs[i].nsplit == 1 && (h < 0 || progs[i].load > progs[h].load)) h = i;
            if (h < 0) break;
            progs[h].nsplit = 2;
            progs[h].load /= 2;
            progs.push_back({progs[h].w, 1, 2, progs[h].load});
        }
    }
    std::stable_sort(progs.begin(), progs.end(), [](const Prog& x, const Prog& y) { return x.load > y.load; });
    constexpr int kSimds = 4;
    double simd_load[kSimds] = {0, 0, 0, 0};
    int simd_used[kSimds] = {0, 0, 0, 0};
    for (int w = 0; w < kWaves; ++w) {
        pa.layout[w] = kLayNone;
        pa.piece[w] = 0;
        pa.nsplit[w] = 1;
        for (int k = 0; k < 4; ++k) {
            pa.wpair[w][k] = -1;
            pa.wswap[w][k] = 0;
        }
    }
    for (const Prog& pr : progs) {
        int sm = -1;
        for (int q = 0; q < kSimds; ++q)
            if (simd_used[q] < kWaves / kSimds && (sm < 0 || simd_load[q] < simd_load[sm])) sm = q;
        const int dst = sm + kSimds * simd_used[sm]++;
        simd_load[sm] += pr.load;
        const Wave& src = waves[pr.w];
        pa.layout[dst] = src.layout;
        pa.piece[dst] = pr.piece;
        pa.nsplit[dst] = pr.nsplit;
        int slot = 0;
        for (size_t k = 0; k < src.items.size(); ++k) {
            const Item& it = src.items[k];
            for (int b = 0; b < 3; ++b) pa.ib[dst][k][b] = it.bits[b];
            // slots: a triangle takes 0-2 and its single 3; stars take 0-1 and 2-3
            if (src.layout == kLayTriOne && it.kind == 1) slot = 3;
            for (int m = 0; m < it.npair; ++m) {
                pa.wswap[dst][slot] = it.swap[m];
                pa.wpair[dst][slot++] = it.pairs[m];
            }
        }
    }
    return true;
}


// Single-site passes: the 4 low bits in every tile, the other bits in chunks of 8 (a short last
// chunk is filled up with bits evaluated before).
std::vector<Rdm1Pass> rdm1_plan(int L) {
    const int T = std::min(L, kTileBits);
    const int c = std::min(kRdmLowBits, T);
    const int W = T - c;
    std::vector<Rdm1Pass> passes;
    for (int first = c; first < L || passes.empty(); first += std::max(W, 1)) {
        Rdm1Pass pa{};
        pa.T = T;
        std::vector<bool> in(L, false), eval(L, false);
        for (int b = 0; b < c; ++b) {
            in[b] = true;
            eval[b] = passes.empty();
        }
        for (int b = first; b < std::min(L, first + W); ++b) in[b] = eval[b] = true;
        int cnt = 0;
        for (int b = 0; b < L; ++b) cnt += in[b];
        for (int b = c; b < L && cnt < T; ++b)
            if (!in[b]) {
                in[b] = true;
                ++cnt;
            }
        int i = 0;
        for (int b = 0; b < L; ++b)
            if (in[b]) {
                if (eval[b]) {
                    pa.lb[pa.nbits] = i;
                    pa.gb[pa.nbits++] = b;
                }
                pa.pos[i++] = b;
            } else {
                pa.comp[pa.ncomp++] = b;
            }
        passes.push_back(pa);
        if (W == 0) break;
    }
    return passes;
}

// Tile bit sets and the pairs each pass evaluates (every pair of bits).
std::vector<RdmPass> rdm_plan(int L) {
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
        int best = -1;  // the least loaded candidate: balanced passes
        for (int s : r.cand)
            if (best < 0 || members[s].size() < members[best].size()) best = s;
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
            for (int i = lo; i < hi; ++i) {
                const int p = mem[i].first, q = mem[i].second;
                pa.lp[i - lo] = local[p];
                pa.lq[i - lo] = local[q];
                pa.slot[i - lo] = pair_slot(L - q, L - p, L);
            }
            // as many triangles as still fit in the waves; pairs one by one always fit
            bool packed = false;
            for (int mt = kRdmMaxPairs / 3; mt >= 0 && !packed; --mt) packed = pack_waves(pa, T == kTileBits, mt);
            if (!packed) pack_waves(pa, false, 0);
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

extern "C" int ed_rdm_plan_pairs(int L, int* pairs, int max_pairs, int* pass_of) {
    if (L < 2 || L > 30) return -1;
    const std::vector<RdmPass> ps = rdm_plan(L);
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

extern "C" int ed_rdm_plan_sites(int L, int* bits, int max_bits, int* pass_of) {
    if (L < 2 || L > 30) return -1;
    const std::vector<Rdm1Pass> ps = rdm1_plan(L);
    int n = 0;
    for (int i = 0; i < int(ps.size()); ++i)
        for (int j = 0; j < ps[i].nbits; ++j) {
            if (n < max_bits && bits && pass_of) {
                bits[n] = ps[i].gb[j];
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
    const double2* p = reinterpret_cast<const double2*>(psi);
    if (!rho2) {
        static_assert(size_t(kRdmMaxBlocks) * kWaves * kTileBits * kRdm1Vals <= size_t(kRdmMaxPairs) * kRdmMaxBlocks * kRdmOff,
                      "single-site rows fit the pair accumulator area");
        for (const Rdm1Pass& pa : rdm1_plan(L)) {
            const int64_t ntiles = int64_t(1) << pa.ncomp;
            const int G = rdm_blocks(ntiles);
            if (pa.T == kTileBits) {
                hipLaunchKernelGGL(rdm1_pass<true>, dim3(G), dim3(kRdmThreads), 0, s, p, pa, ntiles, part);
            } else {
                hipLaunchKernelGGL(rdm1_pass<false>, dim3(G), dim3(kRdmThreads), 0, s, p, pa, ntiles, part);
            }
            ED_HIP_TRY(hipGetLastError());
            hipLaunchKernelGGL(rdm1_reduce, dim3(pa.nbits), dim3(256), 0, s, part, G * kWaves, pa, L,
                               reinterpret_cast<double2*>(rho1));
            ED_HIP_TRY(hipGetLastError());
        }
        return ED_OK;
    }
    const std::vector<RdmPass> passes = rdm_plan(L);
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
