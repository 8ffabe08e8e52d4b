// out = H psi for a site + bond rule set on a dense complex128 state (Sec. ed:sec:krylov: the rule set
// applied to the state without storing H, cost L(2 n_b + n_s) O(d^(L+1)), Eq. ed:eq:OKrylov).
//
// The paper contracts each rule with the rank-L tensor (tensordot + permutation per rule and
// site). Here the state streams through HBM in a few passes. Each pass stages a 2^12-amplitude
// tile in LDS; the tile spans either the 12 low bits (first pass: it also adds the diagonal of
// every term) or c low bits (runs of 2^c amplitudes, c = 3 or 4) times a window of 12 - c high
// bits (later passes, which accumulate into out). Every site and off-diagonal bond term is
// assigned to exactly one pass, so a term whose bits both lie in the tile is evaluated entirely on
// chip: the partner amplitude psi[x ^ flip] comes from LDS, or from the thread's own registers
// when the flipped bits map to the register dimension of the tile. Terms on the few "gathered"
// bits just above a tile read the partner amplitude from the neighbouring tile, which the
// workgroups of the same group stream through the same L2 at the same time.
#include "hpsi_device.h"

namespace ed {
namespace {

// Small-L kernel: one thread per output amplitude, partners read from global memory (the whole
// state is cache resident for L < 12).
template <unsigned CLS>
__global__ __launch_bounds__(256) void hpsi_small(const double2* __restrict__ psi,
                                                  double2* __restrict__ out,
                                                  const double2* __restrict__ site,
                                                  const double2* __restrict__ bond, int L,
                                                  const double2* __restrict__ lr_full) {
    const int64_t D = int64_t(1) << L;
    const int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (x >= D) return;
    double2 y = small_entry<CLS>(psi, site, bond, L, x);
    if (lr_full) {  // long-range zz energy of basis state x
        const double2 e = lr_full[x], v = psi[x];
        y.x += e.x * v.x - e.y * v.y;
        y.y += e.x * v.y + e.y * v.x;
    }
    out[x] = y;
}

// Gathered jobs whose partners a wide tile loads ahead, per round (two rounds). A wide tile holds 4
// amplitudes per thread, so a job costs 16 registers: 4 jobs fit the 128 registers of a
// 1024-thread workgroup with a real diagonal, 3 with a complex one.
template <unsigned CLS>
constexpr int wide_prefetch() { return (CLS & kDiagReal) ? 4 : 3; }

// One tile per workgroup. With gathered bits, consecutive workgroups of one XCD (workgroups are
// dealt to the 8 XCDs round-robin) take the 2^G tiles that differ only in the gathered bits, so
// the neighbouring tiles a workgroup reads are being streamed into the same L2 at the same time.
// DOT: the last pass of a product, also leaving each tile's projection on the input in
// pa.dot_part (window passes only).
template <unsigned CLS, bool FIRST, bool GATHER, bool DOT = false>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(2)))
void hpsi_tile(const double2* __restrict__ psi, double2* __restrict__ out, const double2* __restrict__ site,
               const double2* __restrict__ bond, const double2* __restrict__ dlo, const double2* __restrict__ dmid,
               const double2* __restrict__ dhi, PassArgs pa) {
    __shared__ double2 s[1 << kTileBits];
    __shared__ double2 sF[kTileBits];
    __shared__ double2 sD[kTileThreads / 64];
    int64_t n = blockIdx.x;
    if (GATHER) {
        const int64_t b = blockIdx.x;
        const int64_t xcd = b & 7, j = b >> 3;
        const int64_t member = j & ((int64_t(1) << pa.G) - 1), gl = j >> pa.G;
        const int64_t group = (gl << 3) | xcd;
        const int64_t low = group & ((int64_t(1) << pa.gpos) - 1), high = group >> pa.gpos;
        n = low | (member << pa.gpos) | (high << (pa.gpos + pa.G));
    }
    tile_body<CLS, FIRST, GATHER, false, 8, DOT>(psi, out, site, bond, dlo, dmid, dhi, pa, n, s, 0, nullptr, sF, sD);
}

// One tile per 1024-thread workgroup (4 registers per thread), launched with LDS padding so
// that one workgroup runs per CU: the tiles in flight on an XCD (32) are one gather group of
// G = 5, whose neighbouring tiles then stay in its L2, and 16 waves per CU keep loads, LDS work
// and stores overlapping. Blocks map to tiles like the 256-thread launch.
template <unsigned CLS, bool FIRST, bool DOT = false>
__global__ __launch_bounds__(kTileThreads * 4) void hpsi_tile_wide(
    const double2* __restrict__ psi, double2* __restrict__ out, const double2* __restrict__ site,
    const double2* __restrict__ bond, const double2* __restrict__ dlo, const double2* __restrict__ dmid,
    const double2* __restrict__ dhi, PassArgs pa) {
    __shared__ double2 s[1 << kTileBits];
    __shared__ double2 sF[kTileBits];
    __shared__ double2 sD[kTileThreads * 4 / 64];
    const int64_t b = blockIdx.x;
    const int64_t xcd = b & 7, j = b >> 3;
    const int64_t member = j & ((int64_t(1) << pa.G) - 1), gl = j >> pa.G;
    const int64_t group = (gl << 3) | xcd;
    const int64_t low = group & ((int64_t(1) << pa.gpos) - 1), high = group >> pa.gpos;
    const int64_t n = low | (member << pa.gpos) | (high << (pa.gpos + pa.G));
    tile_body<CLS, FIRST, true, false, 10, DOT, wide_prefetch<CLS>()>(psi, out, site, bond, dlo, dmid, dhi, pa, n,
                                                                      s, 0, nullptr, sF, sD);
}

// The window passes of a wide plan: one tile per 512-thread workgroup (8 amplitudes per thread)
// without LDS padding, so that two workgroups share a CU and one's loads overlap the other's LDS
// work. Their gather groups are small (the plan's few window gathers), so twice the tiles in
// flight still fit an XCD's L2; one gathered job's partners (32 registers) are loaded ahead.
// Blocks map to tiles like the one-tile launches.
template <unsigned CLS, bool DOT = false>
__global__ __launch_bounds__(kTileThreads * 2) void hpsi_tile_mid(
    const double2* __restrict__ psi, double2* __restrict__ out, const double2* __restrict__ site,
    const double2* __restrict__ bond, const double2* __restrict__ dlo, const double2* __restrict__ dmid,
    const double2* __restrict__ dhi, PassArgs pa) {
    __shared__ double2 s[1 << kTileBits];
    __shared__ double2 sF[kTileBits];
    __shared__ double2 sD[kTileThreads * 2 / 64];
    const int64_t b = blockIdx.x;
    const int64_t xcd = b & 7, j = b >> 3;
    const int64_t member = j & ((int64_t(1) << pa.G) - 1), gl = j >> pa.G;
    const int64_t group = (gl << 3) | xcd;
    const int64_t low = group & ((int64_t(1) << pa.gpos) - 1), high = group >> pa.gpos;
    const int64_t n = low | (member << pa.gpos) | (high << (pa.gpos + pa.G));
    tile_body<CLS, false, true, false, 9, DOT, 1>(psi, out, site, bond, dlo, dmid, dhi, pa, n, s, 0, nullptr, sF, sD);
}

// Two tiles per workgroup (512 threads, 128 KiB of LDS, one workgroup per CU): the tiles n and
// n ^ (tile-index bit gpos) that differ in the first gathered bit, one per half. Block b is mapped
// like the one-tile launch, with pairs in place of tiles, so a gather group's pairs still run
// back to back on one XCD.
template <unsigned CLS, bool FIRST, bool DOT = false>
__global__ __launch_bounds__(2 * kTileThreads) __attribute__((amdgpu_waves_per_eu(2)))
void hpsi_tile_pair(const double2* __restrict__ psi, double2* __restrict__ out, const double2* __restrict__ site,
                    const double2* __restrict__ bond, const double2* __restrict__ dlo,
                    const double2* __restrict__ dmid, const double2* __restrict__ dhi, PassArgs pa) {
    __shared__ double2 s[2][1 << kTileBits];
    __shared__ double2 sF[2][kTileBits];
    __shared__ double2 sD[2][kTileThreads / 64];
    const int h = int(threadIdx.x) / kTileThreads, t = int(threadIdx.x) % kTileThreads;
    const int64_t b = blockIdx.x;
    const int64_t xcd = b & 7, j = b >> 3;
    const int gp = pa.G - 1;  // gathered bits besides the paired one
    const int64_t member = j & ((int64_t(1) << gp) - 1), gl = j >> gp;
    const int64_t group = (gl << 3) | xcd;
    const int64_t low = group & ((int64_t(1) << pa.gpos) - 1), high = group >> pa.gpos;
    const int64_t n = low | (int64_t(h) << pa.gpos) | (member << (pa.gpos + 1)) | (high << (pa.gpos + pa.G));
    tile_body<CLS, FIRST, true, true, 8, DOT>(psi, out, site, bond, dlo, dmid, dhi, pa, n, s[h], t, s[h ^ 1], sF[h], sD[h]);
}

// dot_part: the last pass (a window pass) also writes each tile's sum of conj(psi) out
template <unsigned CLS>
hipError_t launch_variant(const ed_model* m, const double2* psi, double2* out, hipStream_t s, double2* dot_part) {
    const int L = m->L;
    if (L < kTileBits) {
        const int64_t D = int64_t(1) << L;
        const int threads = 256;
        const int blocks = int((D + threads - 1) / threads);
        hipLaunchKernelGGL((hpsi_small<CLS>), dim3(blocks), dim3(threads), 0, s, psi, out,
                           m->d_site, m->d_bond, L, m->lr ? m->d_lr_low : nullptr);
        return hipGetLastError();
    }
    const int64_t tiles = int64_t(1) << (L - kTileBits);
    for (int ip = 0; ip < m->n_pass; ++ip) {
        const PassDesc& pd = m->pass[ip];
        PassArgs pa = to_args(pd, m->d_jobs + (size_t(m->plan) * kMaxPasses + ip) * kMaxJobs,
                              m->njobs[m->plan][ip]);
        if (pd.first && m->lr) {
            pa.lr = 1;
            pa.L = L;
            pa.lr_low = m->d_lr_low;
            pa.lr_cross = m->d_lr_cross;
        }
        const dim3 grid{unsigned(tiles)}, block{unsigned(kTileThreads)};
        const bool dot = dot_part && !pd.first && ip == m->n_pass - 1;
        pa.dot_part = dot ? dot_part : nullptr;
#define ED_TILE_ARGS psi, out, m->d_site, m->d_bond, m->d_diag_lo, m->d_diag_mid, m->d_diag_hi, pa
        // optional LDS padding: one workgroup per CU, so that the tiles of a group fit in L2
        const unsigned pad = (pd.G > 0 && pd.occ1) ? unsigned(kOccPadBytes) : 0u;
        if (pd.G > 0 && pd.wide) {
            const dim3 wblock{unsigned(4 * kTileThreads)};
            const dim3 mblock{unsigned(2 * kTileThreads)};
            if (pd.first) hipLaunchKernelGGL((hpsi_tile_wide<CLS, true>), grid, wblock, kOccPadBytes, s, ED_TILE_ARGS);
            else if (dot) hipLaunchKernelGGL((hpsi_tile_mid<CLS, true>), grid, mblock, 0, s, ED_TILE_ARGS);
            else hipLaunchKernelGGL((hpsi_tile_mid<CLS, false>), grid, mblock, 0, s, ED_TILE_ARGS);
        } else if (pd.G > 0 && pd.pair) {
            const dim3 pgrid{unsigned(tiles / 2)}, pblock{unsigned(2 * kTileThreads)};
            if (pd.first) hipLaunchKernelGGL((hpsi_tile_pair<CLS, true>), pgrid, pblock, 0, s, ED_TILE_ARGS);
            else if (dot) hipLaunchKernelGGL((hpsi_tile_pair<CLS, false, true>), pgrid, pblock, 0, s, ED_TILE_ARGS);
            else hipLaunchKernelGGL((hpsi_tile_pair<CLS, false>), pgrid, pblock, 0, s, ED_TILE_ARGS);
        } else if (pd.first) {
            if (pd.G > 0) hipLaunchKernelGGL((hpsi_tile<CLS, true, true>), grid, block, pad, s, ED_TILE_ARGS);
            else hipLaunchKernelGGL((hpsi_tile<CLS, true, false>), grid, block, 0, s, ED_TILE_ARGS);
        } else if (dot) {
            if (pd.G > 0) hipLaunchKernelGGL((hpsi_tile<CLS, false, true, true>), grid, block, pad, s, ED_TILE_ARGS);
            else hipLaunchKernelGGL((hpsi_tile<CLS, false, false, true>), grid, block, 0, s, ED_TILE_ARGS);
        } else {
            if (pd.G > 0) hipLaunchKernelGGL((hpsi_tile<CLS, false, true>), grid, block, pad, s, ED_TILE_ARGS);
            else hipLaunchKernelGGL((hpsi_tile<CLS, false, false>), grid, block, 0, s, ED_TILE_ARGS);
        }
#undef ED_TILE_ARGS
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int I>
hipError_t dispatch(const ed_model* m, const double2* psi, double2* out, hipStream_t s, double2* dot_part) {
    if constexpr (I >= kNumVariants) {
        return hipErrorInvalidValue;
    } else {
        if (variant_fits(kVariants[I], m->op_class)) return launch_variant<kVariants[I]>(m, psi, out, s, dot_part);
        return dispatch<I + 1>(m, psi, out, s, dot_part);
    }
}

}  // namespace

ed_status launch_apply_H(const ed_model* m, const double2* psi, double2* out, hipStream_t s) {
    hipError_t e = dispatch<0>(m, psi, out, s, nullptr);
    if (e != hipSuccess) return fail(ED_ERR_HIP, std::string("apply_H launch: ") + hipGetErrorString(e));
    if (!m->far.empty()) return launch_far_terms(m, psi, out, s);
    return ED_OK;
}

ed_status launch_apply_H_dot(const ed_model* m, const double2* psi, double2* out, double2* dot_part,
                             int64_t max_parts, int64_t* nparts, hipStream_t s) {
    *nparts = 0;
    const bool fusable = m->L >= kTileBits && m->far.empty() && m->n_pass > 0 && !m->pass[m->n_pass - 1].first &&
                         (int64_t(1) << (m->L - kTileBits)) <= max_parts;
    if (!fusable) return launch_apply_H(m, psi, out, s);
    hipError_t e = dispatch<0>(m, psi, out, s, dot_part);
    if (e != hipSuccess) return fail(ED_ERR_HIP, std::string("apply_H launch: ") + hipGetErrorString(e));
    *nparts = int64_t(1) << (m->L - kTileBits);
    return ED_OK;
}

}  // namespace ed
