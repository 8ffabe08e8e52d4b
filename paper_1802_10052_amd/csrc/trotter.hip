// Suzuki-Trotter time evolution (Sec. ed:sec:trotter: Eqs. ed:eq:trotter1, ed:eq:trotter2,
// ed:eq:trotter4, constants Eq. ed:eq:trotter4c).
//
// H = H_o + H_e with H_o the bond terms (k, k+1) for odd k (1-based sites) and H_e those for even
// k; each site's terms are shared by the bonds that contain it (1/2 each, 1 for a site in a single
// bond). A layer exp(-i t H_o) (or H_e) is the product of the commuting two-site propagators
// exp(-i t h_k); the paper contracts each with two legs of the rank-L state tensor (tensordot plus
// a permutation). Here a layer streams the state through LDS tiles in a few in-place passes (the
// 12 low bits, then windows of 8 high bits above 4 contiguous low bits, each starting at the first
// bond of the layer not yet covered): every gate of the layer is applied in the first pass whose
// tile holds both of its bits. Gates of one layer act on disjoint bits, so they commute and the order of the
// passes is free; a tile is read completely before it is written, and tiles of a pass are
// disjoint, so the passes work in place.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dense.h"
#include "ed_vec.h"
#include "krylov_core.h"

namespace ed {
namespace {

constexpr int kGThreads = 256;
constexpr int kGTileBits = 12;
constexpr int kGSlots = (1 << kGTileBits) / kGThreads;  // 16
constexpr int kGLow = 4;                                 // contiguous low bits of a window tile
constexpr int kMaxGates = kGTileBits / 2;                // gates of one parity inside a tile

// One pass of one layer: tile geometry and the gates it applies. A gate on tile-local bits
// (q, q+1) maps the local pair index l = 2 bit(q+1) + bit(q) (bit q+1 is the left site of the
// bond) by the 4x4 matrix U[l][m].
struct GatePass {
    int first;   // contiguous tile of the tbits low bits
    int c, h0;   // window tile: c low bits, window bits [h0, h0 + tbits - c)
    int tbits;   // tile bits (min(L, 12))
    int ngate;
    int q[kMaxGates];
    double2 U[kMaxGates][16];
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ int64_t gate_index(const GatePass& gp, int64_t n, int i) {
    if (gp.first) return (n << gp.tbits) + i;
    const int w = gp.tbits - gp.c;
    const int lo_bits = gp.h0 - gp.c;
    const int64_t nlo = n & ((int64_t(1) << lo_bits) - 1), nhi = n >> lo_bits;
    const int lowmask = (1 << gp.c) - 1;
    return (nlo << gp.c) | (nhi << (gp.h0 + w)) | int64_t(i & lowmask) | (int64_t(i >> gp.c) << gp.h0);
}

// Gate on register bits (8 + R, 9 + R): slots k, k | 1 << R, k | 2 << R, k | 3 << R hold the
// pair indices l = 0..3 of one group (compile-time slot indices keep v in registers).
template <int R>
__device__ __forceinline__ void reg_gate(double2 (&v)[kGSlots], const double2* __restrict__ U) {
#pragma unroll
    for (int k = 0; k < kGSlots; ++k) {
        if (((k >> R) & 3) != 0) continue;
        const double2 a[4] = {v[k], v[k | (1 << R)], v[k | (2 << R)], v[k | (3 << R)]};
        double2 o[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            double2 acc = make_double2(0.0, 0.0);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const double2 p = cmul(U[4 * l + m], a[m]);
                acc.x += p.x;
                acc.y += p.y;
            }
            o[l] = acc;
        }
        v[k] = o[0];
        v[k | (1 << R)] = o[1];
        v[k | (2 << R)] = o[2];
        v[k | (3 << R)] = o[3];
    }
}

// Tile-local index of slot k of thread t: i = t + kGThreads k (bits 0..7 across threads, 8..11
// across the 16 register slots). Gates whose two bits are both register bits are applied in
// registers while the tile is loaded; the others update groups of four amplitudes in LDS.
__global__ __launch_bounds__(kGThreads) void gate_pass(double2* __restrict__ psi, GatePass gp) {
    __shared__ double2 s[1 << kGTileBits];
    const int t = threadIdx.x;
    const int N = 1 << gp.tbits;
    const int64_t n = blockIdx.x;
    double2 v[kGSlots];
#pragma unroll
    for (int k = 0; k < kGSlots; ++k) {
        const int i = t + kGThreads * k;
        if (i < N) v[k] = psi[gate_index(gp, n, i)];
    }
    // register gates first (bits q, q+1 >= 8): the four amplitudes are slots of one thread
    for (int g = 0; g < gp.ngate; ++g) {
        const int q = gp.q[g];
        if (q < 8 || (1 << (q + 2)) > N) continue;
        switch (q - 8) {
            case 0: reg_gate<0>(v, gp.U[g]); break;
            case 1: reg_gate<1>(v, gp.U[g]); break;
            default: reg_gate<2>(v, gp.U[g]); break;
        }
    }
#pragma unroll
    for (int k = 0; k < kGSlots; ++k) {
        const int i = t + kGThreads * k;
        if (i < N) s[i] = v[k];
    }
    __syncthreads();
    // LDS gates (bit q is a thread bit): each thread owns whole groups of the amplitudes a gate
    // mixes (the index with zero bits inserted at q), reads them, writes them back. Two gates on
    // adjacent pairs (q, q+1), (q+2, q+3) share one round on groups of 16. Gates are sorted by q.
    for (int g = 0; g < gp.ngate; ++g) {
        const int q = gp.q[g];
        if (q >= 8 && (1 << (q + 2)) <= N) continue;  // done in registers
        const double2* U = gp.U[g];
        const bool two = g + 1 < gp.ngate && gp.q[g + 1] == q + 2 && !(q + 2 >= 8 && (1 << (q + 4)) <= N);
        if (two) {
            const double2* U2 = gp.U[g + 1];
            const int lowm = (1 << q) - 1;
            for (int j = t; j < (N >> 4); j += kGThreads) {
                const int b = (j & lowm) | ((j >> q) << (q + 4));
                double2 a[16];
#pragma unroll
                for (int m = 0; m < 16; ++m) a[m] = s[b | (m << q)];
                // first gate on the low pair (bits q, q+1) of every group of four
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    double2 o[4];
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            const double2 p = cmul(U[4 * l + m], a[4 * h + m]);
                            acc.x += p.x;
                            acc.y += p.y;
                        }
                        o[l] = acc;
                    }
#pragma unroll
                    for (int l = 0; l < 4; ++l) a[4 * h + l] = o[l];
                }
                // second gate on the high pair (bits q+2, q+3)
#pragma unroll
                for (int lo = 0; lo < 4; ++lo) {
                    double2 o[4];
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            const double2 p = cmul(U2[4 * l + m], a[4 * m + lo]);
                            acc.x += p.x;
                            acc.y += p.y;
                        }
                        o[l] = acc;
                    }
#pragma unroll
                    for (int l = 0; l < 4; ++l) a[4 * l + lo] = o[l];
                }
#pragma unroll
                for (int m = 0; m < 16; ++m) s[b | (m << q)] = a[m];
            }
            ++g;
        } else {
            const int lowm = (1 << q) - 1;
            for (int j = t; j < (N >> 2); j += kGThreads) {
                const int b = (j & lowm) | ((j >> q) << (q + 2));
                double2 a[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) a[m] = s[b | (m << q)];
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const double2 p = cmul(U[4 * l + m], a[m]);
                        acc.x += p.x;
                        acc.y += p.y;
                    }
                    s[b | (l << q)] = acc;
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kGSlots; ++k) {
        const int i = t + kGThreads * k;
        if (i < N) psi[gate_index(gp, n, i)] = s[i];
    }
}

// Tile geometries of the passes of one layer: the 12 low bits, then windows of 8 bits above 4
// contiguous low bits (256-byte runs), each starting at the lower bit of the first bond of the
// layer not yet covered (the layer's bonds are disjoint, so windows need not overlap). `lows`
// lists the lower bits of the layer's bonds in increasing order.
struct Geometry {
    int first, c, h0, tbits;
};

std::vector<Geometry> pass_geometry(int L, const std::vector<int>& lows) {
    std::vector<Geometry> g;
    const int T = std::min(L, kGTileBits);
    g.push_back({1, T, T, T});
    const int wb = kGTileBits - kGLow;
    for (int p : lows) {
        if (p + 1 < T) continue;
        const Geometry& last = g.back();
        const bool in_last = !last.first && p >= last.h0 && p + 1 < last.h0 + wb;
        if (in_last) continue;
        int h0 = p;
        if (h0 + wb > L) h0 = L - wb;
        g.push_back({0, kGLow, h0, kGTileBits});
    }
    return g;
}

// Global bit of tile-local bit q in a pass.
int global_bit(const Geometry& ge, int q) { return ge.first ? q : (q < ge.c ? q : ge.h0 + (q - ge.c)); }

// The two-site Hamiltonian of the bond on bits (p, p+1) (sites k = L-p-1 and k+1), 4x4 with
// index 2 bit(p+1) + bit(p): bond terms plus the shared site terms.
void bond_hamiltonian(const ed_model* m, int p, cplx* h) {
    const int L = m->L;
    auto weight = [&](int bit) {
        const int k = L - bit;  // site
        const int nb = (k > 1 ? 1 : 0) + (k < L ? 1 : 0);
        return 1.0 / nb;
    };
    for (int e = 0; e < 16; ++e) h[e] = cplx(m->bond[16 * p + e].x, m->bond[16 * p + e].y);
    const double wl = weight(p + 1), wr = weight(p);
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            const cplx sl(m->site[4 * (p + 1) + 2 * r + c].x, m->site[4 * (p + 1) + 2 * r + c].y);
            const cplx sr(m->site[4 * p + 2 * r + c].x, m->site[4 * p + 2 * r + c].y);
            for (int o = 0; o < 2; ++o) {
                h[4 * (2 * r + o) + (2 * c + o)] += wl * sl;  // site k (x) I
                h[4 * (2 * o + r) + (2 * o + c)] += wr * sr;  // I (x) site k+1
            }
        }
}

// Passes of one layer: the propagators exp(-i t h) of the bonds whose left site k has the given
// parity (1: odd k, H_o; 0: even k, H_e), each given to the first pass that holds both its bits.
std::vector<GatePass> build_layer(const ed_model* m, int parity, double t) {
    const int L = m->L;
    std::vector<int> lows;
    for (int p = 0; p + 1 < L; ++p)
        if (((L - p - 1) & 1) == parity) lows.push_back(p);
    const std::vector<Geometry> geo = pass_geometry(L, lows);
    std::vector<GatePass> passes(geo.size());
    for (size_t i = 0; i < geo.size(); ++i) {
        std::memset(&passes[i], 0, sizeof(GatePass));
        passes[i].first = geo[i].first;
        passes[i].c = geo[i].c;
        passes[i].h0 = geo[i].h0;
        passes[i].tbits = geo[i].tbits;
    }
    for (int p = 0; p + 1 < L; ++p) {
        const int k = L - p - 1;
        if ((k & 1) != parity) continue;
        cplx h[16], A[16], U[16];
        bool assigned = false;
        bond_hamiltonian(m, p, h);
        for (int e = 0; e < 16; ++e) A[e] = cplx(0.0, -t) * h[e];
        expm_complex(4, A, U);
        for (size_t i = 0; i < geo.size(); ++i) {
            int q = -1;
            for (int qq = 0; qq + 1 < geo[i].tbits; ++qq)
                if (global_bit(geo[i], qq) == p && global_bit(geo[i], qq + 1) == p + 1 && (geo[i].first || qq >= geo[i].c))
                    q = qq;
            if (q < 0) continue;
            GatePass& gp = passes[i];
            gp.q[gp.ngate] = q;
            for (int e = 0; e < 16; ++e) gp.U[gp.ngate][e] = make_double2(U[e].real(), U[e].imag());
            ++gp.ngate;
            assigned = true;
            break;
        }
        if (!assigned) return {};
    }
    // drop passes without gates
    std::vector<GatePass> out;
    for (const GatePass& gp : passes)
        if (gp.ngate > 0) out.push_back(gp);
    return out;
}

hipError_t run_layer(const std::vector<GatePass>& passes, double2* psi, int L, hipStream_t s) {
    for (const GatePass& gp : passes) {
        const int64_t tiles = int64_t(1) << (L - gp.tbits);
        hipLaunchKernelGGL(gate_pass, dim3(unsigned(tiles)), dim3(kGThreads), 0, s, psi, gp);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace
}  // namespace ed

extern "C" ed_status ed_trotter_workspace(const ed_model* model, int with_energy, size_t* bytes) {
    if (!model || !bytes) return ed::fail(ED_ERR_ARG, "null argument");
    const int64_t D = int64_t(1) << model->L;
    *bytes = ed::core_scratch_bytes() + (with_energy ? size_t(2) * size_t(D) * sizeof(double2) + 256 : 0);
    return ED_OK;
}

extern "C" ed_status ed_trotter_evolve(const ed_model* model, ed_c64* psi, double dt, int n_steps, int order,
                                       const ed_observe* obs, void* ws, size_t ws_bytes, void* stream) {
    using namespace ed;
    if (!model || !psi) return fail(ED_ERR_ARG, "null argument");
    if (order != 2 && order != 4) return fail(ED_ERR_ARG, "order must be 2 or 4");
    if (model->lr || model->lv_L > 0) return fail(ED_ERR_UNSUPPORTED, "the Trotter layers take site and bond rules only");
    if (n_steps < 0) return fail(ED_ERR_ARG, "n_steps must be >= 0");
    if (!std::isfinite(dt)) return fail(ED_ERR_ARG, "dt must be finite");
    const bool want_e = obs && obs->energy;
    size_t need = 0;
    ED_TRY(ed_trotter_workspace(model, want_e ? 1 : 0, &need));
    if (!ws) return fail(ED_ERR_ARG, "workspace is null");
    if (ws_bytes < need) return fail(ED_ERR_WORKSPACE, "workspace too small (energy needs with_energy = 1)");
    const int L = model->L;
    const int64_t D = int64_t(1) << L;
    Workspace w;
    ED_TRY(carve(ws, ws_bytes, D, want_e ? 2 : 0, &w));
    hipStream_t s = static_cast<hipStream_t>(stream);
    double2* v = reinterpret_cast<double2*>(psi);

    // layer sequence (part, fraction of dt): Eq. ed:eq:trotter2 or Eq. ed:eq:trotter4 with the
    // constants of Eq. ed:eq:trotter4c; part 0 = H_e (even k), 1 = H_o (odd k)
    const double tau3 = 1.0 / (2.0 * (4.0 - std::cbrt(4.0)));
    const double tau1 = 1.0 - 8.0 * tau3, tau2 = 0.5 * (1.0 - 6.0 * tau3), tau4 = 2.0 * tau3;
    std::vector<std::pair<int, double>> seq;
    if (order == 2) {
        seq = {{0, 0.5}, {1, 1.0}, {0, 0.5}};
    } else {
        seq = {{0, tau3}, {1, tau4}, {0, tau4}, {1, tau4}, {0, tau2}, {1, tau1},
               {0, tau2}, {1, tau4}, {0, tau4}, {1, tau4}, {0, tau3}};
    }
    // one set of passes per distinct (part, fraction)
    std::vector<std::pair<int, double>> keys;
    std::vector<std::vector<GatePass>> layers;
    std::vector<int> which(seq.size());
    for (size_t i = 0; i < seq.size(); ++i) {
        int found = -1;
        for (size_t j = 0; j < keys.size(); ++j)
            if (keys[j] == seq[i]) found = int(j);
        if (found < 0) {
            keys.push_back(seq[i]);
            layers.push_back(build_layer(model, seq[i].first, seq[i].second * dt));
            if (layers.back().empty() && L > 2 - seq[i].first)
                return fail(ED_ERR_UNSUPPORTED, "internal error: a Trotter gate has no pass for L = " + std::to_string(L));
            found = int(keys.size()) - 1;
        }
        which[i] = found;
    }
    auto record = [&](int step) -> ed_status {
        if (obs && (obs->sz || obs->norm)) {
            double nrm = 0.0;
            ED_TRY(measure_state(v, L, w, obs->sz ? obs->sz + size_t(step) * L : nullptr, &nrm, s));
            if (obs->norm) obs->norm[step] = nrm;
        }
        if (want_e) {
            double e = 0.0;
            ED_TRY(energy_of(model, w, v, &e, s));
            obs->energy[step] = e;
        }
        return ED_OK;
    };
    ED_TRY(record(0));
    for (int st = 0; st < n_steps; ++st) {
        for (size_t i = 0; i < seq.size(); ++i) {
            const hipError_t e = run_layer(layers[which[i]], v, L, s);
            if (e != hipSuccess) return fail(ED_ERR_HIP, std::string("Trotter layer launch: ") + hipGetErrorString(e));
        }
        ED_TRY(record(st + 1));
    }
    ED_HIP_TRY(hipStreamSynchronize(s));
    return ED_OK;
}
