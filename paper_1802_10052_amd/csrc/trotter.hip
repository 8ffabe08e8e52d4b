// Suzuki-Trotter time evolution (Sec. ed:sec:trotter: Eqs. ed:eq:trotter1, ed:eq:trotter2,
// ed:eq:trotter4, constants Eq. ed:eq:trotter4c).
//
// H = H_o + H_e with H_o the bond terms (k, k+1) for odd k (1-based sites) and H_e those for even
// k; each site's terms are shared by the bonds that contain it (1/2 each, 1 for a site in a single
// bond). A layer exp(-i t H_o) (or H_e) is the product of the commuting two-site propagators
// exp(-i t h_k); the paper contracts each with two legs of the rank-L state tensor (tensordot plus
// a permutation). Here runs of kFuse consecutive layers stream the state through LDS tiles in a
// few in-place passes (the 12 low bits, then windows of 8 high bits above 4 contiguous low bits):
// a pass applies its gates layer by layer, and each gate goes to the first pass whose tile holds
// both of its bits and in which every gate of an earlier layer that shares one of its bits has
// already been applied (in an earlier pass, or earlier in the same pass). Gates of one layer act
// on disjoint bits and commute, so this keeps the order of the product wherever it matters; a
// tile is read completely before it is written, and tiles of a pass are disjoint, so the passes
// work in place.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dense.h"
#include "ed_vec.h"
#include "krylov_core.h"

namespace ed {
namespace {

// 512 threads per 4096-amplitude tile (measured against 256 and 1024), one gate per LDS round:
// rounds that apply two gates of a layer on adjacent pairs to groups of 16 (kPairRounds) leave
// half of 512 threads idle and were slower
constexpr int kGThreads = 512;
constexpr int kGThreadBits = kGThreads == 256 ? 8 : kGThreads == 512 ? 9 : 10;
constexpr int kGTileBits = 12;
constexpr int kGSlots = (1 << kGTileBits) / kGThreads;  // amplitudes per thread
constexpr int kGSlotBits = kGTileBits - kGThreadBits;
constexpr bool kPairRounds = false;
constexpr int kGLow = 4;                                 // contiguous low bits of a window tile
constexpr int kFuse = 4;                                 // consecutive layers per run of passes
constexpr int kMaxGates = kFuse * (kGTileBits / 2);      // gates of one pass
constexpr int kTableGates = 192;                         // gates one evolve call holds
// the gate table: 16 double2 (the matrix) per gate, then 2 ints (q, layer) per gate
constexpr size_t kGateTableBytes = size_t(kTableGates) * (16 * sizeof(double2) + 2 * sizeof(int));

// One pass: tile geometry and the gates it applies, sorted by (layer, q), in device memory: gate g
// of the pass acts on tile-local bits (q, q+1) = (G[2 g], G[2 g] + 1) for the layer G[2 g + 1] of
// the run, and maps the local pair index l = 2 bit(q+1) + bit(q) (bit q+1 is the left site of the
// bond) by the 4x4 matrix U[16 g + 4 l + m].
struct GatePass {
    int first;   // contiguous tile of the tbits low bits
    int c, h0;   // window tile: c low bits, window bits [h0, h0 + tbits - c)
    int tbits;   // tile bits (min(L, 12))
    int ngate;
    const double2* U;
    const int* G;
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

// Gate on register bits (kGThreadBits + R, kGThreadBits + R + 1): slots k, k | 1 << R, k | 2 << R,
// k | 3 << R hold the pair indices l = 0..3 of one group (compile-time slot indices keep v in
// registers).
template <int R>
__device__ __forceinline__ void reg_gate(double2 (&v)[kGSlots], const double2* __restrict__ U) {
    static_assert(R + 2 <= kGSlotBits, "gate bits beyond the register slots");
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

// A gate of the first layer whose two bits are register bits of an N-amplitude tile.
__device__ __forceinline__ bool in_regs(int layer, int q, int N) {
    return layer == 0 && q >= kGThreadBits && (1 << (q + 2)) <= N;
}

// Tile-local index of slot k of thread t: i = t + kGThreads k (the low kGThreadBits bits across
// threads, the rest across the register slots). Gates of the first layer whose two bits are both
// register bits are applied in registers while the tile is loaded; the others update groups of
// four amplitudes in LDS.
__global__ __launch_bounds__(kGThreads) void gate_pass(double2* __restrict__ psi, GatePass gp,
                                                       const double2* __restrict__ Utab,
                                                       const int* __restrict__ G) {
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
    // the first layer's gates on register bits (q, q+1 >= 8) first: the four amplitudes are slots
    // of one thread (they commute with the rest of that layer)
    // (a switch in the kernel body: written as a chain of ifs, or inside a helper taking the slots
    // by reference, the slots went to scratch memory)
    for (int g = 0; g < gp.ngate; ++g) {
        if (!in_regs(G[2 * g + 1], G[2 * g], N)) continue;
        const double2* U = Utab + 16 * g;
        switch (G[2 * g] - kGThreadBits) {
            case 0: reg_gate<0>(v, U); break;
            case 1:
                if constexpr (kGSlotBits >= 3) reg_gate<1>(v, U);
                break;
            default:
                if constexpr (kGSlotBits >= 4) reg_gate<2>(v, U);
                break;
        }
    }
#pragma unroll
    for (int k = 0; k < kGSlots; ++k) {
        const int i = t + kGThreads * k;
        if (i < N) s[i] = v[k];
    }
    __syncthreads();
    // LDS gates, in list order: each thread owns whole groups of the amplitudes a gate mixes (the
    // index with zero bits inserted at q), reads them, writes them back. With kPairRounds, two
    // gates of one layer on adjacent pairs (q, q+1), (q+2, q+3) share one round on groups of 16.
    for (int g = 0; g < gp.ngate; ++g) {
        const int q = G[2 * g], layer = G[2 * g + 1];
        if (in_regs(layer, q, N)) continue;  // done in registers
        const double2* U = Utab + 16 * g;
        const bool two = kPairRounds && g + 1 < gp.ngate && G[2 * g + 3] == layer && G[2 * g + 2] == q + 2 &&
                         !in_regs(layer, q + 2, N);
        if (two) {
            const double2* U2 = Utab + 16 * (g + 1);
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

struct Geometry {
    int first, c, h0, tbits;
};

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

// Passes of a run of consecutive layers (part, time): layer l holds the propagators exp(-i t_l h)
// of the bonds whose left site k has the layer's parity (1: odd k, H_o; 0: even k, H_e). The first
// pass is the contiguous tile of the 12 low bits; each later pass is a window of 8 bits above 4
// contiguous low bits, starting at the lowest bond still pending. A gate (l, p) on bits (p, p+1)
// is ready once every gate of an earlier layer on bonds p - 1, p, p + 1 has a pass; going through
// the layers in order, each pass takes the ready gates its tile holds. The matrices go to
// table and the (q, layer) pairs to meta (host copies); the passes point at dev_table and
// dev_meta. Returns false when a gate finds no pass or the table is full.
bool build_run(const ed_model* m, const std::vector<std::pair<int, double>>& run, double dt,
               std::vector<double2>* table, std::vector<int>* meta, const double2* dev_table,
               const int* dev_meta, std::vector<GatePass>* out) {
    const int L = m->L;
    const int F = int(run.size());
    const int T = std::min(L, kGTileBits);
    const int wb = kGTileBits - kGLow;
    auto is_bond = [&](int l, int p) { return p >= 0 && p + 1 < L && ((L - p - 1) & 1) == run[l].first; };
    std::vector<std::vector<int>> at(F, std::vector<int>(L, -1));  // pass of gate (l, p)
    int pending = 0;
    for (int l = 0; l < F; ++l)
        for (int p = 0; p + 1 < L; ++p) pending += is_bond(l, p);
    auto ready = [&](int l, int p) {
        for (int e = 0; e < l; ++e)
            for (int d = -1; d <= 1; ++d)
                if (is_bond(e, p + d) && at[e][p + d] < 0) return false;
        return true;
    };
    std::vector<Geometry> geo;
    std::vector<std::vector<std::pair<int, int>>> gates;  // (layer, p) of each pass, by layer then p
    auto fill = [&](const Geometry& ge, int lo, int hi) {  // gates with both bits in [lo, hi)
        const int pass = int(geo.size());
        std::vector<std::pair<int, int>> gs;
        for (int l = 0; l < F; ++l)
            for (int p = lo; p + 1 < hi; ++p)
                if (is_bond(l, p) && at[l][p] < 0 && ready(l, p)) {
                    at[l][p] = pass;
                    gs.push_back({l, p});
                    --pending;
                }
        geo.push_back(ge);
        gates.push_back(gs);
        return !gs.empty();
    };
    fill({1, T, T, T}, 0, T);
    while (pending > 0) {
        int h0 = L;
        for (int l = 0; l < F; ++l)
            for (int p = 0; p + 1 < L; ++p)
                if (is_bond(l, p) && at[l][p] < 0) h0 = std::min(h0, p);
        h0 = std::min(h0, L - wb);
        if (h0 < kGLow) return false;
        if (!fill({0, kGLow, h0, kGTileBits}, h0, h0 + wb)) return false;
    }
    for (size_t i = 0; i < geo.size(); ++i) {
        if (gates[i].empty()) continue;
        if (int(gates[i].size()) > kMaxGates) return false;
        if (table->size() / 16 + gates[i].size() > size_t(kTableGates)) return false;
        GatePass gp;
        std::memset(&gp, 0, sizeof(GatePass));
        gp.first = geo[i].first;
        gp.c = geo[i].c;
        gp.h0 = geo[i].h0;
        gp.tbits = geo[i].tbits;
        gp.U = dev_table ? dev_table + table->size() : nullptr;  // null when only counting passes
        gp.G = dev_meta ? dev_meta + meta->size() : nullptr;
        for (const auto& lp : gates[i]) {
            const int l = lp.first, p = lp.second;
            const int q = geo[i].first ? p : geo[i].c + (p - geo[i].h0);
            if (global_bit(geo[i], q) != p || global_bit(geo[i], q + 1) != p + 1) return false;
            cplx h[16], A[16], U[16];
            bond_hamiltonian(m, p, h);
            for (int e = 0; e < 16; ++e) A[e] = cplx(0.0, -run[l].second * dt) * h[e];
            expm_complex(4, A, U);
            for (int e = 0; e < 16; ++e) table->push_back(make_double2(U[e].real(), U[e].imag()));
            meta->push_back(q);
            meta->push_back(l);
            ++gp.ngate;
        }
        out->push_back(gp);
    }
    return true;
}

hipError_t run_passes(const std::vector<GatePass>& passes, double2* psi, int L, hipStream_t s) {
    for (const GatePass& gp : passes) {
        const int64_t tiles = int64_t(1) << (L - gp.tbits);
        hipLaunchKernelGGL(gate_pass, dim3(unsigned(tiles)), dim3(kGThreads), 0, s, psi, gp, gp.U, gp.G);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The layers of one step (part, fraction of dt): Eq. ed:eq:trotter2 or Eq. ed:eq:trotter4 with
// the constants of Eq. ed:eq:trotter4c; part 0 = H_e (even k), 1 = H_o (odd k).
std::vector<std::pair<int, double>> step_layers(int order) {
    const double tau3 = 1.0 / (2.0 * (4.0 - std::cbrt(4.0)));
    const double tau1 = 1.0 - 8.0 * tau3, tau2 = 0.5 * (1.0 - 6.0 * tau3), tau4 = 2.0 * tau3;
    if (order == 2) return {{0, 0.5}, {1, 1.0}, {0, 0.5}};
    return {{0, tau3}, {1, tau4}, {0, tau4}, {1, tau4}, {0, tau2}, {1, tau1},
            {0, tau2}, {1, tau4}, {0, tau4}, {1, tau4}, {0, tau3}};
}

// The passes of one step: the step's layers in runs of kFuse, one set of passes per distinct run
// (runs), the run of each position (which); the gate matrices go to table and their (q, layer)
// to meta, the passes point at dev_table and dev_meta.
struct StepPlan {
    std::vector<std::vector<GatePass>> runs;
    std::vector<int> which;
    std::vector<double2> table;
    std::vector<int> meta;
};

ed_status plan_step(const ed_model* m, int order, double dt, const double2* dev_table, const int* dev_meta,
                    StepPlan* sp) {
    const std::vector<std::pair<int, double>> seq = step_layers(order);
    std::vector<std::vector<std::pair<int, double>>> keys;
    for (size_t i0 = 0; i0 < seq.size(); i0 += kFuse) {
        const std::vector<std::pair<int, double>> run(seq.begin() + i0, seq.begin() + std::min(seq.size(), i0 + kFuse));
        int found = -1;
        for (size_t j = 0; j < keys.size(); ++j)
            if (keys[j] == run) found = int(j);
        if (found < 0) {
            std::vector<GatePass> passes;
            if (!build_run(m, run, dt, &sp->table, &sp->meta, dev_table, dev_meta, &passes))
                return fail(ED_ERR_UNSUPPORTED, "internal error: no Trotter pass plan for L = " + std::to_string(m->L));
            keys.push_back(run);
            sp->runs.push_back(passes);
            found = int(keys.size()) - 1;
        }
        sp->which.push_back(found);
    }
    return ED_OK;
}

}  // namespace
}  // namespace ed

extern "C" ed_status ed_trotter_workspace(const ed_model* model, int with_energy, size_t* bytes) {
    if (!model || !bytes) return ed::fail(ED_ERR_ARG, "null argument");
    const int64_t D = int64_t(1) << model->L;
    // the scratch of the norm and energy kernels, two state vectors for the energy, the gate table
    *bytes = ed::core_scratch_bytes() + (with_energy ? size_t(2) * size_t(D) * sizeof(double2) + 256 : 0) +
             ed::kGateTableBytes;
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
    ObsStage stage;
    obs = stage.begin(obs, n_steps, L);

    // the step's passes; their gate matrices in the table at the end of the workspace
    const size_t vec_bytes = want_e ? (size_t(2) * size_t(D) * sizeof(double2) + 255) & ~size_t(255) : 0;
    const size_t table_off = core_scratch_bytes() + vec_bytes;  // after what carve hands out
    if (table_off + kGateTableBytes > ws_bytes) return fail(ED_ERR_WORKSPACE, "workspace too small for the gate table");
    char* const tab = static_cast<char*>(ws) + table_off;
    double2* const dev_table = reinterpret_cast<double2*>(tab);
    int* const dev_meta = reinterpret_cast<int*>(tab + size_t(kTableGates) * 16 * sizeof(double2));
    StepPlan sp;
    ED_TRY(plan_step(model, order, dt, dev_table, dev_meta, &sp));
    if (!sp.table.empty()) {
        ED_HIP_TRY(hipMemcpyAsync(dev_table, sp.table.data(), sp.table.size() * sizeof(double2),
                                  hipMemcpyHostToDevice, s));
        ED_HIP_TRY(hipMemcpyAsync(dev_meta, sp.meta.data(), sp.meta.size() * sizeof(int), hipMemcpyHostToDevice, s));
        ED_HIP_TRY(hipStreamSynchronize(s));  // the host tables are locals
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
        for (int r : sp.which) {
            const hipError_t e = run_passes(sp.runs[r], v, L, s);
            if (e != hipSuccess) return fail(ED_ERR_HIP, std::string("Trotter layer launch: ") + hipGetErrorString(e));
        }
        ED_TRY(record(st + 1));
    }
    ED_HIP_TRY(hipStreamSynchronize(s));
    return stage.finish(s);
}

extern "C" ed_status ed_trotter_passes(const ed_model* model, int order, int* passes) {
    using namespace ed;
    if (!model || !passes) return fail(ED_ERR_ARG, "null argument");
    if (order != 2 && order != 4) return fail(ED_ERR_ARG, "order must be 2 or 4");
    if (model->lr || model->lv_L > 0) return fail(ED_ERR_UNSUPPORTED, "the Trotter layers take site and bond rules only");
    StepPlan sp;
    ED_TRY(plan_step(model, order, 0.0, nullptr, nullptr, &sp));
    int n = 0;
    for (int r : sp.which) n += int(sp.runs[r].size());
    *passes = n;
    return ED_OK;
}
