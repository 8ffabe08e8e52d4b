// Internal declarations shared by the translation units of libed.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ed.h"

namespace ed {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
ed_status fail(ed_status code, const std::string& msg);

#define ED_HIP_TRY(expr)                                                                   \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess)                                                              \
            return ::ed::fail(ED_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

#define ED_TRY(expr)                     \
    do {                                 \
        ed_status _s = (expr);           \
        if (_s != ED_OK) return _s;      \
    } while (0)

ed_status require_device(int* device);

// ---------------------------------------------------------------- H psi plan
// Tile of one streaming pass: the low `c` bits of the index plus the window of `w` bits starting
// at bit h0 (h0 >= c, or w == 0). Sites and off-diagonal bonds are assigned to one pass each.
constexpr int kTileBits = 12;      // amplitudes per workgroup tile = 2^12 (64 KiB of LDS)
constexpr int kTileThreads = 256;  // threads per tile workgroup
constexpr int kTileSlots = (1 << kTileBits) / kTileThreads;  // register slots per thread (16)
constexpr int kMaxPasses = 4;

constexpr int kMaxGather = 8;     // index bits above a tile whose partner tiles are read from L2
constexpr int kMaxPlans = 96;     // candidate pass plans per model (chosen by ed_model_tune)
constexpr int kOccPadBytes = 40960;  // extra LDS that leaves room for one tile workgroup per CU

struct PassDesc {
    int c;            // contiguous low bits in the tile (window passes: 1..8)
    int h0;           // first bit of the window
    int w;            // window width (0 for the first pass)
    int first;        // 1: writes out (and adds the diagonal); 0: accumulates into out
    uint32_t site_mask;  // bit q set: the site on tile-local bit q belongs to this pass
    uint32_t bond_mask;  // bit q set: the bond on tile-local bits (q, q+1) belongs to this pass
    int bit_of[kTileBits];  // global bit of tile-local bit q
    // gathered bits [gb, gb + G) directly above the tile's top bit: their terms read the partner
    // amplitude from the neighbouring tile (tile index bit gpos + (g - gb)) instead of LDS
    int G;
    int gb;
    int gpos;
    int gcross;          // the bond (gb-1, gb) between the tile's top bit and the first gathered bit
    uint32_t site_gmask;  // bit i: site on gathered bit gb + i belongs to this pass
    uint32_t bond_gmask;  // bit i: bond (gb + i, gb + i + 1) belongs to this pass
    int occ1;            // launch with one workgroup per CU (a group's tiles then fit in L2)
    int pair;            // two tiles per workgroup: the first gathered bit's partner comes from LDS
    int wide;            // first pass: 1024 threads per tile, one per CU; window passes: 512, two per CU
};

// One gathered term of a pass as the kernels evaluate it: out[x] += coef * psi[partner of x], the
// partner sitting in tile n ^ txor at register slot k ^ sx of the same thread; coef depends on two
// bits of the tile index (pattern (n >> shift) & 3) and on the tile-local top bit (the upper half
// of the register slots). Built on the host from the plan and the folded operators.
struct GatherJob {
    int64_t txor;
    int sx;
    int shift;
    double2 coef[4][2];  // [pattern][local top bit]
};
constexpr int kMaxJobs = 4 * kMaxGather;  // G sites + 3 (G - 1) bond flips + 2 crossing-bond flips

enum OpClass : unsigned {
    kSiteOff = 1u,      // some site operator has off-diagonal entries
    kBondSingle = 2u,   // some bond operator flips exactly one of its two sites
    kBondDouble = 4u,   // some bond operator flips both sites
    kOffReal = 8u,      // every off-diagonal entry is real
    kDiagReal = 16u,    // every diagonal entry is real
};

}  // namespace ed

// Device-side coefficient tables of a model. All indices are by BIT position p (site at bit p is
// site k = L - p; the bond at bit p couples bits p and p+1, i.e. sites L-p-1 and L-p).
namespace ed {
// A two-site operator on the bit pair (p, q), q > p, at any distance: K[4 r + c] is the entry of
// row r = 2 bit(q) + bit(p) and column c; bit 4 r + c of mask is set where K is nonzero. Applied by
// a gather pass after the streaming passes of H psi (the jump terms of a Liouvillian).
struct FarTerm {
    int p, q;
    uint32_t mask;
    int pad;
    double2 K[16];
};
}  // namespace ed

struct ed_model {
    int L = 0;
    int device = 0;
    unsigned op_class = 0;
    // host copies (folded over the rule terms)
    std::vector<double2> site;   // [L][2][2]  per bit
    std::vector<double2> bond;   // [L-1][4][4] per bond bit, local index 2*bit(p+1) + bit(p)
    // device copies
    double2* d_site = nullptr;   // [L][4]
    double2* d_bond = nullptr;   // [L-1][16]
    double2* d_diag_lo = nullptr;  // [256]   bonds 0..6, sites 0..7   (low table)
    double2* d_diag_mid = nullptr; // [2^(T-7)] bonds 7..T-2, sites 8..T-1
    double2* d_diag_hi = nullptr;  // [2^(L-T+1)] bonds T-1..L-2, sites T..L-1 (+ long-range pairs
                                   //  with both bits in T-1..L-1)
    // long-range zz couplings (diagonal InfiniteFunc rules): H += sum_{p<q} lrz[p][q] z_p z_q (bits)
    bool lr = false;
    std::vector<double2> lrz;      // [L][L], upper triangle p < q
    double2* d_lr_low = nullptr;   // [2^T] pairs with both bits in 0..T-1 (L >= T) or all pairs (L < T)
    double2* d_lr_cross = nullptr; // [T-1][L] lrz[p][q] for p < T-1, q >= T (L >= T)
    int tile_bits = 0;           // T = min(L, kTileBits)
    int n_pass = 0;              // the selected plan (copied from cand[plan])
    ed::PassDesc pass[ed::kMaxPasses];
    int n_cand = 0;              // candidate plans and their pass counts
    int plan = 0;
    int cand_np[ed::kMaxPlans] = {};
    ed::PassDesc cand[ed::kMaxPlans][ed::kMaxPasses];
    // gathered terms of every candidate pass: [plan][pass][job], counts in njobs
    std::vector<ed::GatherJob> jobs;
    int njobs[ed::kMaxPlans][ed::kMaxPasses] = {};
    ed::GatherJob* d_jobs = nullptr;
    // Liouvillian models (ed_liouville_create): L = 2 lv_L bits of a superket, far terms = jump
    // sandwiches; 0 / empty for Hamiltonians
    int lv_L = 0;
    std::vector<ed::FarTerm> far;
    ed::FarTerm* d_far = nullptr;
};

namespace ed {
// Launch the passes of out = H psi (apply_h.hip), then the far terms if the model has any.
ed_status launch_apply_H(const ed_model* m, const double2* psi, double2* out, hipStream_t s);
// H psi whose last pass also leaves, per tile n, dot_part[n] = sum over the tile of conj(psi) out
// (*nparts = the number of tiles), when the plan ends with a window pass, there are no far terms
// and the tiles fit max_parts entries; otherwise a plain product with *nparts = 0.
ed_status launch_apply_H_dot(const ed_model* m, const double2* psi, double2* out, double2* dot_part,
                             int64_t max_parts, int64_t* nparts, hipStream_t s);
// out += sum of the far terms applied to psi (liouville.hip)
ed_status launch_far_terms(const ed_model* m, const double2* psi, double2* out, hipStream_t s);
// trace and sum_j rho_jj z_k(j), k = 1..Ls (site order), of a superket of an Ls-site system,
// into res[0] and res[1..Ls] (device, real parts) (liouville.hip)
ed_status superket_diag(const double2* rho, int Ls, double2* res, hipStream_t s);
}  // namespace ed
