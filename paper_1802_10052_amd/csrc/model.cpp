// Model handle: folds the rule-set terms (Eq. ed:eq:genericH, App. A site and bond rules) into
// one 2x2 operator per site and one 4x4 operator per bond, classifies the non-zero pattern so the
// H psi kernels can skip absent terms ("iterate only over non-zero elements", Sec. ed:sec:statics), builds the
// diagonal tables, and plans the streaming passes of H psi.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>

#include "ed_internal.h"

namespace ed {

using cplx = std::complex<double>;

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

ed_status fail(ed_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

ed_status require_device(int* device) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) return fail(ED_ERR_NODEVICE, "no HIP device visible");
    ED_HIP_TRY(hipGetDevice(device));
    return ED_OK;
}

// One pass plan. The first pass covers the 12 low bits plus `g_first` gathered bits above them;
// each later pass covers a window of 12 - cw bits above cw contiguous low bits (runs of 2^cw
// amplitudes), plus up to `gw_max` gathered bits above the window. With off-diagonal bond terms
// (`bonds`) consecutive passes overlap by one bit so that the bond crossing between them lies
// inside one tile; without them the passes tile the bits edge to edge. Returns the pass count, or
// -1 if this combination does not give a plan for L.
// Launch shape of a gathered pass: 0 two tile workgroups per CU, 1 one (LDS padding), 2 paired
// tiles, 3 one 1024-thread tile per CU.
static void set_shape(PassDesc& pd, int shape) {
    pd.occ1 = shape == 1 ? 1 : 0;
    pd.pair = shape == 2 ? 1 : 0;
    pd.wide = shape == 3 ? 1 : 0;
}

static int plan_make(int L, int g_first, int cw, int gw_max, bool bonds, int shape_first, int shape_win,
                     PassDesc* out) {
    const int T = kTileBits;
    const int tile_index_bits = L - T;
    // at least 8 groups, one per XCD
    auto gathers_fit = [&](int G) { return G <= kMaxGather && tile_index_bits >= 3 + G; };
    if (cw < 1 || cw > 8) return -1;
    int np = 0;
    PassDesc& p0 = out[np++];
    std::memset(&p0, 0, sizeof(PassDesc));
    p0.c = T;
    p0.h0 = T;
    p0.first = 1;
    for (int q = 0; q < T; ++q) p0.bit_of[q] = q;
    p0.site_mask = (1u << T) - 1u;
    p0.bond_mask = bonds ? (1u << (T - 1)) - 1u : 0u;
    const int G0 = std::min(g_first, L - T);
    if (G0 > 0) {
        if (!gathers_fit(G0)) return -1;
        p0.G = G0;
        p0.gb = T;
        p0.gpos = 0;
        p0.gcross = bonds ? 1 : 0;
        p0.site_gmask = (1u << G0) - 1u;
        p0.bond_gmask = (bonds && G0 > 1) ? (1u << (G0 - 1)) - 1u : 0u;
        set_shape(p0, shape_first);
    }
    int done = T + G0;  // sites on bits < done are assigned, and bonds (p, p+1) with p + 1 < done
    const int wb = T - cw;
    while (done < L) {
        if (np >= kMaxPasses) return -1;
        PassDesc& pd = out[np++];
        std::memset(&pd, 0, sizeof(PassDesc));
        int h0 = bonds ? done - 1 : done;
        int G = 0;
        if (h0 + wb >= L) {
            h0 = L - wb;  // last window: flush with the top bit
        } else {
            G = std::min(gw_max, L - (h0 + wb));
            if (G > 0 && !gathers_fit(G)) G = 0;
        }
        pd.c = cw;
        pd.h0 = h0;
        pd.w = wb;
        for (int q = 0; q < T; ++q) pd.bit_of[q] = q < cw ? q : h0 + (q - cw);
        for (int q = cw; q < T; ++q) {
            const int p = pd.bit_of[q];
            if (p >= done) pd.site_mask |= 1u << q;
            if (bonds && q + 1 < T && p + 1 >= done && p + 1 < L) pd.bond_mask |= 1u << q;
        }
        if (G > 0) {
            pd.G = G;
            pd.gb = h0 + wb;
            pd.gpos = h0 - cw;  // the window pass's tile index: bits [cw, h0) then [h0 + wb, L)
            pd.gcross = bonds ? 1 : 0;
            pd.site_gmask = (1u << G) - 1u;
            pd.bond_gmask = (bonds && G > 1) ? (1u << (G - 1)) - 1u : 0u;
            set_shape(pd, shape_win);
        }
        done = h0 + wb + G;
    }
    return np;
}

// Rough cost of a plan in units of one full read of the state, used only to order the candidates
// (the first one is the default before tuning): 2 state streams for the first pass, 3 for each
// accumulating window, windows of 128-byte runs high up slower, and each gathered bit a fraction
// of a stream (mostly L2 hits in the first pass, mostly misses in windows, whose partner lines sit
// a power-of-two apart).
static double plan_cost(const PassDesc* pass, int np) {
    double cost = 0.0;
    for (int i = 0; i < np; ++i) {
        const PassDesc& pd = pass[i];
        const int gl2 = pd.pair ? pd.G - 1 : pd.G;  // gathered bits read through L2
        const double stream = pd.pair ? 0.95 : (pd.wide ? 0.97 : 1.0);
        // one tile per CU keeps more of a gather group's neighbours in L2
        const double per_bit = pd.wide ? 0.8 : 1.0;
        if (pd.first) {
            cost += 2.0 * stream + 0.35 * per_bit * gl2;
        } else {
            const double slow = (pd.c <= 3 && pd.h0 >= 17) ? 1.25 : (pd.c <= 3 ? 1.05 : 1.0);
            cost += 3.0 * slow * stream + 1.2 * per_bit * gl2;
        }
    }
    return cost;
}

// Candidate plans: every combination of first-pass gathers, window run length, window gathers and
// the launch shapes of the first and the window passes that reaches the fewest passes, cheapest
// first by plan_cost, then the plain plan (no gathers) if it is not among them. ed_model_tune
// times them on the device.
static void plan_passes(ed_model* m) {
    const int L = m->L;
    const int T = kTileBits;
    const bool bonds = (m->op_class & (kBondSingle | kBondDouble)) != 0;
    m->tile_bits = L < T ? L : T;
    m->n_cand = 0;
    m->plan = 0;
    if (L < T) {
        m->n_cand = 1;
        m->cand_np[0] = 1;
        std::memset(&m->cand[0][0], 0, sizeof(PassDesc));
        m->cand[0][0].first = 1;
        m->cand[0][0].c = L;
        m->n_pass = 1;
        m->pass[0] = m->cand[0][0];
        return;
    }
    struct Cand {
        PassDesc p[kMaxPasses];
        int np;
        double cost;
    };
    std::vector<Cand> all;
    Cand plain{};
    plain.np = plan_make(L, 0, 3, 0, bonds, 0, 0, plain.p);
    plain.cost = plain.np > 0 ? plan_cost(plain.p, plain.np) : 0.0;
    for (int g = 0; g <= kMaxGather; ++g)
        for (int cw = 3; cw <= 4; ++cw)
            for (int gw : {0, 2, 4})
                for (int shape = 0; shape < 9; ++shape) {  // launch shapes of the first and window passes
                    // normal, paired or wide each (the one-workgroup-per-CU shape of 256 threads is
                    // never faster than the wide one with the same L2 footprint)
                    static const int kShapes[3] = {0, 2, 3};
                    Cand c{};
                    c.np = plan_make(L, g, cw, gw, bonds, kShapes[shape % 3], kShapes[shape / 3], c.p);
                    if (c.np <= 0) continue;  // (a shape on passes without gathers gives a duplicate)
                    c.cost = plan_cost(c.p, c.np);
                    bool dup = false;
                    for (const Cand& o : all)
                        dup = dup || (o.np == c.np && std::memcmp(o.p, c.p, sizeof(PassDesc) * c.np) == 0);
                    if (!dup) all.push_back(c);
                }
    int best_np = kMaxPasses + 1;
    for (const Cand& c : all) best_np = std::min(best_np, c.np);
    std::vector<Cand> keep;
    for (const Cand& c : all)
        if (c.np == best_np) keep.push_back(c);
    std::stable_sort(keep.begin(), keep.end(), [](const Cand& a, const Cand& b) { return a.cost < b.cost; });
    auto add = [&](const Cand& c) {
        if (m->n_cand >= kMaxPlans) return;
        for (int i = 0; i < m->n_cand; ++i)
            if (m->cand_np[i] == c.np && std::memcmp(m->cand[i], c.p, sizeof(PassDesc) * c.np) == 0) return;
        m->cand_np[m->n_cand] = c.np;
        for (int i = 0; i < c.np; ++i) m->cand[m->n_cand][i] = c.p[i];
        ++m->n_cand;
    };
    const int room = plain.np > 0 ? kMaxPlans - 1 : kMaxPlans;
    for (size_t i = 0; i < keep.size() && m->n_cand < room; ++i) add(keep[i]);
    if (plain.np > 0) add(plain);
    m->n_pass = m->cand_np[0];
    for (int i = 0; i < m->n_pass; ++i) m->pass[i] = m->cand[0][i];
}

// Every site must belong to exactly one pass, and so must every bond when the model has
// off-diagonal bond terms (otherwise a bond may belong to at most one); every gathered bit must
// sit where the tile-index mapping expects it. A plan that breaks this is a bug, reported as such.
static bool plan_is_valid(int L, bool bonds_needed, const PassDesc* pass, int n_pass) {
    if (L < kTileBits) return n_pass == 1;
    if (n_pass < 1 || n_pass > kMaxPasses) return false;
    std::vector<int> sites(L, 0), bonds(L - 1, 0);
    for (int ip = 0; ip < n_pass; ++ip) {
        const PassDesc& pd = pass[ip];
        if (pd.first != (ip == 0 ? 1 : 0)) return false;
        if (pd.first) {
            if (pd.c != kTileBits || pd.h0 != kTileBits) return false;
        } else {
            if (pd.c < 1 || pd.c > 8 || pd.w != kTileBits - pd.c || pd.h0 < pd.c || pd.h0 + pd.w > L) return false;
        }
        if (pd.occ1 != 0 && pd.occ1 != 1) return false;
        if (pd.pair != 0 && (pd.pair != 1 || pd.G < 1 || pd.occ1)) return false;
        if (pd.wide != 0 && (pd.wide != 1 || pd.G < 1 || pd.occ1 || pd.pair || (!pd.first && pd.c > 10))) return false;
        for (int q = 0; q < kTileBits; ++q) {
            const int p = pd.bit_of[q];
            if (p < 0 || p >= L) return false;
            if ((pd.site_mask >> q) & 1) ++sites[p];
            if ((pd.bond_mask >> q) & 1) {
                if (q + 1 >= kTileBits || pd.bit_of[q + 1] != p + 1 || p + 1 >= L) return false;
                ++bonds[p];
            }
        }
        if (pd.G > 0) {
            if (pd.G > kMaxGather || pd.gb + pd.G > L) return false;
            if (pd.gpos + pd.G > L - kTileBits || L - kTileBits < 3 + pd.G) return false;
            if (pd.bit_of[kTileBits - 1] != pd.gb - 1) return false;
            // the tile index bit gpos + i must be global bit gb + i
            const int expect_gpos = pd.first ? pd.gb - kTileBits : pd.h0 - pd.c;
            if (pd.gpos != expect_gpos || (!pd.first && pd.gb != pd.h0 + kTileBits - pd.c)) return false;
            for (int i = 0; i < pd.G; ++i) {
                if ((pd.site_gmask >> i) & 1) ++sites[pd.gb + i];
                if ((pd.bond_gmask >> i) & 1) {
                    if (i + 1 >= pd.G) return false;
                    ++bonds[pd.gb + i];
                }
            }
            if (pd.gcross) ++bonds[pd.gb - 1];
        } else if (pd.site_gmask || pd.bond_gmask || pd.gcross || pd.occ1 || pd.pair || pd.wide) {
            return false;
        }
    }
    for (int c : sites)
        if (c != 1) return false;
    for (int c : bonds)
        if (bonds_needed ? c != 1 : c > 1) return false;
    return true;
}

// Gathered terms of one pass (see GatherJob), skipping terms whose coefficients all vanish.
static int build_jobs(const ed_model* m, const PassDesc& pd, GatherJob* out) {
    if (pd.G == 0) return 0;
    int nj = 0;
    auto push = [&](int64_t txor, int sx, int shift, auto coef) {
        GatherJob j{};
        j.txor = txor;
        j.sx = sx;
        j.shift = shift;
        bool nz = false;
        for (int p = 0; p < 4; ++p)
            for (int lt = 0; lt < 2; ++lt) {
                j.coef[p][lt] = coef(p, lt);
                nz = nz || j.coef[p][lt].x != 0.0 || j.coef[p][lt].y != 0.0;
            }
        if (nz && nj < kMaxJobs) out[nj++] = j;
    };
    for (int gi = 0; gi < pd.G; ++gi) {
        const int g = pd.gb + gi;
        const int sh = pd.gpos + gi;
        if ((pd.site_gmask >> gi) & 1) {
            const double2* S = m->site.data() + 4 * g;
            push(int64_t(1) << sh, 0, sh, [&](int p, int) { return S[(p & 1) ? 2 : 1]; });
        }
        if ((pd.bond_gmask >> gi) & 1) {
            // bond (g, g+1): local index l = 2 bit(g+1) + bit(g) = the pattern
            const double2* B = m->bond.data() + 16 * g;
            push(int64_t(1) << sh, 0, sh, [&](int p, int) { return B[4 * p + (p ^ 1)]; });
            push(int64_t(2) << sh, 0, sh, [&](int p, int) { return B[4 * p + (p ^ 2)]; });
            push(int64_t(3) << sh, 0, sh, [&](int p, int) { return B[4 * p + (p ^ 3)]; });
        }
    }
    if (pd.gcross) {
        // bond (gb-1, gb): local index l = 2 bit(gb) + (tile-local top bit); flipping only the local
        // top bit stays in registers (kernel), flipping bit gb or both reads tile n ^ bit(gb)
        const double2* B = m->bond.data() + 16 * (pd.gb - 1);
        const int sh = pd.gpos;
        push(int64_t(1) << sh, 0, sh, [&](int p, int lt) {
            const int l = 2 * (p & 1) + lt;
            return B[4 * l + (l ^ 2)];
        });
        push(int64_t(1) << sh, kTileSlots / 2, sh, [&](int p, int lt) {
            const int l = 2 * (p & 1) + lt;
            return B[4 * l + (l ^ 3)];
        });
    }
    return nj;
}

static inline double2 c2(double re, double im) { return make_double2(re, im); }

// diagonal contribution of the sites on bits [s_lo, s_hi) and bonds on bits [b_lo, b_hi)
// evaluated at index x
static double2 diag_part(const ed_model* m, uint64_t x, int s_lo, int s_hi, int b_lo, int b_hi) {
    double re = 0.0, im = 0.0;
    for (int p = s_lo; p < s_hi; ++p) {
        const int b = int((x >> p) & 1u);
        const double2 v = m->site[4 * p + 3 * b];
        re += v.x;
        im += v.y;
    }
    for (int p = b_lo; p < b_hi; ++p) {
        const int l = int((x >> p) & 3u);
        const double2 v = m->bond[16 * p + 5 * l];
        re += v.x;
        im += v.y;
    }
    return c2(re, im);
}

static ed_status upload(double2** dst, const std::vector<double2>& src) {
    const size_t bytes = (src.empty() ? 1 : src.size()) * sizeof(double2);
    ED_HIP_TRY(hipMalloc(dst, bytes));
    if (!src.empty()) ED_HIP_TRY(hipMemcpy(*dst, src.data(), src.size() * sizeof(double2), hipMemcpyHostToDevice));
    return ED_OK;
}

static void free_tables(ed_model* m) {
    double2** ptrs[] = {&m->d_site, &m->d_bond, &m->d_diag_lo, &m->d_diag_mid, &m->d_diag_hi, &m->d_lr_low,
                        &m->d_lr_cross};
    for (double2** p : ptrs) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    if (m->d_jobs) (void)hipFree(m->d_jobs);
    m->d_jobs = nullptr;
    if (m->d_far) (void)hipFree(m->d_far);
    m->d_far = nullptr;
}

// long-range zz energy of the pairs p < q with both bits in [lo, hi), evaluated at index x
static double2 lr_part(const ed_model* m, uint64_t x, int lo, int hi) {
    double re = 0.0, im = 0.0;
    const int L = m->L;
    for (int p = lo; p < hi; ++p)
        for (int q = p + 1; q < hi; ++q) {
            const double2 v = m->lrz[size_t(p) * L + q];
            if (v.x == 0.0 && v.y == 0.0) continue;
            const double zz = (((x >> p) ^ (x >> q)) & 1) ? -1.0 : 1.0;
            re += zz * v.x;
            im += zz * v.y;
        }
    return c2(re, im);
}

ed_status build_device_tables(ed_model* m) {
    const int L = m->L;
    ED_TRY(upload(&m->d_site, m->site));
    ED_TRY(upload(&m->d_bond, m->bond));
    if (L >= kTileBits) {
        const int T = kTileBits;
        std::vector<double2> lo(256), mid(size_t(1) << (T - 7)), hi(size_t(1) << (L - T + 1));
        for (uint64_t j = 0; j < lo.size(); ++j) lo[j] = diag_part(m, j, 0, 8, 0, 7);
        for (uint64_t j = 0; j < mid.size(); ++j) mid[j] = diag_part(m, j << 7, 8, T, 7, T - 1);
        for (uint64_t j = 0; j < hi.size(); ++j) {
            hi[j] = diag_part(m, j << (T - 1), T, L, T - 1, L - 1);
            if (m->lr) {
                const double2 e = lr_part(m, j << (T - 1), T - 1, L);
                hi[j].x += e.x;
                hi[j].y += e.y;
            }
        }
        ED_TRY(upload(&m->d_diag_lo, lo));
        ED_TRY(upload(&m->d_diag_mid, mid));
        ED_TRY(upload(&m->d_diag_hi, hi));
        if (m->lr) {
            // pairs inside the 12 low bits; pairs (p < T-1, q >= T) as per-tile fields; pairs with
            // both bits in [T-1, L) are in the high table above
            std::vector<double2> low(size_t(1) << T), cross(size_t(T - 1) * L, c2(0, 0));
            for (uint64_t i = 0; i < low.size(); ++i) low[i] = lr_part(m, i, 0, T);
            for (int p = 0; p < T - 1; ++p)
                for (int q = T; q < L; ++q) cross[size_t(p) * L + q] = m->lrz[size_t(p) * L + q];
            ED_TRY(upload(&m->d_lr_low, low));
            ED_TRY(upload(&m->d_lr_cross, cross));
        }
    } else if (m->lr) {
        std::vector<double2> full(size_t(1) << L);
        for (uint64_t x = 0; x < full.size(); ++x) full[x] = lr_part(m, x, 0, L);
        ED_TRY(upload(&m->d_lr_low, full));
    }
    const size_t jb = m->jobs.size() * sizeof(GatherJob);
    ED_HIP_TRY(hipMalloc(reinterpret_cast<void**>(&m->d_jobs), jb ? jb : sizeof(GatherJob)));
    if (jb) ED_HIP_TRY(hipMemcpy(m->d_jobs, m->jobs.data(), jb, hipMemcpyHostToDevice));
    return ED_OK;
}

// Fold the rule terms into per-bit operators and classify them.
ed_status fold_model(const ed_model_desc* desc, ed_model* m) {
    const int L = desc->L;
    m->L = L;
    m->site.assign(size_t(4) * L, c2(0, 0));
    m->bond.assign(size_t(16) * (L - 1), c2(0, 0));
    for (int z = 0; z < desc->n_site; ++z) {
        for (int k = 1; k <= L; ++k) {
            const double c = desc->site_coef[size_t(z) * L + (k - 1)];
            if (c == 0.0) continue;
            const int p = L - k;
            for (int e = 0; e < 4; ++e) {
                const ed_c64 o = desc->site_op[size_t(z) * 4 + e];
                m->site[4 * p + e].x += c * o.re;
                m->site[4 * p + e].y += c * o.im;
            }
        }
    }
    for (int z = 0; z < desc->n_bond; ++z) {
        for (int k = 1; k <= L - 1; ++k) {
            const double c = desc->bond_coef[size_t(z) * (L - 1) + (k - 1)];
            if (c == 0.0) continue;
            const int p = L - k - 1;  // bits (p, p+1) = sites (k+1, k); local index 2*i_k + i_{k+1}
            for (int e = 0; e < 16; ++e) {
                const ed_c64 o = desc->bond_op[size_t(z) * 16 + e];
                m->bond[16 * p + e].x += c * o.re;
                m->bond[16 * p + e].y += c * o.im;
            }
        }
    }
    // diagonal InfiniteFunc rules: c f(j-k) O_k O'_j with O = diag(o0, o1), O' = diag(p0, p1) is
    // (a + b z_k)(c + d z_j) c f, a = (o0+o1)/2, b = (o0-o1)/2, c = (p0+p1)/2, d = (p0-p1)/2
    // (z = +1 for index 0): its constant and field parts go to the site diagonals, its zz part to
    // the long-range coupling table
    m->lrz.assign(size_t(L) * L, c2(0, 0));
    for (int z = 0; z < desc->n_inf; ++z) {
        const ed_c64* O = desc->inf_op + 4 * z;
        const ed_c64* Q = desc->inf_op2 + 4 * z;
        const cplx o0(O[0].re, O[0].im), o1(O[3].re, O[3].im), p0(Q[0].re, Q[0].im), p1(Q[3].re, Q[3].im);
        const cplx a = 0.5 * (o0 + o1), b = 0.5 * (o0 - o1), c = 0.5 * (p0 + p1), d = 0.5 * (p0 - p1);
        for (int k = 1; k < L; ++k)
            for (int j = k + 1; j <= L; ++j) {
                const double w = desc->inf_coef[size_t(z) * L + (k - 1)] * desc->inf_f[size_t(z) * (L - 1) + (j - k - 1)];
                if (w == 0.0) continue;
                const int pk = L - k, pj = L - j;  // bits of sites k and j
                auto add_site = [&](int p, cplx v0, cplx v1) {
                    m->site[4 * p + 0].x += v0.real();
                    m->site[4 * p + 0].y += v0.imag();
                    m->site[4 * p + 3].x += v1.real();
                    m->site[4 * p + 3].y += v1.imag();
                };
                const cplx cst = w * a * c, fk = w * b * c, fj = w * a * d, zz = w * b * d;
                add_site(pk, cst + fk, cst - fk);
                add_site(pj, fj, -fj);
                double2& e = m->lrz[size_t(pj) * L + pk];  // pj < pk
                e.x += zz.real();
                e.y += zz.imag();
            }
    }
    for (const double2& e : m->lrz) m->lr = m->lr || e.x != 0.0 || e.y != 0.0;
    unsigned cls = kOffReal | kDiagReal;
    for (const double2& e : m->lrz)
        if (e.y != 0.0) cls &= ~unsigned(kDiagReal);
    for (int p = 0; p < L; ++p) {
        for (int e = 0; e < 4; ++e) {
            const double2 v = m->site[4 * p + e];
            const bool diag = (e == 0 || e == 3);
            if (v.x == 0.0 && v.y == 0.0) continue;
            if (!diag) cls |= kSiteOff;
            if (v.y != 0.0) cls &= diag ? ~unsigned(kDiagReal) : ~unsigned(kOffReal);
        }
    }
    for (int p = 0; p + 1 < L; ++p) {
        for (int r = 0; r < 4; ++r) {
            for (int cc = 0; cc < 4; ++cc) {
                const double2 v = m->bond[16 * p + 4 * r + cc];
                if (v.x == 0.0 && v.y == 0.0) continue;
                const int f = r ^ cc;
                if (f == 1 || f == 2) cls |= kBondSingle;
                if (f == 3) cls |= kBondDouble;
                if (v.y != 0.0) cls &= (f == 0) ? ~unsigned(kDiagReal) : ~unsigned(kOffReal);
            }
        }
    }
    m->op_class = cls;
    plan_passes(m);
    for (int c = 0; c < m->n_cand; ++c)
        if (!plan_is_valid(L, (cls & (kBondSingle | kBondDouble)) != 0, m->cand[c], m->cand_np[c]))
            return fail(ED_ERR_UNSUPPORTED, "internal error: invalid H psi pass plan " + std::to_string(c) + " for L = " +
                                                std::to_string(L));
    m->jobs.assign(size_t(kMaxPlans) * kMaxPasses * kMaxJobs, GatherJob{});
    for (int c = 0; c < m->n_cand; ++c)
        for (int i = 0; i < m->cand_np[c]; ++i)
            m->njobs[c][i] = build_jobs(m, m->cand[c][i], m->jobs.data() + (size_t(c) * kMaxPasses + i) * kMaxJobs);
    return ED_OK;
}

ed_status validate_desc(const ed_model_desc* desc) {
    if (!desc) return fail(ED_ERR_ARG, "desc is null");
    if (desc->d != 2) return fail(ED_ERR_UNSUPPORTED, "only d = 2 is supported");
    if (desc->L < 2 || desc->L > 30) return fail(ED_ERR_UNSUPPORTED, "L must be in [2, 30]");
    if (desc->n_site < 0 || desc->n_bond < 0) return fail(ED_ERR_ARG, "negative term count");
    if (desc->n_site > 0 && (!desc->site_op || !desc->site_coef))
        return fail(ED_ERR_ARG, "site_op/site_coef is null with n_site > 0");
    if (desc->n_bond > 0 && (!desc->bond_op || !desc->bond_coef))
        return fail(ED_ERR_ARG, "bond_op/bond_coef is null with n_bond > 0");
    for (int z = 0; z < desc->n_site; ++z) {
        for (int e = 0; e < 4; ++e) {
            const ed_c64 o = desc->site_op[4 * z + e];
            if (!std::isfinite(o.re) || !std::isfinite(o.im)) return fail(ED_ERR_NUMERIC, "non-finite site_op");
        }
        for (int k = 0; k < desc->L; ++k)
            if (!std::isfinite(desc->site_coef[size_t(z) * desc->L + k])) return fail(ED_ERR_NUMERIC, "non-finite site_coef");
    }
    if (desc->n_inf < 0) return fail(ED_ERR_ARG, "negative term count");
    if (desc->n_inf > 0 && (!desc->inf_op || !desc->inf_op2 || !desc->inf_coef || !desc->inf_f))
        return fail(ED_ERR_ARG, "inf_op/inf_op2/inf_coef/inf_f is null with n_inf > 0");
    for (int z = 0; z < desc->n_inf; ++z) {
        for (int e = 0; e < 4; ++e) {
            const ed_c64 o = desc->inf_op[4 * z + e], q = desc->inf_op2[4 * z + e];
            if (!std::isfinite(o.re) || !std::isfinite(o.im) || !std::isfinite(q.re) || !std::isfinite(q.im))
                return fail(ED_ERR_NUMERIC, "non-finite inf_op");
            if ((e == 1 || e == 2) && (o.re != 0.0 || o.im != 0.0 || q.re != 0.0 || q.im != 0.0))
                return fail(ED_ERR_UNSUPPORTED, "InfiniteFunc rules need diagonal operators");
        }
        for (int k = 0; k < desc->L; ++k)
            if (!std::isfinite(desc->inf_coef[size_t(z) * desc->L + k])) return fail(ED_ERR_NUMERIC, "non-finite inf_coef");
        for (int r = 0; r + 1 < desc->L; ++r)
            if (!std::isfinite(desc->inf_f[size_t(z) * (desc->L - 1) + r])) return fail(ED_ERR_NUMERIC, "non-finite inf_f");
    }
    for (int z = 0; z < desc->n_bond; ++z) {
        for (int e = 0; e < 16; ++e) {
            const ed_c64 o = desc->bond_op[16 * z + e];
            if (!std::isfinite(o.re) || !std::isfinite(o.im)) return fail(ED_ERR_NUMERIC, "non-finite bond_op");
        }
        for (int k = 0; k < desc->L - 1; ++k)
            if (!std::isfinite(desc->bond_coef[size_t(z) * (desc->L - 1) + k])) return fail(ED_ERR_NUMERIC, "non-finite bond_coef");
    }
    return ED_OK;
}

void apply_cached_plan(ed_model* m);

ed_status create_model(const ed_model_desc* desc, ed_model** out) {
    ED_TRY(validate_desc(desc));
    ed_model* m = new (std::nothrow) ed_model();
    if (!m) return fail(ED_ERR_NOMEM, "host allocation failed");
    ed_status st = fold_model(desc, m);
    if (st == ED_OK) st = require_device(&m->device);
    if (st == ED_OK) st = build_device_tables(m);
    if (st != ED_OK) {
        free_tables(m);
        delete m;
        return st;
    }
    apply_cached_plan(m);
    *out = m;
    return ED_OK;
}

void destroy_model(ed_model* m);

// The Liouvillian of H (Hermitian, no InfiniteFunc rules) with jump operators J_nu on every site
// at rates gamma_nu[k], as a model on the 2L-bit superket: i Lcal = H_eff (x) 1 - 1 (x) H_eff^*
// + i sum gamma J (x) J^* (see liouville.hip). Doubled chain: sites 1..L are the row digits
// (bits 2L-1 .. L), sites L+1..2L the column digits (bits L-1 .. 0).
ed_status create_liouville(const ed_model_desc* H, int n_jump, const ed_c64* jump_op, const double* rates,
                           ed_model** out) {
    ED_TRY(validate_desc(H));
    const int L = H->L;
    if (2 * L > 30) return fail(ED_ERR_UNSUPPORTED, "the superket of L sites has 2L bits: L <= 15");
    if (H->n_inf > 0) return fail(ED_ERR_UNSUPPORTED, "Liouvillians do not take InfiniteFunc rules");
    if (n_jump < 0) return fail(ED_ERR_ARG, "n_jump must be >= 0");
    if (n_jump > 0 && (!jump_op || !rates)) return fail(ED_ERR_ARG, "jump_op/rates is null with n_jump > 0");
    for (int z = 0; z < n_jump; ++z) {
        for (int e = 0; e < 4; ++e)
            if (!std::isfinite(jump_op[4 * z + e].re) || !std::isfinite(jump_op[4 * z + e].im))
                return fail(ED_ERR_NUMERIC, "non-finite jump_op");
        for (int k = 0; k < L; ++k)
            if (!std::isfinite(rates[size_t(z) * L + k]) || rates[size_t(z) * L + k] < 0.0)
                return fail(ED_ERR_ARG, "rates must be finite and >= 0");
    }
    const int L2 = 2 * L;
    auto c64 = [](cplx v) { return ed_c64{v.real(), v.imag()}; };
    auto cx = [](const ed_c64& v) { return cplx(v.re, v.im); };
    std::vector<ed_c64> sop;
    std::vector<double> scoef;
    std::vector<ed_c64> bop;
    std::vector<double> bcoef;
    // site rules: O on the row digits, -O^* on the column digits
    for (int z = 0; z < H->n_site; ++z) {
        for (int half = 0; half < 2; ++half) {
            for (int e = 0; e < 4; ++e) {
                const cplx o = cx(H->site_op[4 * z + e]);
                sop.push_back(c64(half == 0 ? o : -std::conj(o)));
            }
            for (int k = 0; k < L2; ++k) scoef.push_back((k < L) == (half == 0) ? H->site_coef[size_t(z) * L + (k % L)] : 0.0);
        }
    }
    // -(i/2) gamma J^dagger J in H_eff: on the rows as is, on the columns -(its conjugate)
    for (int z = 0; z < n_jump; ++z) {
        cplx J[2][2], JdJ[2][2];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) J[a][b] = cx(jump_op[4 * z + 2 * a + b]);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) JdJ[a][b] = std::conj(J[0][a]) * J[0][b] + std::conj(J[1][a]) * J[1][b];
        for (int half = 0; half < 2; ++half) {
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    const cplx o = cplx(0.0, -0.5) * JdJ[a][b];
                    sop.push_back(c64(half == 0 ? o : -std::conj(o)));
                }
            for (int k = 0; k < L2; ++k) scoef.push_back((k < L) == (half == 0) ? rates[size_t(z) * L + (k % L)] : 0.0);
        }
    }
    // bond rules: B on the row bonds, -B^* on the column bonds, nothing on the middle bond
    for (int z = 0; z < H->n_bond; ++z) {
        for (int half = 0; half < 2; ++half) {
            for (int e = 0; e < 16; ++e) {
                const cplx o = cx(H->bond_op[16 * z + e]);
                bop.push_back(c64(half == 0 ? o : -std::conj(o)));
            }
            for (int k = 0; k < L2 - 1; ++k) {
                double c = 0.0;
                if (half == 0 && k < L - 1) c = H->bond_coef[size_t(z) * (L - 1) + k];
                if (half == 1 && k >= L) c = H->bond_coef[size_t(z) * (L - 1) + (k - L)];
                bcoef.push_back(c);
            }
        }
    }
    ed_model_desc d{};
    d.L = L2;
    d.d = 2;
    d.n_site = int(scoef.size()) / L2;
    d.site_op = sop.data();
    d.site_coef = scoef.data();
    d.n_bond = int(bcoef.size()) / (L2 - 1);
    d.bond_op = bop.data();
    d.bond_coef = bcoef.data();
    d.n_inf = 0;
    ed_model* m = nullptr;
    ED_TRY(create_model(&d, &m));
    m->lv_L = L;
    // jump sandwiches i gamma J (x) J^*, row bit q = 2L - k, column bit p = L - k of site k
    for (int k = 1; k <= L; ++k) {
        FarTerm ft{};
        ft.p = L - k;
        ft.q = L2 - k;
        bool any = false;
        for (int z = 0; z < n_jump; ++z) {
            const double g = rates[size_t(z) * L + (k - 1)];
            if (g == 0.0) continue;
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c) {
                    const cplx Ja = cx(jump_op[4 * z + 2 * (r >> 1) + (c >> 1)]);
                    const cplx Jb = cx(jump_op[4 * z + 2 * (r & 1) + (c & 1)]);
                    const cplx v = cplx(0.0, g) * Ja * std::conj(Jb);
                    ft.K[4 * r + c].x += v.real();
                    ft.K[4 * r + c].y += v.imag();
                }
        }
        for (int e = 0; e < 16; ++e)
            if (ft.K[e].x != 0.0 || ft.K[e].y != 0.0) {
                ft.mask |= 1u << e;
                any = true;
            }
        if (any) m->far.push_back(ft);
    }
    if (!m->far.empty()) {
        const size_t bytes = m->far.size() * sizeof(FarTerm);
        hipError_t e = hipMalloc(reinterpret_cast<void**>(&m->d_far), bytes);
        if (e == hipSuccess) e = hipMemcpy(m->d_far, m->far.data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            destroy_model(m);
            return fail(ED_ERR_HIP, std::string("far-term upload: ") + hipGetErrorString(e));
        }
    }
    apply_cached_plan(m);
    *out = m;
    return ED_OK;
}

// One-line description of candidate plan `index`, e.g. "first +G5 wide | c4 h17 +G3".
std::string describe_plan(const ed_model* m, int index) {
    std::string d;
    for (int i = 0; i < m->cand_np[index]; ++i) {
        const PassDesc& pd = m->cand[index][i];
        if (i) d += " | ";
        if (m->L < kTileBits) {
            d += "small";
        } else if (pd.first) {
            d += "first";
        } else {
            d += "c" + std::to_string(pd.c) + " h" + std::to_string(pd.h0);
        }
        if (pd.G > 0) d += " +G" + std::to_string(pd.G);
        if (pd.occ1) d += " occ1";
        if (pd.pair) d += " pair";
        if (pd.wide) d += " wide";
    }
    return d;
}

// ------------------------------------------------------------------------ tuned-plan cache
// Key -> description of the fastest plan. The key names the GPU architecture, L, the operator
// class (the kernel variant), the Liouville and long-range flags and a hash of the whole candidate
// list, so an entry applies only to a model whose planner proposes exactly the same candidates.
namespace {
struct PlanCache {
    std::mutex mu;
    std::map<std::string, std::string> map;
};
PlanCache& plan_cache() {
    static PlanCache c;
    return c;
}

std::string arch_name(int device) {
    static std::mutex mu;
    static std::map<int, std::string> names;
    std::lock_guard<std::mutex> lock(mu);
    auto it = names.find(device);
    if (it != names.end()) return it->second;
    hipDeviceProp_t prop;
    std::string a = "unknown";
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        a = prop.gcnArchName;
        const size_t colon = a.find(':');
        if (colon != std::string::npos) a = a.substr(0, colon);
    }
    names[device] = a;
    return a;
}
}  // namespace

std::string plan_key(const ed_model* m) {
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the candidate descriptions
    for (int c = 0; c < m->n_cand; ++c) {
        for (char ch : describe_plan(m, c) + ";") {
            h ^= uint64_t(uint8_t(ch));
            h *= 1099511628211ull;
        }
    }
    char hex[17];
    std::snprintf(hex, sizeof hex, "%016llx", static_cast<unsigned long long>(h));
    return arch_name(m->device) + " L=" + std::to_string(m->L) + " class=" + std::to_string(m->op_class) +
           " liouville=" + std::to_string(m->lv_L) + " lr=" + std::to_string(m->lr ? 1 : 0) +
           " far=" + std::to_string(m->far.size()) + " cands=" + hex;
}

// Select the cached plan of m, if the cache holds one for its key (no-op otherwise).
void apply_cached_plan(ed_model* m) {
    std::string want;
    {
        PlanCache& pc = plan_cache();
        std::lock_guard<std::mutex> lock(pc.mu);
        auto it = pc.map.find(plan_key(m));
        if (it == pc.map.end()) return;
        want = it->second;
    }
    for (int c = 0; c < m->n_cand; ++c) {
        if (describe_plan(m, c) == want) {
            m->plan = c;
            m->n_pass = m->cand_np[c];
            for (int i = 0; i < m->n_pass; ++i) m->pass[i] = m->cand[c][i];
            return;
        }
    }
}

void remember_plan(const ed_model* m) {
    PlanCache& pc = plan_cache();
    const std::string key = plan_key(m), val = describe_plan(m, m->plan);
    std::lock_guard<std::mutex> lock(pc.mu);
    pc.map[key] = val;
}

void destroy_model(ed_model* m) {
    if (!m) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(m->device);
    free_tables(m);
    (void)hipSetDevice(cur);
    delete m;
}

}  // namespace ed

extern "C" {

const char* ed_last_error(void) { return ed::g_last_error.c_str(); }

const char* ed_version(void) { return "libed 0.1 (gfx950)"; }

ed_status ed_model_create(const ed_model_desc* desc, ed_model** out) {
    if (!out) return ed::fail(ED_ERR_ARG, "out is null");
    *out = nullptr;
    return ed::create_model(desc, out);
}

ed_status ed_liouville_create(const ed_model_desc* H, int n_jump, const ed_c64* jump_op, const double* rates,
                              ed_model** out) {
    if (!out) return ed::fail(ED_ERR_ARG, "out is null");
    *out = nullptr;
    return ed::create_liouville(H, n_jump, jump_op, rates, out);
}

ed_status ed_model_liouville_sites(const ed_model* model, int* L) {
    if (!model || !L) return ed::fail(ED_ERR_ARG, "null argument");
    *L = model->lv_L;
    return ED_OK;
}

ed_status ed_model_destroy(ed_model* model) {
    ed::destroy_model(model);
    return ED_OK;
}

ed_status ed_model_dims(const ed_model* model, int* L, int64_t* D) {
    if (!model) return ed::fail(ED_ERR_ARG, "model is null");
    if (L) *L = model->L;
    if (D) *D = int64_t(1) << model->L;
    return ED_OK;
}

ed_status ed_model_passes(const ed_model* model, int* passes) {
    if (!model || !passes) return ed::fail(ED_ERR_ARG, "null argument");
    *passes = model->n_pass;
    return ED_OK;
}

ed_status ed_model_plans(const ed_model* model, int* count, int* selected) {
    if (!model) return ed::fail(ED_ERR_ARG, "model is null");
    if (count) *count = model->n_cand;
    if (selected) *selected = model->plan;
    return ED_OK;
}

ed_status ed_model_select_plan(ed_model* model, int index) {
    if (!model) return ed::fail(ED_ERR_ARG, "model is null");
    if (index < 0 || index >= model->n_cand) return ed::fail(ED_ERR_ARG, "plan index out of range");
    model->plan = index;
    model->n_pass = model->cand_np[index];
    for (int i = 0; i < model->n_pass; ++i) model->pass[i] = model->cand[index][i];
    return ED_OK;
}

ed_status ed_model_plan_describe(const ed_model* model, int index, char* buf, int buf_len) {
    if (!model || !buf || buf_len < 1) return ed::fail(ED_ERR_ARG, "null argument");
    if (index < 0 || index >= model->n_cand) return ed::fail(ED_ERR_ARG, "plan index out of range");
    const std::string d = ed::describe_plan(model, index);
    std::strncpy(buf, d.c_str(), size_t(buf_len) - 1);
    buf[buf_len - 1] = 0;
    return ED_OK;
}

ed_status ed_model_plan_key(const ed_model* model, char* buf, int buf_len) {
    if (!model || !buf || buf_len < 1) return ed::fail(ED_ERR_ARG, "null argument");
    const std::string k = ed::plan_key(model);
    if (int(k.size()) >= buf_len) return ed::fail(ED_ERR_ARG, "buffer too small for the plan key");
    std::memcpy(buf, k.c_str(), k.size() + 1);
    return ED_OK;
}

ed_status ed_plan_cache_put(const char* key, const char* plan) {
    if (!key || !plan || !*key || !*plan) return ed::fail(ED_ERR_ARG, "empty key or plan");
    if (std::strpbrk(key, "\t\n") || std::strpbrk(plan, "\t\n"))
        return ed::fail(ED_ERR_ARG, "key and plan may not contain tabs or newlines");
    ed::PlanCache& pc = ed::plan_cache();
    std::lock_guard<std::mutex> lock(pc.mu);
    pc.map[key] = plan;
    return ED_OK;
}

ed_status ed_plan_cache_get(const char* key, char* buf, int buf_len) {
    if (!key || !buf || buf_len < 1) return ed::fail(ED_ERR_ARG, "null argument");
    ed::PlanCache& pc = ed::plan_cache();
    std::lock_guard<std::mutex> lock(pc.mu);
    auto it = pc.map.find(key);
    if (it == pc.map.end()) return ed::fail(ED_ERR_ARG, std::string("no cached plan for key '") + key + "'");
    if (int(it->second.size()) >= buf_len) return ed::fail(ED_ERR_ARG, "buffer too small for the plan");
    std::memcpy(buf, it->second.c_str(), it->second.size() + 1);
    return ED_OK;
}

ed_status ed_plan_cache_clear(void) {
    ed::PlanCache& pc = ed::plan_cache();
    std::lock_guard<std::mutex> lock(pc.mu);
    pc.map.clear();
    return ED_OK;
}

ed_status ed_plan_cache_load(const char* path, int* entries) {
    if (!path) return ed::fail(ED_ERR_ARG, "path is null");
    std::ifstream f(path);
    if (!f) return ed::fail(ED_ERR_ARG, std::string("cannot read plan cache ") + path);
    std::string line;
    int n = 0, lineno = 0;
    std::map<std::string, std::string> add;
    while (std::getline(f, line)) {
        ++lineno;
        if (line.empty() || line[0] == '#') continue;
        const size_t tab = line.find('\t');
        if (tab == std::string::npos || tab == 0 || tab + 1 >= line.size())
            return ed::fail(ED_ERR_ARG, std::string(path) + ":" + std::to_string(lineno) + ": expected <key>\\t<plan>");
        add[line.substr(0, tab)] = line.substr(tab + 1);
        ++n;
    }
    ed::PlanCache& pc = ed::plan_cache();
    std::lock_guard<std::mutex> lock(pc.mu);
    for (auto& kv : add) pc.map[kv.first] = kv.second;
    if (entries) *entries = n;
    return ED_OK;
}

ed_status ed_plan_cache_save(const char* path) {
    if (!path) return ed::fail(ED_ERR_ARG, "path is null");
    std::ostringstream o;
    o << "# libed tuned H psi plans: <GPU arch, L, operator class, flags, candidate-list hash> TAB <plan>\n";
    {
        ed::PlanCache& pc = ed::plan_cache();
        std::lock_guard<std::mutex> lock(pc.mu);
        for (auto& kv : pc.map) o << kv.first << '\t' << kv.second << '\n';
    }
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return ed::fail(ED_ERR_ARG, std::string("cannot write ") + tmp);
        f << o.str();
        if (!f) return ed::fail(ED_ERR_ARG, std::string("write failed: ") + tmp);
    }
    if (std::rename(tmp.c_str(), path) != 0) return ed::fail(ED_ERR_ARG, std::string("cannot replace ") + path);
    return ED_OK;
}

ed_status ed_model_tune(ed_model* model, const ed_c64* psi, ed_c64* out, int reps, void* stream, int* best,
                        float* times_ms) {
    if (!model || !psi || !out) return ed::fail(ED_ERR_ARG, "null argument");
    if (reps < 1) return ed::fail(ED_ERR_ARG, "reps must be >= 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    ED_HIP_TRY(hipEventCreate(&e0));
    ED_HIP_TRY(hipEventCreate(&e1));
    int arg = 0;
    float best_ms = 0.0f;
    ed_status st = ED_OK;
    for (int c = 0; c < model->n_cand && st == ED_OK; ++c) {
        ed_model_select_plan(model, c);
        st = ed_apply_H(model, psi, out, stream);  // warm-up
        if (st != ED_OK) break;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && st == ED_OK; ++r) st = ed_apply_H(model, psi, out, stream);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= float(reps);
        if (times_ms) times_ms[c] = ms;
        if (c == 0 || ms < best_ms) {
            best_ms = ms;
            arg = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ED_TRY(st);
    ed_model_select_plan(model, arg);
    ed::remember_plan(model);
    if (best) *best = arg;
    return ED_OK;
}

ed_status ed_apply_H(const ed_model* model, const ed_c64* psi, ed_c64* out, void* stream) {
    if (!model || !psi || !out) return ed::fail(ED_ERR_ARG, "null argument");
    const int64_t D = int64_t(1) << model->L;
    const char* a = reinterpret_cast<const char*>(psi);
    const char* b = reinterpret_cast<const char*>(out);
    if (a < b + D * 16 && b < a + D * 16) return ed::fail(ED_ERR_ARG, "psi and out overlap");
    return ed::launch_apply_H(model, reinterpret_cast<const double2*>(psi), reinterpret_cast<double2*>(out),
                              static_cast<hipStream_t>(stream));
}

}  // extern "C"
