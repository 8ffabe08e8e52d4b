// Gradient of a final-time observable with respect to piecewise-constant bond couplings, by
// costate (adjoint) back-propagation through the Krylov time evolution of Sec. ed:sec:krylov.
//
//   H_s = sum_b J[s][b] h_b + H_site    (h_b: the template's bond operator on bond b)
//   psi_s = exp(-i H_s Delta) psi_{s-1},  Loss = <psi_S|O|psi_S>,  O = sum_k w_k sigma^z_k
//   lam_S = O psi_S,  lam_{s-1} = exp(+i H_s Delta) lam_s
//   dLoss/dJ[s][b] = 2 int_0^Delta Im <mu(tau)| h_b |phi(tau)> dtau,
//       phi(tau) = exp(-i H_s tau) psi_{s-1},  mu(tau) = exp(-i H_s tau) lam_{s-1}.
// The forward pass stores psi_s at every slice boundary (checkpoints). The backward pass
// propagates the costate one slice back, then walks the slice in sub-steps: a Krylov basis of
// phi and of mu at the sub-step start gives both at every Gauss-Legendre node, and one fused
// pass per node returns Im<mu|h_b|phi> for every bond at once.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "dense.h"
#include "ed_vec.h"
#include "hpsi_device.h"
#include "krylov_core.h"

namespace ed {

ed_status create_model(const ed_model_desc* desc, ed_model** out);
void destroy_model(ed_model* m);

namespace {

constexpr int kBT = 256;
constexpr int kMaxBonds = 31;

// part[blk][b] = sum_{x in block} conj(mu[x]) (h_b phi)[x] for every bond bit p = 0..L-2
// (bond ops per bit in `bond`, 16 entries each). Partner amplitudes come straight from global
// memory: the vectors of this path (L <= 24) live in the last-level cache.
__global__ __launch_bounds__(kBT) void bond_expect_partial(const double2* __restrict__ mu, const double2* __restrict__ phi,
                                                           const double2* __restrict__ bond, int L,
                                                           double2* __restrict__ part, int part_ld) {
    __shared__ double red[kBT / 64][2 * kMaxBonds];
    double a[2 * kMaxBonds];
#pragma unroll
    for (int i = 0; i < 2 * kMaxBonds; ++i) a[i] = 0.0;
    const int64_t D = int64_t(1) << L;
    const int64_t chunk = (D + gridDim.x - 1) / gridDim.x;
    const int64_t lo = int64_t(blockIdx.x) * chunk;
    const int64_t hi = lo + chunk < D ? lo + chunk : D;
    for (int64_t x = lo + threadIdx.x; x < hi; x += kBT) {
        const double2 m = mu[x];
        const double2 f = phi[x];
#pragma unroll
        for (int p = 0; p < kMaxBonds; ++p) {
            if (p + 1 < L) {
                const int l = (x >> p) & 3;
                const double2* B = bond + 16 * p;
                double2 hv = cmul(B[5 * l], f);
#pragma unroll
                for (int mm = 1; mm < 4; ++mm) {
                    const double2 c = B[4 * l + (l ^ mm)];
                    if (c.x != 0.0 || c.y != 0.0) {
                        const double2 g = phi[x ^ (int64_t(mm) << p)];
                        hv.x += c.x * g.x - c.y * g.y;
                        hv.y += c.x * g.y + c.y * g.x;
                    }
                }
                // conj(m) * hv
                a[2 * p] += m.x * hv.x + m.y * hv.y;
                a[2 * p + 1] += m.x * hv.y - m.y * hv.x;
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 2 * kMaxBonds; ++i) {
        double v = a[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[wv][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < 2 * (L - 1)) {
        double s = 0.0;
        for (int w = 0; w < kBT / 64; ++w) s += red[w][threadIdx.x];
        reinterpret_cast<double*>(part + int64_t(blockIdx.x) * part_ld)[threadIdx.x] = s;
    }
}

// out[x] = (sum_k w_k (1 - 2 bit_{L-k}(x))) psi[x]   (O = sum_k w_k sigma^z_k, diagonal)
__global__ __launch_bounds__(kBT) void apply_zobs(const double2* __restrict__ psi, double2* __restrict__ out, int L,
                                                 const double* __restrict__ w) {
    const int64_t D = int64_t(1) << L;
    const int64_t stride = int64_t(gridDim.x) * kBT;
    for (int64_t x = int64_t(blockIdx.x) * kBT + threadIdx.x; x < D; x += stride) {
        double o = 0.0;
        for (int k = 1; k <= L; ++k) o += ((x >> (L - k)) & 1) ? -w[k - 1] : w[k - 1];
        const double2 y = psi[x];
        out[x] = make_double2(o * y.x, o * y.y);
    }
}

// __global__ reduce of the partials lives in vec.hip; reuse through the public launchers
}  // namespace

hipError_t bond_expect(const double2* mu, const double2* phi, const double2* bond, int L, double2* out,
                       double2* part, hipStream_t s);

// Gauss-Legendre nodes x_q in (-1, 1) and weights, by Newton iteration on P_n (from the
// three-term recurrence of the Legendre polynomials).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                const double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            const double z1 = z;
            z = z1 - p1 / pp;
            if (std::fabs(z - z1) < 1e-16) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
        w[n - 1 - i] = w[i];
    }
}

namespace {

struct ModelSet {
    std::vector<ed_model*> m;
    ~ModelSet() {
        for (ed_model* x : m) destroy_model(x);
    }
};

// H_s from the template: its folded site operators unchanged, bond operator of bond b (sites
// b+1, b+2) scaled by J[s][b].
ed_status slice_models(const ed_model* tmpl, int S, const double* J, ModelSet* ms) {
    const int L = tmpl->L;
    std::vector<ed_c64> sop(4 * L), bop(16 * (L - 1));
    std::vector<double> scoef(size_t(L) * L, 0.0), bcoef(size_t(L - 1) * (L - 1), 0.0);
    for (int k = 1; k <= L; ++k) {
        const int p = L - k;
        for (int e = 0; e < 4; ++e) sop[4 * (k - 1) + e] = ed_c64{tmpl->site[4 * p + e].x, tmpl->site[4 * p + e].y};
        scoef[size_t(k - 1) * L + (k - 1)] = 1.0;
    }
    for (int k = 1; k <= L - 1; ++k) {
        const int p = L - k - 1;
        for (int e = 0; e < 16; ++e) bop[16 * (k - 1) + e] = ed_c64{tmpl->bond[16 * p + e].x, tmpl->bond[16 * p + e].y};
    }
    for (int s = 0; s < S; ++s) {
        for (int b = 0; b < L - 1; ++b) bcoef[size_t(b) * (L - 1) + b] = J[size_t(s) * (L - 1) + b];
        ed_model_desc d{L, 2, L, sop.data(), scoef.data(), L - 1, bop.data(), bcoef.data()};
        ed_model* m = nullptr;
        ED_TRY(create_model(&d, &m));
        ms->m.push_back(m);
    }
    return ED_OK;
}

struct Basis {
    Workspace w;
    std::vector<xreal> d, Z;  // eigenpairs of the tridiagonal T (extended precision)
    int m = 0;
    double nrm = 0.0;
};

// Lanczos basis of psi under model (three-term recurrence with local re-projection, or fixed m)
ed_status build_basis(const ed_model* mod, const double2* psi, double dt_err, const ed_adjoint_params* p, Basis* B,
                      hipStream_t s) {
    ED_TRY(start_vector(B->w, psi, &B->nrm, s));
    const int mmax = p->m_max;
    std::vector<double> a(mmax + 1), b(mmax + 1);
    std::vector<cplx> h(mmax + 2);
    int m = 0;
    for (int j = 0; j < mmax; ++j) {
        const int lo = std::max(j - 1, 0);
        double beta = 0.0;
        bool brk = false;
        // both projections swept (local re-projection): the bases run at a fixed dimension well
        // past convergence, where the gradient check needs the more orthogonal basis
        ED_TRY(krylov_step(mod, B->w, j, lo, 1, 1e-14, h.data(), &beta, &brk, s));
        a[j] = h[j - lo].real();
        m = j + 1;
        bool stop = brk || m >= mmax;
        if (p->m_fixed > 0) {
            stop = brk || m >= std::min(p->m_fixed, mmax);
        } else if (!stop) {
            std::vector<xreal> dd(a.begin(), a.begin() + m), ee(m, 0.0L), Z(size_t(m) * m, 0.0L);
            for (int i = 0; i + 1 < m; ++i) ee[i] = b[i];
            for (int i = 0; i < m; ++i) Z[size_t(i) * m + i] = 1.0L;
            if (!tridiag_ql_ext(m, dd.data(), ee.data(), Z.data()))
                return fail(ED_ERR_NUMERIC, "tridiagonal eigensolver did not converge");
            std::vector<cplx> u(m);
            expm_col_sym_ext(m, dd.data(), Z.data(), std::fabs(dt_err), u.data());
            stop = B->nrm * beta * std::abs(u[m - 1]) <= p->tol;
        }
        if (stop) break;
        b[j] = beta;
    }
    B->m = m;
    B->d.assign(a.begin(), a.begin() + m);
    std::vector<xreal> ee(m, 0.0L);
    for (int i = 0; i + 1 < m; ++i) ee[i] = b[i];
    B->Z.assign(size_t(m) * m, 0.0L);
    for (int i = 0; i < m; ++i) B->Z[size_t(i) * m + i] = 1.0L;
    if (!tridiag_ql_ext(m, B->d.data(), ee.data(), B->Z.data()))
        return fail(ED_ERR_NUMERIC, "tridiagonal eigensolver did not converge");
    return ED_OK;
}

// out = nrm V exp(-i tau T) e_1
ed_status eval_basis(const Basis& B, double tau, double2* out, hipStream_t s) {
    std::vector<cplx> u(B.m);
    expm_col_sym_ext(B.m, B.d.data(), B.Z.data(), tau, u.data());
    std::vector<double2> c(B.m);
    for (int i = 0; i < B.m; ++i) c[i] = make_double2(B.nrm * u[i].real(), B.nrm * u[i].imag());
    return combine_basis(B.w, B.m, c.data(), out, s);
}

// psi <- exp(-i H dt) psi through K sub-steps
ed_status propagate(const ed_model* mod, double2* psi, double dt, int K, const ed_adjoint_params* p, Basis* B,
                    hipStream_t s) {
    for (int k = 0; k < K; ++k) {
        ED_TRY(build_basis(mod, psi, dt / K, p, B, s));
        ED_TRY(eval_basis(*B, dt / K, psi, s));
    }
    return ED_OK;
}

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

ed_status check_params(const ed_model* tmpl, int S, double Delta, const double* J, const ed_c64* psi0, const double* w,
                       const ed_adjoint_params* p) {
    if (tmpl && tmpl->lr) return fail(ED_ERR_UNSUPPORTED, "the adjoint does not take long-range (InfiniteFunc) terms");
    if (tmpl && tmpl->lv_L > 0) return fail(ED_ERR_UNSUPPORTED, "the adjoint does not take Liouvillian models");
    if (!tmpl || !J || !psi0 || !w || !p) return fail(ED_ERR_ARG, "null argument");
    if (S < 1 || !(Delta > 0.0)) return fail(ED_ERR_ARG, "n_slices >= 1 and slice_len > 0 required");
    if (tmpl->L > 24) return fail(ED_ERR_UNSUPPORTED, "the adjoint path supports L <= 24");
    if (p->substeps < 1 || p->quad_nodes < 1 || p->quad_nodes > 64) return fail(ED_ERR_ARG, "bad substeps / quad_nodes");
    if (p->m_max < 2 || p->m_max > 64) return fail(ED_ERR_ARG, "m_max must be in [2, 64]");
    if (p->m_fixed <= 0 && !(p->tol > 0.0)) return fail(ED_ERR_ARG, "tol must be > 0");
    for (int i = 0; i < S * (tmpl->L - 1); ++i)
        if (!std::isfinite(J[i])) return fail(ED_ERR_NUMERIC, "non-finite coupling");
    return ED_OK;
}

ed_status loss_of(const double2* psi, int L, const double* w, const Workspace& ws, double* loss, hipStream_t s) {
    std::vector<double> sz(L);
    double nrm = 0.0;
    ED_TRY(measure_state(psi, L, ws, sz.data(), &nrm, s));
    double acc = 0.0;
    for (int k = 0; k < L; ++k) acc += w[k] * sz[k];
    *loss = acc * nrm * nrm;
    return ED_OK;
}

}  // namespace
}  // namespace ed

using namespace ed;

extern "C" ed_status ed_adjoint_workspace(const ed_model* tmpl, int n_slices, const ed_adjoint_params* p, size_t* bytes) {
    if (!tmpl || !p || !bytes || n_slices < 1) return fail(ED_ERR_ARG, "bad argument");
    const int64_t D = int64_t(1) << tmpl->L;
    const size_t vec = size_t(D) * sizeof(double2);
    // two bases (phi, mu) of m_max + 1 vectors, checkpoints S + 1, lambda, 2 node vectors, w (L doubles)
    *bytes = 2 * (core_scratch_bytes() + al(size_t(p->m_max + 1) * vec)) + al(size_t(n_slices + 1) * vec) + 3 * al(vec) +
             al(64 * sizeof(double));
    return ED_OK;
}

extern "C" ed_status ed_evolve_adjoint(const ed_model* tmpl, int n_slices, double slice_len, const double* J,
                                      const ed_c64* psi0, const double* obs_w, const ed_adjoint_params* p,
                                      double* loss, double* grad, void* ws, size_t ws_bytes, void* stream) {
    ED_TRY(check_params(tmpl, n_slices, slice_len, J, psi0, obs_w, p));
    if (!loss || !grad) return fail(ED_ERR_ARG, "null output");
    size_t need = 0;
    ED_TRY(ed_adjoint_workspace(tmpl, n_slices, p, &need));
    if (!ws) return fail(ED_ERR_ARG, "workspace is null");
    if (ws_bytes < need) return fail(ED_ERR_WORKSPACE, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int L = tmpl->L, S = n_slices, NB = L - 1;
    const int64_t D = int64_t(1) << L;
    const size_t vec = size_t(D) * sizeof(double2);
    char* c = static_cast<char*>(ws);
    Basis Bp, Bm;
    const size_t basis_bytes = core_scratch_bytes() + al(size_t(p->m_max + 1) * vec);
    ED_TRY(carve(c, basis_bytes, D, p->m_max + 1, &Bp.w));
    c += basis_bytes;
    ED_TRY(carve(c, basis_bytes, D, p->m_max + 1, &Bm.w));
    c += basis_bytes;
    double2* ck = reinterpret_cast<double2*>(c);
    c += al(size_t(S + 1) * vec);
    double2* lam = reinterpret_cast<double2*>(c);
    c += al(vec);
    double2* phin = reinterpret_cast<double2*>(c);
    c += al(vec);
    double2* mun = reinterpret_cast<double2*>(c);
    c += al(vec);
    double* dw = reinterpret_cast<double*>(c);

    ModelSet ms;
    ED_TRY(slice_models(tmpl, S, J, &ms));
    const int K = p->substeps;
    // forward with checkpoints
    ED_HIP_TRY(hipMemcpyAsync(ck, psi0, vec, hipMemcpyDeviceToDevice, s));
    for (int sl = 0; sl < S; ++sl) {
        double2* nxt = ck + int64_t(sl + 1) * D;
        ED_HIP_TRY(hipMemcpyAsync(nxt, ck + int64_t(sl) * D, vec, hipMemcpyDeviceToDevice, s));
        ED_TRY(propagate(ms.m[sl], nxt, slice_len, K, p, &Bp, s));
    }
    ED_TRY(loss_of(ck + int64_t(S) * D, L, obs_w, Bp.w, loss, s));
    // costate lam_S = O psi_S
    ED_HIP_TRY(hipMemcpyAsync(dw, obs_w, sizeof(double) * L, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(apply_zobs, dim3(unsigned(std::min<int64_t>((D + kBT - 1) / kBT, 4096))), dim3(kBT), 0, s,
                       ck + int64_t(S) * D, lam, L, dw);
    ED_HIP_TRY(hipGetLastError());
    std::vector<double> xq, wq;
    gauss_legendre(p->quad_nodes, xq, wq);
    const double delta = slice_len / K;
    std::vector<double2> z(NB);
    for (int sl = S - 1; sl >= 0; --sl) {
        const ed_model* Hs = ms.m[sl];
        // lam_{s-1} = exp(+i H_s Delta) lam_s
        ED_TRY(propagate(Hs, lam, -slice_len, K, p, &Bm, s));
        // walk the slice: phi from the checkpoint, mu from lam_{s-1}
        ED_HIP_TRY(hipMemcpyAsync(phin, ck + int64_t(sl) * D, vec, hipMemcpyDeviceToDevice, s));
        ED_HIP_TRY(hipMemcpyAsync(mun, lam, vec, hipMemcpyDeviceToDevice, s));
        std::vector<double> g(NB, 0.0);
        for (int k = 0; k < K; ++k) {
            ED_TRY(build_basis(Hs, phin, delta, p, &Bp, s));
            ED_TRY(build_basis(Hs, mun, delta, p, &Bm, s));
            for (int q = 0; q < p->quad_nodes; ++q) {
                const double sig = 0.5 * delta * (1.0 + xq[q]);
                ED_TRY(eval_basis(Bp, sig, phin, s));
                ED_TRY(eval_basis(Bm, sig, mun, s));
                if (bond_expect(mun, phin, tmpl->d_bond, L, Bp.w.scal + kObs, Bp.w.part, s) != hipSuccess)
                    return fail(ED_ERR_HIP, "bond reduction");
                ED_TRY(fetch_scalars(Bp.w.scal + kObs, NB, z.data(), s));
                // bond bit p = L - b - 2 for bond b (sites b+1, b+2)
                for (int b = 0; b < NB; ++b) g[b] += 0.5 * delta * wq[q] * 2.0 * z[L - b - 2].y;
            }
            // advance phi and mu to the end of the sub-step
            ED_TRY(eval_basis(Bp, delta, phin, s));
            ED_TRY(eval_basis(Bm, delta, mun, s));
        }
        for (int b = 0; b < NB; ++b) grad[size_t(sl) * NB + b] = g[b];
    }
    ED_HIP_TRY(hipStreamSynchronize(s));
    return ED_OK;
}

extern "C" ed_status ed_evolve_loss_workspace(const ed_model* tmpl, const ed_adjoint_params* p, size_t* bytes) {
    if (!tmpl || !p || !bytes) return fail(ED_ERR_ARG, "bad argument");
    const int64_t D = int64_t(1) << tmpl->L;
    *bytes = core_scratch_bytes() + al(size_t(p->m_max + 1) * size_t(D) * sizeof(double2)) + al(size_t(D) * sizeof(double2));
    return ED_OK;
}

extern "C" ed_status ed_evolve_loss(const ed_model* tmpl, int n_slices, double slice_len, const double* J,
                                   const ed_c64* psi0, const double* obs_w, const ed_adjoint_params* p, double* loss,
                                   void* ws, size_t ws_bytes, void* stream) {
    ED_TRY(check_params(tmpl, n_slices, slice_len, J, psi0, obs_w, p));
    if (!loss) return fail(ED_ERR_ARG, "null output");
    size_t need = 0;
    ED_TRY(ed_evolve_loss_workspace(tmpl, p, &need));
    if (!ws) return fail(ED_ERR_ARG, "workspace is null");
    if (ws_bytes < need) return fail(ED_ERR_WORKSPACE, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int L = tmpl->L;
    const int64_t D = int64_t(1) << L;
    Basis B;
    const size_t basis_bytes = core_scratch_bytes() + al(size_t(p->m_max + 1) * size_t(D) * sizeof(double2));
    ED_TRY(carve(ws, basis_bytes, D, p->m_max + 1, &B.w));
    double2* psi = reinterpret_cast<double2*>(static_cast<char*>(ws) + basis_bytes);
    ModelSet ms;
    ED_TRY(slice_models(tmpl, n_slices, J, &ms));
    ED_HIP_TRY(hipMemcpyAsync(psi, psi0, size_t(D) * sizeof(double2), hipMemcpyDeviceToDevice, s));
    for (int sl = 0; sl < n_slices; ++sl) ED_TRY(propagate(ms.m[sl], psi, slice_len, p->substeps, p, &B, s));
    ED_TRY(loss_of(psi, L, obs_w, B.w, loss, s));
    return ED_OK;
}

namespace ed {
hipError_t bond_expect(const double2* mu, const double2* phi, const double2* bond, int L, double2* out, double2* part,
                       hipStream_t s) {
    const int64_t D = int64_t(1) << L;
    int G = reduction_blocks(D);
    hipLaunchKernelGGL(bond_expect_partial, dim3(G), dim3(kBT), 0, s, mu, phi, bond, L, part, kPartLd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_partial_rows(part, G, L - 1, out, s);
}
}  // namespace ed
