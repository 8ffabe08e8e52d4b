// Krylov machinery on top of H psi (Sec. ed:sec:krylov): the basis recurrence shared by the Lanczos
// ground state and the Krylov time step, the thick-restart ground-state driver, the time
// evolution driver with per-step observables, and the one-pass measurement.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "dense.h"
#include "ed_vec.h"
#include "krylov_core.h"

namespace ed {

// ------------------------------------------------------------------------ workspace layout
static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

size_t core_scratch_bytes() { return align_up(kPartBytes) + align_up(sizeof(double2) * kScalars); }

ed_status carve(void* ws, size_t ws_bytes, int64_t D, int nvec, Workspace* w) {
    const size_t need = core_scratch_bytes() + align_up(size_t(nvec) * size_t(D) * sizeof(double2));
    if (!ws) return fail(ED_ERR_ARG, "workspace is null");
    if (ws_bytes < need)
        return fail(ED_ERR_WORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes < required " +
                                          std::to_string(need));
    char* p = static_cast<char*>(ws);
    w->part = reinterpret_cast<double2*>(p);
    p += align_up(kPartBytes);
    w->scal = reinterpret_cast<double2*>(p);
    p += align_up(sizeof(double2) * kScalars);
    w->V = reinterpret_cast<double2*>(p);
    w->nvec = nvec;
    w->D = D;
    return ED_OK;
}

// Pinned host staging buffer for the per-iteration scalars: allocated on a thread's first use and
// freed when that thread ends (thread-local objects of the main thread are destroyed before the
// runtime's static state).
namespace {
struct HostStage {
    double2* buf = nullptr;
    ~HostStage() {
        if (buf) (void)hipHostFree(buf);
    }
};
}  // namespace

double2* host_stage() {
    static thread_local HostStage st;
    if (!st.buf) {
        if (hipHostMalloc(reinterpret_cast<void**>(&st.buf), sizeof(double2) * kScalars) != hipSuccess) st.buf = nullptr;
    }
    return st.buf;
}

ed_status fetch_scalars(const double2* dev, int n, double2* host, hipStream_t s) {
    double2* st = host_stage();
    if (!st) return fail(ED_ERR_NOMEM, "pinned host buffer");
    ED_HIP_TRY(hipMemcpyAsync(st, dev, sizeof(double2) * n, hipMemcpyDeviceToHost, s));
    ED_HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(host, st, sizeof(double2) * n);
    return ED_OK;
}

#define ED_K(expr)                                                                           \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess) return fail(ED_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

// One step of the recurrence on the scaled basis: y = H u_j into slot j+1, orthogonalised against
// u_lo..u_j by classical Gram-Schmidt once (dots, then subtraction + norm) or twice (dots; the
// first subtraction together with the second pass's dots; subtraction + norm). With beta_prev
// (Hermitian H), the first pass's projections on v_{j-1} and v_j are beta_{j-1} and the sum the
// product's last pass leaves per tile, so that pass needs no dot sweep. Returns the true
// projections h_i = <v_i|H v_j> (i = lo..j) and the norm beta of the orthogonalised H v_j; the new
// basis vector is u_{j+1} = y with c_{j+1} = 1/|y|.
ed_status krylov_step(const ed_model* m, const Workspace& w, int j, int lo, int passes, double tiny_rel,
                      cplx* h, double* beta, bool* breakdown, hipStream_t s, int first_lo, double beta_prev,
                      const double* known) {
    const int64_t D = w.D;
    const int n = j - lo + 1;
    if (n > kMaxProj) return fail(ED_ERR_UNSUPPORTED, "too many projections");
    if (int(w.u.size()) < j + 2) {
        w.u.resize(j + 2, nullptr);
        w.c.resize(j + 2, 0.0);
    }
    double2* y = w.slot(j + 1);
    // Hermitian three-term recurrence (n = 2), or its first step (j = 0, n = 1: <v_0|H v_0> only)
    const bool three_term = passes == 1 && beta_prev >= 0.0 && ((n == 2 && lo == j - 1) || (n == 1 && j == 0));
    // CGS2 whose first pass takes only v_{j-1}, v_j: that pass's projections are beta_{j-1} and
    // <v_j|H v_j> as well (the second pass takes the whole basis)
    const bool local_first = passes > 1 && first_lo == j - 1 && first_lo > lo && beta_prev >= 0.0;
    const bool known_first = known && passes > 1 && lo == 0 && first_lo < 0;
    int64_t nparts = 0;
    if (three_term || local_first || known_first) {
        // the product's last pass also leaves per-tile partials of <u_j|y> in the partial buffer
        ED_TRY(launch_apply_H_dot(m, w.u[j], y, w.part, int64_t(kPartBytes / sizeof(double2)), &nparts, s));
    } else {
        ED_TRY(launch_apply_H(m, w.u[j], y, s));
    }
    double2* nr = w.scal + kNrm;
    double2* g1 = w.scal + 1;
    double2* g2 = w.scal + 1 + n;
    const double2* const* U = const_cast<const double2* const*>(w.u.data() + lo);
    std::vector<double> sc(n);
    for (int i = 0; i < n; ++i) sc[i] = w.c[lo + i] * w.c[lo + i];
    if (three_term) {
        // <u_{j-1}|y> = beta_{j-1} / (c_{j-1} c_j) for a Hermitian H; <u_j|y> from the product's
        // partials, or one dot sweep
        if (n == 2) ED_K(set_scalar(g1, make_double2(beta_prev / (w.c[lo] * w.c[j]), 0.0), s));
        if (nparts > 0) ED_K(sum_partials(w.part, nparts, g1 + (n - 1), s));
        else ED_K(dots_ptr(U + (n - 1), 1, y, D, g1 + (n - 1), w.part, s));
    } else if (known_first) {
        // <u_i|y> = h_i / (c_i c_j) for the known projections; <u_j|y> from the product
        std::vector<double2> gk(n - 1);
        for (int i = 0; i + 1 < n; ++i) gk[i] = make_double2(known[i] / (w.c[i] * w.c[j]), 0.0);
        for (int i = 0; i + 1 < n; ++i) ED_K(set_scalar(g1 + i, gk[i], s));
        if (nparts > 0) ED_K(sum_partials(w.part, nparts, g1 + (n - 1), s));
        else ED_K(dots_ptr(U + (n - 1), 1, y, D, g1 + (n - 1), w.part, s));
    } else if (local_first) {
        ED_HIP_TRY(hipMemsetAsync(g1, 0, sizeof(double2) * size_t(n - 2), s));
        ED_K(set_scalar(g1 + (n - 2), make_double2(beta_prev / (w.c[j - 1] * w.c[j]), 0.0), s));
        if (nparts > 0) ED_K(sum_partials(w.part, nparts, g1 + (n - 1), s));
        else ED_K(dots_ptr(U + (n - 1), 1, y, D, g1 + (n - 1), w.part, s));
    } else if (passes > 1 && first_lo > lo) {
        // the recurrence's own vectors first; the other coefficients of the first pass are zero
        const int nf = j - first_lo + 1;
        ED_HIP_TRY(hipMemsetAsync(g1, 0, sizeof(double2) * size_t(n - nf), s));
        ED_K(dots_ptr(U + (n - nf), nf, y, D, g1 + (n - nf), w.part, s));
    } else {
        ED_K(dots_ptr(U, n, y, D, g1, w.part, s));
    }
    // Plain CGS2 (both passes over lo..j): the second pass runs only when the first removed more
    // than half of the squared norm (the DGKS test |y'| < |y| / sqrt(2), with |y|^2 = |y'|^2 +
    // sum_i |<v_i|y>|^2 taken from the first pass's projections). Otherwise y' is orthogonal to the
    // basis to working precision already.
    const bool plain2 = passes > 1 && !local_first && !known_first && first_lo <= lo;
    bool second = passes > 1;
    if (plain2) {
        int nd = 0;
        ED_K(axpy_dots_norm_ptr(U, n, g1, sc.data(), y, D, g2, nr, &nd, w.part, s));
        std::vector<double2> h1(1 + n);
        ED_TRY(fetch_scalars(w.scal, 1 + n, h1.data(), s));
        double removed = 0.0;
        for (int i = 0; i < n; ++i) removed += sc[i] * (h1[1 + i].x * h1[1 + i].x + h1[1 + i].y * h1[1 + i].y);
        second = !(h1[kNrm].x >= removed);
        if (second) {
            if (nd < n) ED_K(dots_ptr(U + nd, n - nd, y, D, g2 + nd, w.part, s));
            ED_K(axpy_norm_ptr(U, n, g2, sc.data(), y, D, nr, w.part, s));
        } else if (w.cgs_skipped) {
            ++*w.cgs_skipped;
        }
    } else if (passes > 1) {
        // the first subtraction and the second pass's dots share a sweep
        ED_K(axpy_dots_ptr(U, n, g1, sc.data(), y, D, g2, w.part, s));
        ED_K(axpy_norm_ptr(U, n, g2, sc.data(), y, D, nr, w.part, s));
    } else {
        ED_K(axpy_norm_ptr(U, n, g1, sc.data(), y, D, nr, w.part, s));
    }
    std::vector<double2> hs(1 + 2 * n);
    ED_TRY(fetch_scalars(w.scal, second ? 1 + 2 * n : 1 + n, hs.data(), s));
    const double cj = w.c[j];
    for (int i = 0; i < n; ++i) {
        cplx g(hs[1 + i].x, hs[1 + i].y);
        if (second) g += cplx(hs[1 + n + i].x, hs[1 + n + i].y);
        h[i] = w.c[lo + i] * cj * g;
    }
    const double nrm2v = hs[kNrm].x;
    if (!std::isfinite(nrm2v)) return fail(ED_ERR_NUMERIC, "non-finite value in the Krylov recurrence");
    const double ny = std::sqrt(std::max(nrm2v, 0.0));
    *beta = cj * ny;
    double hmax = 0.0;
    for (int i = 0; i < n; ++i) hmax = std::max(hmax, std::abs(h[i]));
    *breakdown = (*beta <= tiny_rel * std::max(hmax, 1e-300)) || *beta == 0.0;
    w.u[j + 1] = y;
    w.c[j + 1] = *breakdown ? 0.0 : 1.0 / ny;
    // |u_{j+1}| = |y| grows like the product of the betas over a run of steps; keep it inside a
    // safe exponent range so long recurrences (and vectors carried across restarts) never
    // overflow: rescale in memory, which is rare (one pass every few dozen steps at most).
    if (!*breakdown && (ny > 1e100 || ny < 1e-100)) {
        ED_K(scale(y, y, make_double2(1.0 / ny, 0.0), D, s));
        w.c[j + 1] = 1.0;
    }
    return ED_OK;
}

ed_status start_vector(const Workspace& w, const double2* psi, double* nrm, hipStream_t s, bool alias) {
    double2* nr = w.scal + kNrm;
    ED_K(norm2(psi, w.D, nr, w.part, s));
    double2 hv[1];
    ED_TRY(fetch_scalars(w.scal, 1, hv, s));
    const double n2 = hv[kNrm].x;
    if (!std::isfinite(n2)) return fail(ED_ERR_NUMERIC, "non-finite start vector");
    if (n2 <= 0.0) return fail(ED_ERR_ARG, "start vector is zero");
    *nrm = std::sqrt(n2);
    if (w.u.empty()) {
        w.u.resize(1);
        w.c.resize(1);
    }
    if (alias) {
        w.u[0] = const_cast<double2*>(psi);
        w.c[0] = 1.0 / *nrm;
    } else {
        ED_K(normalize(psi, w.V, nr, w.D, s));
        w.u[0] = w.V;
        w.c[0] = 1.0;
    }
    return ED_OK;
}

// One step of the Lanczos recurrence with partial reorthogonalisation: y = H u_j into slot j+1,
// projected on v_{j-1} and v_j (the three-term recurrence: beta_{j-1} is known and <v_j|H v_j> comes
// from the product's last pass) and, by one classical Gram-Schmidt pass computed from the same y, on
// the nk kept Ritz vectors u_0..u_{nk-1} of a thick restart (the directions in which new vectors
// lose orthogonality fastest). Returns alpha_j = <v_j|H v_j> and beta_j = |orthogonalised H v_j|.
ed_status lanczos_local_step(const ed_model* m, const Workspace& w, int j, int nk, double beta_prev, double* alpha,
                             double* beta, bool* breakdown, hipStream_t s) {
    const int64_t D = w.D;
    if (nk + 2 > kMaxProj) return fail(ED_ERR_UNSUPPORTED, "too many kept vectors");
    if (int(w.u.size()) < j + 2) {
        w.u.resize(j + 2, nullptr);
        w.c.resize(j + 2, 0.0);
    }
    double2* y = w.slot(j + 1);
    int64_t nparts = 0;
    ED_TRY(launch_apply_H_dot(m, w.u[j], y, w.part, int64_t(kPartBytes / sizeof(double2)), &nparts, s));
    const int n = nk + 2;
    std::vector<const double2*> U(n);
    std::vector<double> sc(n);
    for (int i = 0; i < nk; ++i) U[i] = w.u[i];
    U[nk] = w.u[j - 1];
    U[nk + 1] = w.u[j];
    for (int i = 0; i < nk; ++i) sc[i] = w.c[i] * w.c[i];
    sc[nk] = w.c[j - 1] * w.c[j - 1];
    sc[nk + 1] = w.c[j] * w.c[j];
    double2* nr = w.scal + kNrm;
    double2* g = w.scal + 1;
    // <u_j|y> from the product's partials first (the dots below reuse the partial buffer)
    if (nparts > 0) ED_K(sum_partials(w.part, nparts, g + nk + 1, s));
    else ED_K(dots_ptr(U.data() + nk + 1, 1, y, D, g + nk + 1, w.part, s));
    ED_K(set_scalar(g + nk, make_double2(beta_prev / (w.c[j - 1] * w.c[j]), 0.0), s));
    if (nk > 0) ED_K(dots_ptr(U.data(), nk, y, D, g, w.part, s));
    ED_K(axpy_norm_ptr(U.data(), n, g, sc.data(), y, D, nr, w.part, s));
    std::vector<double2> hs(1 + n);
    ED_TRY(fetch_scalars(w.scal, 1 + n, hs.data(), s));
    const double cj = w.c[j];
    *alpha = cj * cj * hs[1 + nk + 1].x;
    const double nrm2v = hs[kNrm].x;
    if (!std::isfinite(nrm2v) || !std::isfinite(*alpha))
        return fail(ED_ERR_NUMERIC, "non-finite value in the Lanczos recurrence");
    const double ny = std::sqrt(std::max(nrm2v, 0.0));
    *beta = cj * ny;
    *breakdown = (*beta <= 1e-14 * std::max(std::max(std::fabs(*alpha), beta_prev), 1e-300)) || *beta == 0.0;
    w.u[j + 1] = y;
    w.c[j + 1] = *breakdown ? 0.0 : 1.0 / ny;
    if (!*breakdown && (ny > 1e100 || ny < 1e-100)) {
        ED_K(scale(y, y, make_double2(1.0 / ny, 0.0), D, s));
        w.c[j + 1] = 1.0;
    }
    return ED_OK;
}

// Re-orthogonalise basis vector jn against the vectors listed in sel (one classical Gram-Schmidt
// pass: its components there are small, at most the trigger level of the orthogonality estimates).
// Returns the projections <v_i|v_jn before> in proj (real parts, in sel order) and the new |u_jn|.
ed_status reorth_selected(const Workspace& w, int jn, const std::vector<int>& sel, std::vector<double>* proj,
                          double* ny_new, hipStream_t s) {
    const int n = int(sel.size());
    if (n + 1 > kScalars) return fail(ED_ERR_UNSUPPORTED, "too many vectors to re-orthogonalise against");
    std::vector<const double2*> U(n);
    std::vector<double> sc(n);
    for (int k = 0; k < n; ++k) {
        U[k] = w.u[sel[k]];
        sc[k] = w.c[sel[k]] * w.c[sel[k]];
    }
    double2* y = w.u[jn];
    double2* nr = w.scal + kNrm;
    double2* g = w.scal + 1;
    ED_K(dots_ptr(U.data(), n, y, w.D, g, w.part, s));
    ED_K(axpy_norm_ptr(U.data(), n, g, sc.data(), y, w.D, nr, w.part, s));
    std::vector<double2> hs(1 + n);
    ED_TRY(fetch_scalars(w.scal, 1 + n, hs.data(), s));
    proj->resize(n);
    for (int k = 0; k < n; ++k) (*proj)[k] = w.c[sel[k]] * w.c[jn] * hs[1 + k].x;
    *ny_new = std::sqrt(std::max(hs[kNrm].x, 0.0));
    return ED_OK;
}

ed_status combine_basis(const Workspace& w, int m, const double2* xi, double2* out, hipStream_t s) {
    if (m > kMaxComb && out == w.u[0]) return fail(ED_ERR_UNSUPPORTED, "in-place combination of more than 64 vectors");
    std::vector<double2> c(m);
    for (int i = 0; i < m; ++i) c[i] = make_double2(xi[i].x * w.c[i], xi[i].y * w.c[i]);
    ED_K(combination_ptr(const_cast<const double2* const*>(w.u.data()), m, c.data(), out, w.D, s));
    return ED_OK;
}

}  // namespace ed

using namespace ed;

// ============================================================================ Lanczos ground
extern "C" ed_status ed_lanczos_workspace(const ed_model* model, const ed_lanczos_params* p, size_t* bytes) {
    if (!model || !p || !bytes) return fail(ED_ERR_ARG, "null argument");
    if (p->max_basis < 2 || p->max_basis > 512) return fail(ED_ERR_ARG, "max_basis must be in [2, 512]");
    const int keep = p->n_keep > 0 ? p->n_keep : std::min(10, p->max_basis / 2);
    if (keep >= p->max_basis) return fail(ED_ERR_ARG, "n_keep must be < max_basis");
    const int64_t D = int64_t(1) << model->L;
    *bytes = core_scratch_bytes() + ((size_t(p->max_basis + 1 + keep) * size_t(D) * sizeof(double2) + 255) & ~size_t(255));
    return ED_OK;
}

extern "C" ed_status ed_lanczos_ground(const ed_model* model, const ed_c64* v0, const ed_lanczos_params* p,
                                       double* E0, ed_c64* psi0, ed_lanczos_info* info, void* ws,
                                       size_t ws_bytes, void* stream) {
    if (!model || !v0 || !p || !E0 || !psi0) return fail(ED_ERR_ARG, "null argument");
    if (p->max_iter < 1) return fail(ED_ERR_ARG, "max_iter must be >= 1");
    if (!(p->tol > 0.0)) return fail(ED_ERR_ARG, "tol must be > 0");
    if (model->lv_L > 0) return fail(ED_ERR_UNSUPPORTED, "Lanczos needs a Hermitian model, not a Liouvillian");
    if (p->reorth != ED_REORTH_FULL && p->reorth != ED_REORTH_PARTIAL)
        return fail(ED_ERR_ARG, "reorth must be ED_REORTH_FULL or ED_REORTH_PARTIAL");
    size_t need = 0;
    ED_TRY(ed_lanczos_workspace(model, p, &need));
    const int mb = p->max_basis;
    const int keep = p->n_keep > 0 ? p->n_keep : std::min(10, mb / 2);
    const int64_t D = int64_t(1) << model->L;
    Workspace w;
    ED_TRY(carve(ws, ws_bytes, D, mb + 1 + keep, &w));
    if (ws_bytes < need) return fail(ED_ERR_WORKSPACE, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);

    // Ritz vector psi0 = V s of the first m basis vectors, renormalised, and the explicit residual
    auto finish = [&](int m, double theta, const std::vector<double>& svec, int iters, int restarts, int extra,
                      bool converged, bool device, ed_status result) -> ed_status {
        std::vector<double2> c(m);
        for (int r = 0; r < m; ++r) c[r] = make_double2(svec[r], 0.0);
        double2* out = reinterpret_cast<double2*>(psi0);
        ED_TRY(combine_basis(w, m, c.data(), out, s));
        double2* nr = w.scal + kNrm;
        ED_K(norm2(out, D, nr, w.part, s));
        ED_K(normalize(out, out, nr, D, s));
        // explicit residual |H psi0 - theta psi0|
        double2* r = w.V;  // basis no longer needed
        ED_TRY(launch_apply_H(model, out, r, s));
        ED_K(axpby(out, r, make_double2(-theta, 0.0), make_double2(1.0, 0.0), D, s));
        ED_K(norm2(r, D, nr, w.part, s));
        double2 hv[1];
        ED_TRY(fetch_scalars(w.scal, 1, hv, s));
        *E0 = theta;
        if (info) {
            info->iters = iters;
            info->restarts = restarts;
            info->residual = std::sqrt(std::max(hv[kNrm].x, 0.0));
            info->converged = converged ? 1 : 0;
            info->extra_reorth = extra;
            info->device_resident = device ? 1 : 0;
        }
        return result;
    };

    double nrm0 = 0.0;
    // Full reorthogonalisation on a basis that never restarts, for a short chain: the whole
    // recurrence on the device in one launch
    if (p->reorth == ED_REORTH_FULL && mb >= p->max_iter + 1 && lanczos_device_fits(model, p->max_iter)) {
        ED_TRY(start_vector(w, reinterpret_cast<const double2*>(v0), &nrm0, s, false));
        int m = 0, prods = 0;
        bool conv = false;
        std::vector<double> al, be;
        const ed_status ds = lanczos_device(model, w, p->max_iter, p->tol, &m, &prods, &conv, &al, &be, s);
        if (ds == ED_ERR_UNSUPPORTED) goto host_path;  // not co-resident now: the host-driven recurrence
        if (ds != ED_OK) return ds;
        std::vector<double> svec(m, 0.0);
        double theta = 0.0;
        tridiag_lowest(m, al.data(), be.data(), &theta, svec.data());
        w.u.resize(m);
        w.c.resize(m);
        for (int i = 0; i < m; ++i) {
            w.u[i] = w.slot(i);
            w.c[i] = 1.0;
        }
        const ed_status res =
            conv ? ED_OK : fail(ED_ERR_NOCONV, "Lanczos did not reach the tolerance within max_iter products");
        return finish(m, theta, svec, prods, 0, 0, conv, true, res);
    }
host_path:
    ED_TRY(start_vector(w, reinterpret_cast<const double2*>(v0), &nrm0, s, true));

    std::vector<double> T(size_t(mb + 1) * (mb + 1), 0.0);
    auto Tij = [&](int i, int j) -> double& { return T[size_t(i) * (mb + 1) + j]; };
    // partial reorthogonalisation: W(i, l) estimates <v_i|v_l> (Simon's recurrence, here on the
    // whole projected matrix, so that it also holds across the arrow of a thick restart)
    const bool partial = p->reorth == ED_REORTH_PARTIAL;
    std::vector<double> Wv(partial ? size_t(mb + 2) * (mb + 2) : 0, 0.0);
    auto Wij = [&](int i, int l) -> double& { return Wv[size_t(i) * (mb + 2) + l]; };
    if (partial) Wij(0, 0) = 1.0;
    double anorm = 0.0;
    bool reorth_pending = false;
    std::vector<int> sel;
    std::vector<double> proj, restart_coef;
    std::vector<cplx> h(mb + 1);
    int j = 0, iters = 0, restarts = 0, k_locked = 0, extra = 0;
    bool converged = false;
    double theta = 0.0;
    std::vector<double> svec;
    int m = 0;
    ed_status result = ED_OK;
    auto step_fail = [&](ed_status st) {
        return fail(st, std::string(ed_last_error()) + " (Lanczos product " + std::to_string(iters + 1) + ", restarts " +
                            std::to_string(restarts) + ", basis index " + std::to_string(j) + ")");
    };
    while (true) {
        double beta = 0.0;
        bool brk = false;
        // Full steps: every step with reorth = FULL; with PARTIAL only the first step of a cycle (its
        // projections on the kept Ritz vectors are the arrow of the restarted matrix).
        const bool full = !partial || j == 0 || j == k_locked;
        if (full) {
            // past the first step of a cycle the recurrence is three-term: the first Gram-Schmidt
            // pass needs only v_{j-1}, v_j (the second one takes the whole basis); at the first step
            // after a restart the first pass's projections on the kept vectors are the arrow
            const int first_lo = (j >= 1 && j > k_locked) ? j - 1 : -1;
            const double beta_prev = first_lo >= 0 ? Tij(j, j - 1) : -1.0;
            std::vector<double> arrow;
            if (restarts > 0 && j == k_locked) {
                arrow.resize(j);
                for (int i = 0; i < j; ++i) arrow[i] = Tij(i, j);
            }
            const ed_status st = krylov_step(model, w, j, 0, 2, 1e-14, h.data(), &beta, &brk, s, first_lo, beta_prev,
                                             arrow.empty() ? nullptr : arrow.data());
            if (st != ED_OK) return step_fail(st);
            for (int i = 0; i <= j; ++i) {
                Tij(i, j) = h[i].real();
                Tij(j, i) = h[i].real();
            }
            if (partial) {
                for (int i = 0; i <= j; ++i) Wij(j + 1, i) = Wij(i, j + 1) = kOrthEps;
            }
        } else {
            double alpha = 0.0;
            const double beta_prev = Tij(j, j - 1);
            const ed_status st = lanczos_local_step(model, w, j, k_locked, beta_prev, &alpha, &beta, &brk, s);
            if (st != ED_OK) return step_fail(st);
            Tij(j, j) = alpha;
            if (!brk) {
                // estimates for the new vector j+1: beta_j W(j+1, i) = sum_l T(l, i) W(l, j) - sum_l T(l, j) W(i, l)
                // + a rounding term, for the vectors it was not explicitly projected on
                anorm = std::max(anorm, std::fabs(alpha) + beta + beta_prev);
                const double noise = kOrthEps * anorm / beta;
                double wmax = 0.0;
                for (int i = k_locked; i + 1 < j; ++i) {
                    double t1 = 0.0, t2 = 0.0;
                    for (int l = 0; l <= j; ++l) {
                        t1 += Tij(l, i) * Wij(l, j);
                        t2 += Tij(l, j) * Wij(i, l);
                    }
                    double wn = (t1 - t2) / beta;
                    wn += std::copysign(noise, wn);
                    Wij(j + 1, i) = Wij(i, j + 1) = wn;
                    wmax = std::max(wmax, std::fabs(wn));
                }
                for (int i = 0; i < k_locked; ++i) Wij(j + 1, i) = Wij(i, j + 1) = kOrthEps;
                Wij(j + 1, j) = Wij(j, j + 1) = Wij(j + 1, j - 1) = Wij(j - 1, j + 1) = kOrthEps;
                if (reorth_pending || wmax > kOrthTrigger) {
                    // the vector and its successor are re-orthogonalised against the vectors whose
                    // estimate exceeds kOrthSelect (both, since the recurrence carries the component
                    // of v_j into v_{j+2})
                    sel.clear();
                    for (int i = k_locked; i + 1 < j; ++i)
                        if (std::fabs(Wij(j + 1, i)) > kOrthSelect) sel.push_back(i);
                    if (!sel.empty()) {
                        double ny = 0.0;
                        const ed_status st2 = reorth_selected(w, j + 1, sel, &proj, &ny, s);
                        if (st2 != ED_OK) return step_fail(st2);
                        for (size_t k = 0; k < sel.size(); ++k) {
                            Tij(sel[k], j) += beta * proj[k];
                            Tij(j, sel[k]) = Tij(sel[k], j);
                            Wij(j + 1, sel[k]) = Wij(sel[k], j + 1) = kOrthEps;
                        }
                        beta = w.c[j] * ny;
                        w.c[j + 1] = 1.0 / ny;
                        ++extra;
                    }
                    reorth_pending = !reorth_pending;
                }
            }
            Tij(j - 1, j) = beta_prev;
        }
        if (partial) Wij(j + 1, j + 1) = 1.0;
        ++iters;
        m = j + 1;
        // lowest Ritz pair of the m x m projected matrix
        svec.assign(m, 0.0);
        if (restarts == 0) {
            std::vector<double> a(m), b(std::max(m - 1, 1));
            for (int i = 0; i < m; ++i) a[i] = Tij(i, i);
            for (int i = 0; i + 1 < m; ++i) b[i] = Tij(i + 1, i);
            tridiag_lowest(m, a.data(), b.data(), &theta, svec.data());
        } else {
            std::vector<double> A(size_t(m) * m), wv(m), Z(size_t(m) * m);
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < m; ++c) A[size_t(r) * m + c] = Tij(r, c);
            sym_eig_jacobi(m, A.data(), wv.data(), Z.data());
            theta = wv[0];
            for (int r = 0; r < m; ++r) svec[r] = Z[size_t(r) * m];
        }
        const double res = beta * std::fabs(svec[m - 1]);
        if (brk || res <= p->tol) {
            converged = true;
            break;
        }
        if (iters >= p->max_iter) {
            result = fail(ED_ERR_NOCONV, "Lanczos did not reach the tolerance within max_iter products");
            break;
        }
        Tij(j + 1, j) = beta;
        Tij(j, j + 1) = beta;
        if (m == mb) {
            // thick restart: keep the `keep` lowest Ritz vectors plus the residual direction V_m
            std::vector<double> A(size_t(m) * m), wv(m), Z(size_t(m) * m);
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < m; ++c) A[size_t(r) * m + c] = Tij(r, c);
            sym_eig_jacobi(m, A.data(), wv.data(), Z.data());
            const double cm = w.c[m];
            if (m + 1 <= kMultiIn && keep + 1 <= kMultiOut) {
                // one sweep over the basis writes the Ritz vectors y_i = sum_r Z(r, i) v_r and the
                // normalised residual direction into slots 0..keep, in place
                restart_coef.assign(size_t(m + 1) * (keep + 1), 0.0);
                for (int r = 0; r < m; ++r)
                    for (int i = 0; i < keep; ++i) restart_coef[size_t(r) * (keep + 1) + i] = Z[size_t(r) * m + i] * w.c[r];
                restart_coef[size_t(m) * (keep + 1) + keep] = cm;
                double* cdev = reinterpret_cast<double*>(w.part);
                ED_HIP_TRY(hipMemcpyAsync(cdev, restart_coef.data(), restart_coef.size() * sizeof(double),
                                          hipMemcpyHostToDevice, s));
                std::vector<double2*> outs(keep + 1);
                for (int i = 0; i <= keep; ++i) outs[i] = w.slot(i);
                ED_K(combination_multi(const_cast<const double2* const*>(w.u.data()), m + 1, cdev, outs.data(), keep + 1,
                                       D, s));
                // the coefficient upload must be complete before restart_coef is touched again
                ED_HIP_TRY(hipStreamSynchronize(s));
            } else {
                double2* tmp = w.V + int64_t(mb + 1) * D;
                for (int i = 0; i < keep; ++i) {
                    std::vector<double2> c(m);
                    for (int r = 0; r < m; ++r) c[r] = make_double2(Z[size_t(r) * m + i], 0.0);
                    ED_TRY(combine_basis(w, m, c.data(), tmp + int64_t(i) * D, s));
                }
                ED_HIP_TRY(hipMemcpyAsync(w.V, tmp, size_t(keep) * D * sizeof(double2), hipMemcpyDeviceToDevice, s));
                // the residual direction v_m = c_m u_m is stored normalised in slot `keep`
                ED_K(scale(w.u[m], w.slot(keep), make_double2(cm, 0.0), D, s));
            }
            for (int i = 0; i <= keep; ++i) {
                w.u[i] = w.slot(i);
                w.c[i] = 1.0;
            }
            std::fill(T.begin(), T.end(), 0.0);
            for (int i = 0; i < keep; ++i) {
                Tij(i, i) = wv[i];
                Tij(i, keep) = beta * Z[size_t(m - 1) * m + i];
                Tij(keep, i) = Tij(i, keep);
            }
            if (partial) {
                std::fill(Wv.begin(), Wv.end(), 0.0);
                for (int i = 0; i <= keep; ++i)
                    for (int l = 0; l <= keep; ++l) Wij(i, l) = i == l ? 1.0 : kOrthEps;
                reorth_pending = false;
            }
            j = keep;
            k_locked = keep;
            ++restarts;
            continue;
        }
        ++j;
    }
    return finish(m, theta, svec, iters, restarts, extra, converged, false, result);
}

// ============================================================================ Krylov evolve
extern "C" ed_status ed_krylov_workspace(const ed_model* model, const ed_krylov_params* p, size_t* bytes) {
    if (!model || !p || !bytes) return fail(ED_ERR_ARG, "null argument");
    if (p->m_max < 1 || p->m_max > kMaxProj - 1) return fail(ED_ERR_ARG, "m_max must be in [1, 64]");
    const int64_t D = int64_t(1) << model->L;
    *bytes = core_scratch_bytes() + ((size_t(p->m_max + 1) * size_t(D) * sizeof(double2) + 255) & ~size_t(255));
    return ED_OK;
}

namespace ed {

// Observables of psi: sz (site order) normalised, and |psi|. sz may be null.
ed_status measure_state(const double2* psi, int L, const Workspace& w, double* sz, double* nrm, hipStream_t s) {
    double2* res = w.scal + kObs;
    ED_K(sz_all(psi, L, res, w.part, s));
    double2 hv[32];
    ED_TRY(fetch_scalars(res, L + 1, hv, s));
    const double n2 = hv[0].x;
    if (nrm) *nrm = std::sqrt(std::max(n2, 0.0));
    if (sz)
        for (int k = 1; k <= L; ++k) sz[k - 1] = hv[1 + (L - k)].x / n2;
    return ED_OK;
}

// tr(rho) and tr(sigma^z_k rho)/tr(rho) of a superket of an Ls-site system
ed_status measure_superket(const double2* rho, int Ls, const Workspace& w, double* sz, double* tr, hipStream_t s) {
    double2* res = w.scal + kObs;
    ED_TRY(superket_diag(rho, Ls, res, s));
    double2 hv[32];
    ED_TRY(fetch_scalars(res, Ls + 1, hv, s));
    if (tr) *tr = hv[0].x;
    if (sz)
        for (int k = 1; k <= Ls; ++k) sz[k - 1] = hv[k].x / hv[0].x;
    return ED_OK;
}

// One Krylov time step of psi in place: returns the dimension used, the error estimate and
// alpha_0 = <v_0|H v_0> (the energy of the incoming state).
ed_status krylov_time_step(const ed_model* m, const Workspace& w, double2* psi, double dt,
                           const ed_krylov_params* p, int* m_used, double* err_out, double* e_in,
                           double* nrm_in, hipStream_t s) {
    const int mmax = p->m_max;
    double nrm0 = 0.0;
    ED_TRY(start_vector(w, psi, &nrm0, s, true));
    std::vector<cplx> T(size_t(mmax + 1) * (mmax + 1), 0.0);
    auto Tij = [&](int i, int j) -> cplx& { return T[size_t(i) * (mmax + 1) + j]; };
    std::vector<cplx> h(mmax + 1), u(mmax + 1);
    const bool herm = p->hermitian != 0;
    const int passes = (p->reorth || !herm) ? 2 : 1;
    int mm = 0;
    double err = 0.0;
    for (int j = 0; j < mmax; ++j) {
        const bool three_term = herm && !p->reorth;
        const int lo = three_term ? std::max(j - 1, 0) : 0;
        double beta = 0.0;
        bool brk = false;
        // the first step has no previous norm: 0 marks the recurrence as three-term
        const double beta_prev = three_term ? (j >= 1 ? Tij(j, j - 1).real() : 0.0) : -1.0;
        ED_TRY(krylov_step(m, w, j, lo, passes, 1e-14, h.data(), &beta, &brk, s, -1, beta_prev));
        if (herm) {
            Tij(j, j) = h[j - lo].real();
        } else {
            for (int i = 0; i <= j; ++i) Tij(i, j) = h[i];
        }
        mm = j + 1;
        // u = exp(-i dt T_m) e_1
        if (herm) {
            std::vector<xreal> d(mm), e(mm), Z(size_t(mm) * mm, 0.0L);
            for (int i = 0; i < mm; ++i) {
                d[i] = Tij(i, i).real();
                e[i] = (i + 1 < mm) ? Tij(i + 1, i).real() : 0.0;
                Z[size_t(i) * mm + i] = 1.0L;
            }
            if (!tridiag_ql_ext(mm, d.data(), e.data(), Z.data()))
                return fail(ED_ERR_NUMERIC, "tridiagonal eigensolver did not converge");
            expm_col_sym_ext(mm, d.data(), Z.data(), dt, u.data());
        } else {
            std::vector<cplx> A(size_t(mm) * mm), E(size_t(mm) * mm);
            for (int r = 0; r < mm; ++r)
                for (int c = 0; c < mm; ++c) A[size_t(r) * mm + c] = cplx(0.0, -dt) * Tij(r, c);
            expm_complex(mm, A.data(), E.data());
            for (int r = 0; r < mm; ++r) u[r] = E[size_t(r) * mm];
        }
        err = nrm0 * beta * std::abs(u[mm - 1]);
        if (j == 0 && e_in) *e_in = Tij(0, 0).real();
        bool stop;
        if (p->fixed_m > 0) stop = brk || mm >= std::min(p->fixed_m, mmax);
        else stop = brk || err <= p->tol || mm >= mmax;
        if (brk) err = 0.0;
        if (stop) break;
        Tij(j + 1, j) = beta;
        if (herm) Tij(j, j + 1) = beta;
    }
    std::vector<double2> c(mm);
    for (int i = 0; i < mm; ++i) c[i] = make_double2(nrm0 * u[i].real(), nrm0 * u[i].imag());
    ED_TRY(combine_basis(w, mm, c.data(), psi, s));
    *m_used = mm;
    *err_out = err;
    if (nrm_in) *nrm_in = nrm0;
    return ED_OK;
}

// <psi|H|psi>/<psi|psi> using V_0, V_1 of the workspace as scratch
ed_status energy_of(const ed_model* m, const Workspace& w, const double2* psi, double* e, hipStream_t s) {
    double nrm0 = 0.0;
    ED_TRY(start_vector(w, psi, &nrm0, s));
    double2* Hv = w.V + w.D;
    ED_TRY(launch_apply_H(m, w.V, Hv, s));
    ED_K(dots(w.V, w.D, 1, Hv, w.D, w.scal + 1, w.part, s));
    double2 hv[2];
    ED_TRY(fetch_scalars(w.scal, 2, hv, s));
    *e = hv[1].x;
    return ED_OK;
}

}  // namespace ed

extern "C" ed_status ed_krylov_evolve(const ed_model* model, ed_c64* psi, double dt, int n_steps,
                                      const ed_krylov_params* p, const ed_observe* obs, ed_krylov_info* info,
                                      void* ws, size_t ws_bytes, void* stream) {
    if (!model || !psi || !p) return fail(ED_ERR_ARG, "null argument");
    if (n_steps < 0) return fail(ED_ERR_ARG, "n_steps must be >= 0");
    if (!std::isfinite(dt)) return fail(ED_ERR_ARG, "dt must be finite");
    if (!(p->tol > 0.0) && p->fixed_m <= 0) return fail(ED_ERR_ARG, "tol must be > 0");
    if (!p->hermitian && !p->reorth) return fail(ED_ERR_ARG, "Arnoldi (hermitian = 0) needs reorth = 1");
    const int lvL = model->lv_L;
    if (lvL > 0 && p->hermitian) return fail(ED_ERR_ARG, "a Liouvillian model needs hermitian = 0 (Arnoldi)");
    if (lvL > 0 && obs && obs->energy) return fail(ED_ERR_UNSUPPORTED, "no energy observable for a Liouvillian model");
    size_t need = 0;
    ED_TRY(ed_krylov_workspace(model, p, &need));
    if (ws_bytes < need) return fail(ED_ERR_WORKSPACE, "workspace too small");
    const int L = model->L;
    const int64_t D = int64_t(1) << L;
    Workspace w;
    ED_TRY(carve(ws, ws_bytes, D, p->m_max + 1, &w));
    int skipped = 0;
    w.cgs_skipped = &skipped;
    ObsStage stage;
    obs = stage.begin(obs, n_steps, lvL > 0 ? lvL : L);
    hipStream_t s = static_cast<hipStream_t>(stream);
    double2* v = reinterpret_cast<double2*>(psi);
    int total_m = 0, max_m = 0;
    double max_err = 0.0;
    const bool want_e = obs && obs->energy;
    auto record = [&](int step) -> ed_status {
        if (!obs || (!obs->sz && !obs->norm)) return ED_OK;
        if (lvL > 0) {  // observables of rho: tr(sigma^z_k rho)/tr(rho) and tr(rho)
            double tr = 0.0;
            ED_TRY(measure_superket(v, lvL, w, obs->sz ? obs->sz + size_t(step) * lvL : nullptr, &tr, s));
            if (obs->norm) obs->norm[step] = tr;
            return ED_OK;
        }
        double nrm = 0.0;
        ED_TRY(measure_state(v, L, w, obs->sz ? obs->sz + size_t(step) * L : nullptr, &nrm, s));
        if (obs->norm) obs->norm[step] = nrm;
        return ED_OK;
    };
    ED_TRY(record(0));
    for (int st = 0; st < n_steps; ++st) {
        int mu = 0;
        double err = 0.0, e_in = 0.0, n_in = 0.0;
        ED_TRY(krylov_time_step(model, w, v, dt, p, &mu, &err, &e_in, &n_in, s));
        if (want_e) obs->energy[st] = e_in;
        total_m += mu;
        max_m = std::max(max_m, mu);
        max_err = std::max(max_err, err);
        ED_TRY(record(st + 1));
    }
    if (want_e) {
        double e = 0.0;
        ED_TRY(energy_of(model, w, v, &e, s));
        obs->energy[n_steps] = e;
    }
    ED_HIP_TRY(hipStreamSynchronize(s));
    ED_TRY(stage.finish(s));
    if (info) {
        info->steps = n_steps;
        info->total_m = total_m;
        info->max_m = max_m;
        info->max_err = max_err;
        info->reorth_skipped = skipped;
    }
    return ED_OK;
}

// ============================================================================ measurement
extern "C" ed_status ed_measure_workspace(int L, size_t* bytes) {
    if (!bytes || L < 1 || L > 30) return fail(ED_ERR_ARG, "bad argument");
    *bytes = core_scratch_bytes();
    return ED_OK;
}

extern "C" ed_status ed_liouville_measure(const ed_c64* rho, int L, double* sz, double* trace, void* ws,
                                          size_t ws_bytes, void* stream) {
    if (!rho || !sz || L < 1 || L > 15) return fail(ED_ERR_ARG, "bad argument (rho or sz null, L outside 1..15)");
    Workspace w;
    ED_TRY(carve(ws, ws_bytes, int64_t(1) << (2 * L), 0, &w));
    return measure_superket(reinterpret_cast<const double2*>(rho), L, w, sz, trace, static_cast<hipStream_t>(stream));
}

extern "C" ed_status ed_measure(const ed_c64* psi, int L, double* sz, double* norm, void* ws, size_t ws_bytes,
                                void* stream) {
    if (!psi || !sz || L < 1 || L > 30) return fail(ED_ERR_ARG, "bad argument");
    Workspace w;
    ED_TRY(carve(ws, ws_bytes, int64_t(1) << L, 0, &w));
    return measure_state(reinterpret_cast<const double2*>(psi), L, w, sz, norm, static_cast<hipStream_t>(stream));
}

// ============================================================================ measurement, no allocation
// ed_measure_noalloc runs the kernels of ed_measure on a file-scope device array instead of a
// caller workspace: the per-block partial sums of the one-pass reduction (at most kSzBlocks
// rows of kPartLd complex values) and the L + 1 reduced sums. Each device that the library runs
// on holds its own copy of the array until the process ends; host code uses the address that
// hipGetSymbolAddress returns for the current device, never the array's name.
namespace ed {
namespace {

constexpr size_t kNoAllocPartBytes = (size_t(kSzBlocks) * kPartLd * sizeof(double2) + 255) & ~size_t(255);
constexpr size_t kNoAllocResultBytes = 256 * sizeof(double2);  // >= (L + 1) entries for L <= 30
constexpr size_t kNoAllocScratchBytes = kNoAllocPartBytes + kNoAllocResultBytes;
constexpr int kNoAllocMaxL = 30;
constexpr int kNoAllocMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};

// Device address of `scratch` on the current device, resolved once per device.
ed_status noalloc_scratch(void** out) {
    int dev = -1;
    ED_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        return fail(ED_ERR_UNSUPPORTED, "device index " + std::to_string(dev) + " outside the no-allocation table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ED_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ED_OK;
}

}  // namespace
}  // namespace ed

extern "C" ed_status ed_measure_noalloc(const ed_c64* psi, int L, double* sz, double* norm, void* stream) {
    if (!psi || !sz) return fail(ED_ERR_ARG, "bad argument (psi or sz null)");
    if (L < 1 || L > kNoAllocMaxL)
        return fail(ED_ERR_ARG, "L = " + std::to_string(L) + " outside 1.." + std::to_string(kNoAllocMaxL) +
                                    " (the no-allocation scratch holds the reduction of at most 2^30 amplitudes)");
    static_assert(size_t(kSzBlocks) * kPartLd * sizeof(double2) <= kNoAllocPartBytes, "partial rows exceed scratch");
    static_assert(size_t(kNoAllocMaxL + 1) * sizeof(double2) <= kNoAllocResultBytes, "results exceed scratch");
    void* base = nullptr;
    ED_TRY(noalloc_scratch(&base));
    hipStream_t s = static_cast<hipStream_t>(stream);
    double2* part = static_cast<double2*>(base);
    double2* res = reinterpret_cast<double2*>(static_cast<char*>(base) + kNoAllocPartBytes);
    // Every partial row and every result that the reduction reads is written earlier on the same
    // stream by this call, so nothing has to be cleared first.
    ED_K(sz_all(reinterpret_cast<const double2*>(psi), L, res, part, s));
    double2 hv[kNoAllocMaxL + 1];
    ED_HIP_TRY(hipMemcpyAsync(hv, res, sizeof(double2) * (L + 1), hipMemcpyDeviceToHost, s));
    ED_HIP_TRY(hipStreamSynchronize(s));
    const double n2 = hv[0].x;
    if (norm) *norm = std::sqrt(std::max(n2, 0.0));
    for (int k = 1; k <= L; ++k) sz[k - 1] = hv[1 + (L - k)].x / n2;
    return ED_OK;
}

