// Shared Krylov recurrence (krylov.cpp) used by the ground-state, time-evolution, trajectory and
// adjoint drivers.
#pragma once
#include <vector>

#include "dense.h"
#include "ed_internal.h"

namespace ed {

constexpr int kMaxProj = 520;                  // max vectors one step projects against
constexpr int kNrm = 0;                        // scalar area: [norm^2, h1[n], h2[n] ... | obs]
constexpr int kObs = 1 + 2 * kMaxProj;
constexpr int kScalars = kObs + 64;
// Partial reorthogonalisation of the Lanczos ground state: a new vector whose estimated overlap with
// an earlier one exceeds kOrthTrigger is re-orthogonalised (with its successor) against the vectors
// whose estimate exceeds kOrthSelect; vectors projected explicitly start at kOrthEps (the unit
// roundoff). The trigger sits well below sqrt(eps): semi-orthogonality alone keeps the Ritz values
// exact but not the Ritz vector's residual at the 1e-10 level.
constexpr double kOrthEps = 1.1102230246251565e-16;
constexpr double kOrthTrigger = 1e-12;
constexpr double kOrthSelect = 1e-14;

// Caller workspace carved into: partial-reduction buffer, device scalars, nvec vectors of D.
// The Krylov basis lives there as (u_i, c_i) with v_i = c_i u_i: u_i is slot i of V except that
// u_0 may be the caller's state itself; c_i is a host scalar, so a new basis vector is never
// rescaled in memory.
struct Workspace {
    double2* part = nullptr;
    double2* scal = nullptr;
    double2* V = nullptr;
    int nvec = 0;
    int64_t D = 0;
    mutable std::vector<double2*> u;
    mutable std::vector<double> c;
    int* cgs_skipped = nullptr;  // when set, counts the second Gram-Schmidt passes skipped
    double2* slot(int i) const { return V + int64_t(i) * D; }
};

size_t core_scratch_bytes();
ed_status carve(void* ws, size_t ws_bytes, int64_t D, int nvec, Workspace* w);
ed_status fetch_scalars(const double2* dev, int n, double2* host, hipStream_t s);
// passes = 2 with both passes over lo..j (no first_lo, beta_prev or known): the second pass runs
// only when the first removed more than half of the squared norm of H v_j.
// first_lo > lo (with passes = 2): the first Gram-Schmidt pass takes only vectors first_lo..j (the
// ones a three-term recurrence couples), the second pass all of lo..j.
// beta_prev >= 0 (Hermitian H; passes = 1 with lo = j - 1 or j = lo = 0, or passes = 2 with
// first_lo = j - 1): the projection of H v_j on v_{j-1} (in the first pass) is taken as
// beta_prev, the previous step's norm (they are equal for a Hermitian H), and <v_j|H v_j> comes
// from the product's last pass where the plan allows, else from one dot sweep.
// known (host, passes = 2, lo = 0, first_lo < 0): the first pass's projections <v_i|H v_j> for
// i = 0..j-1 are known in advance (the first step after a thick restart: the restarted matrix's
// arrow), so that pass needs only <v_j|H v_j>, from the product.
ed_status krylov_step(const ed_model* m, const Workspace& w, int j, int lo, int passes, double tiny_rel,
                      cplx* h, double* beta, bool* breakdown, hipStream_t s, int first_lo = -1,
                      double beta_prev = -1.0, const double* known = nullptr);
// Device-resident Lanczos (lanczos_dev.hip): full reorthogonalisation with no restart, the whole
// recurrence in one cooperative launch. Fits chains of L <= kDevLanczosMaxL without long-range
// rules or far terms and max_iter <= 511 products (within the partial-sum area). On return the
// first m basis slots hold v_0..v_{m-1} (slot 0 must hold the unit start vector at entry),
// alpha/beta the m diagonal and off-diagonal entries of T, products the H psi count and converged
// whether beta_{m-1} |s_{m-1}| <= tol (tested every 8 products) or the space became invariant.
// Returns ED_ERR_UNSUPPORTED without touching the basis when the cooperative launch cannot have all
// its workgroups resident (the caller then runs the host-driven recurrence).
// Observables of an evolve call whose arrays may be device memory (obs->on_device): the call
// writes host arrays (begin returns the ed_observe to use) and finish copies them to the
// caller's arrays, synchronising the stream. For host arrays both are pass-throughs.
struct ObsStage {
    ed_observe host{};
    const ed_observe* user = nullptr;
    std::vector<double> sz, energy, norm;
    size_t nsz = 0, nt = 0;
    const ed_observe* begin(const ed_observe* obs, int n_steps, int per_step) {
        user = obs;
        if (!obs || !obs->on_device) return obs;
        nt = size_t(n_steps) + 1;
        nsz = nt * size_t(per_step);
        host = *obs;
        host.on_device = 0;
        if (obs->sz) {
            sz.assign(nsz, 0.0);
            host.sz = sz.data();
        }
        if (obs->energy) {
            energy.assign(nt, 0.0);
            host.energy = energy.data();
        }
        if (obs->norm) {
            norm.assign(nt, 0.0);
            host.norm = norm.data();
        }
        return &host;
    }
    ed_status finish(hipStream_t s) {
        if (!user || !user->on_device) return ED_OK;
        if (user->sz) ED_HIP_TRY(hipMemcpyAsync(user->sz, sz.data(), nsz * sizeof(double), hipMemcpyHostToDevice, s));
        if (user->energy)
            ED_HIP_TRY(hipMemcpyAsync(user->energy, energy.data(), nt * sizeof(double), hipMemcpyHostToDevice, s));
        if (user->norm)
            ED_HIP_TRY(hipMemcpyAsync(user->norm, norm.data(), nt * sizeof(double), hipMemcpyHostToDevice, s));
        ED_HIP_TRY(hipStreamSynchronize(s));
        return ED_OK;
    }
};

constexpr int kDevLanczosMaxL = 16;
bool lanczos_device_fits(const ed_model* m, int max_iter);
ed_status lanczos_device(const ed_model* m, const Workspace& w, int max_iter, double tol, int* m_out,
                         int* products, bool* converged, std::vector<double>* alpha, std::vector<double>* beta,
                         hipStream_t s);
// Basis vector 0 from psi: alias = true uses psi itself as u_0 (c_0 = 1/|psi|); otherwise psi/|psi|
// is written to slot 0 (c_0 = 1).
ed_status start_vector(const Workspace& w, const double2* psi, double* nrm, hipStream_t s, bool alias = false);
// out = sum_i xi_i v_i over the first m basis vectors (xi host); out may be u_0.
ed_status combine_basis(const Workspace& w, int m, const double2* xi, double2* out, hipStream_t s);
ed_status measure_state(const double2* psi, int L, const Workspace& w, double* sz, double* nrm, hipStream_t s);
ed_status krylov_time_step(const ed_model* m, const Workspace& w, double2* psi, double dt,
                           const ed_krylov_params* p, int* m_used, double* err_out, double* e_in,
                           double* nrm_in, hipStream_t s);
ed_status energy_of(const ed_model* m, const Workspace& w, const double2* psi, double* e, hipStream_t s);

}  // namespace ed
