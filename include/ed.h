/*
 * ed.h -- C ABI of the MI355X exact-diagonalisation hot path (libed.so).
 *
 * The library applies a local 1-D lattice Hamiltonian to a dense complex128 state without ever
 * storing H (the "rule set x psi" product of Sec. ed:sec:krylov, Eq. ed:eq:OKrylov), and builds on that
 * product: Lanczos ground states (Sec. ed:sec:statics, computed matrix-free), Krylov time steps
 * (Sec. ed:sec:krylov), quantum trajectories (Sec. ed:sec:QT), a bond-coupling adjoint gradient and the
 * half-chain bond entropy (Sec. ed:sec:meas).
 *
 * Conventions shared by every call
 *   - d = 2. The state index is x = sum_{k=1..L} i_k 2^(L-k): site 1 is the most significant
 *     digit (the row-major rank-L tensor view of Sec. ed:sec:meas). Local index 0 = up (sigma^z = +1).
 *     Site k therefore sits at bit p = L-k, and bond (k, k+1) occupies bits (L-k-1, L-k).
 *   - Amplitudes are ed_c64 (interleaved re, im; the layout of torch.complex128), D = 2^L.
 *   - "device" pointers are HIP device memory owned by the caller; the library never frees or
 *     reallocates them. Host pointers are plain CPU memory.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream). Calls that return host
 *     scalars synchronise that stream before returning; ed_apply_H is asynchronous.
 *   - Every call returns ed_status. On error the outputs are unspecified and ed_last_error()
 *     returns a message (thread-local). No C++ exception crosses this boundary.
 *   - Model handles are immutable after creation: concurrent calls that share a handle on
 *     different streams are safe. Calls that share a workspace must not overlap.
 */
#ifndef ED_H
#define ED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } ed_c64;

typedef enum {
    ED_OK = 0,
    ED_ERR_ARG = -1,          /* invalid argument (null pointer, size, range)          */
    ED_ERR_UNSUPPORTED = -2,  /* valid request outside what the library supports (d != 2, L > 30 ...) */
    ED_ERR_NODEVICE = -3,     /* no HIP device visible                                  */
    ED_ERR_NOMEM = -4,        /* a small internal device/host allocation failed         */
    ED_ERR_WORKSPACE = -5,    /* caller workspace smaller than the size query returned  */
    ED_ERR_HIP = -6,          /* a HIP runtime call failed                              */
    ED_ERR_NOCONV = -7,       /* iteration limit reached before the tolerance           */
    ED_ERR_NUMERIC = -8       /* non-finite value detected                               */
} ed_status;

/* Thread-local message describing the last error of this thread ("" if none). */
const char* ed_last_error(void);

/* Library version string. */
const char* ed_version(void);

/* ----------------------------------------------------------------------------------------
 * Model: a rule-set Hamiltonian (Eq. ed:eq:genericH; site and bond rules of App. A,
 * Eqs. ed:eq:appsiters and ed:eq:appbondrs), with the general coupling w and the
 * site-dependent c_k folded into one coefficient per term:
 *
 *   H = sum_{z<n_site} sum_{k=1..L} site_coef[z][k-1] * O^z_k
 *     + sum_{z<n_bond} sum_{k=1..L-1} bond_coef[z][k-1] * B^z_{k,k+1}
 *
 *   site_op  host, [n_site][2][2] row-major (<i|O|j> at [i][j])
 *   bond_op  host, [n_bond][4][4] row-major, index i_k*2 + i_{k+1} (site k is the left
 *            Kronecker factor)
 *   site_coef host, [n_site][L];  bond_coef host, [n_bond][L-1]   (real)
 *
 * InfiniteFunc rules (App. A, Eq. ed:eq:appinfrs) without phase operators (Q = identity):
 *
 *     + sum_{z<n_inf} sum_{1<=k<j<=L} inf_coef[z][k-1] * inf_f[z][j-k-1] * O^z_k O'^z_j
 *
 *   inf_op, inf_op2 host, [n_inf][2][2] (O and O'); both must be diagonal (the long-range zz
 *            couplings of the long-range Ising chain, densities, ...), else ED_ERR_UNSUPPORTED;
 *   inf_coef host, [n_inf][L] (c_k, real); inf_f host, [n_inf][L-1] (f(r) for r = 1..L-1, real).
 *   They enter only the diagonal of H; ed_apply_H and the Krylov calls support them, the
 *   trajectory, adjoint and Trotter calls (which take the model apart into sites and bonds)
 *   return ED_ERR_UNSUPPORTED for a model that has them.
 *
 * Operators may be non-Hermitian (the effective Hamiltonian of a trajectory); Hermiticity of a
 * Hamiltonian is the caller's responsibility, as in the paper's rule sets. All host arrays are
 * copied; the handle keeps small coefficient tables in device memory of the current device.
 * Requires 2 <= L <= 30 and d == 2 (else ED_ERR_UNSUPPORTED); n_site, n_bond, n_inf >= 0; a null
 * array is allowed only when its count is 0.
 * ---------------------------------------------------------------------------------------- */
typedef struct ed_model ed_model;

typedef struct {
    int L;
    int d;
    int n_site;
    const ed_c64* site_op;
    const double* site_coef;
    int n_bond;
    const ed_c64* bond_op;
    const double* bond_coef;
    int n_inf;
    const ed_c64* inf_op;
    const ed_c64* inf_op2;
    const double* inf_coef;
    const double* inf_f;
} ed_model_desc;

ed_status ed_model_create(const ed_model_desc* desc, ed_model** out);
ed_status ed_model_destroy(ed_model* model);
/* L and D = 2^L of a model. */
ed_status ed_model_dims(const ed_model* model, int* L, int64_t* D);
/* Number of streaming passes over the state one ed_apply_H makes (diagnostic). */
ed_status ed_model_passes(const ed_model* model, int* passes);

/* Autotuning of H psi. A model holds up to 96 candidate pass plans (which index bits each
 * streaming pass covers, how many bits above a tile are read from neighbouring tiles in L2, and
 * whether a pass runs one workgroup per CU, two tiles per workgroup, or one tile per 1024-thread
 * workgroup). All candidates compute the same H psi (up to the order of floating-point sums). Candidates have the fewest passes possible for L (plus the plan
 * without neighbour reads), ordered by an estimated cost; the first is selected at creation.
 * ed_model_tune times every candidate on the caller's device buffers psi, out (D amplitudes each,
 * `reps` products per candidate, HIP events on stream), selects the fastest and returns its
 * index and the per-candidate times (host, may be NULL; count from ed_model_plans). Selecting or
 * tuning a plan modifies the handle: it must not run concurrently with any other call that uses
 * the same model. ed_model_plan_describe writes a one-line description of candidate `index`
 * (NUL-terminated, truncated to buf_len bytes), e.g. "first+G5 | c3 h16 +G3", into buf. */
ed_status ed_model_plans(const ed_model* model, int* count, int* selected);
ed_status ed_model_select_plan(ed_model* model, int index);
ed_status ed_model_plan_describe(const ed_model* model, int index, char* buf, int buf_len);
ed_status ed_model_tune(ed_model* model, const ed_c64* psi, ed_c64* out, int reps, void* stream, int* best,
                        float* times_ms);

/* ----------------------------------------------------------------------------------------
 * Tuned-plan cache (host memory, process-wide). An entry maps a model's plan key to the
 * description of its fastest plan. The key names the GPU architecture, L, the operator class
 * (kernel variant), the Liouville and long-range flags and a hash of the model's whole candidate
 * list, so it applies only to models whose planner proposes the same candidates.
 *   ed_model_create / ed_liouville_create select the cached plan when the key has an entry whose
 *     plan is among the candidates (else the planner's first candidate, as without a cache);
 *   ed_model_tune stores its choice under the model's key;
 *   ed_plan_cache_load merges "<key> TAB <plan>" lines from a text file ('#' starts a comment)
 *     and returns the number of entries read; ed_plan_cache_save writes every entry (replacing the
 *     file through a temporary in the same directory);
 *   ed_plan_cache_get / _put / _clear read, set and empty entries (host only, no GPU needed);
 *   ed_model_plan_key writes the model's key (NUL-terminated; ED_ERR_ARG if buf_len is too small).
 * Keys and plans must not contain tabs or newlines. The cache is guarded by a mutex. */
ed_status ed_model_plan_key(const ed_model* model, char* buf, int buf_len);
ed_status ed_plan_cache_load(const char* path, int* entries);
ed_status ed_plan_cache_save(const char* path);
ed_status ed_plan_cache_get(const char* key, char* buf, int buf_len);
ed_status ed_plan_cache_put(const char* key, const char* plan);
ed_status ed_plan_cache_clear(void);

/* ----------------------------------------------------------------------------------------
 * ed_apply_H: out = H psi (Sec. ed:sec:krylov, the rule set applied to the state without building H,
 * Eq. ed:eq:OKrylov). psi and out are device arrays of D amplitudes that must not overlap.
 * Asynchronous on stream.
 * ---------------------------------------------------------------------------------------- */
ed_status ed_apply_H(const ed_model* model, const ed_c64* psi, ed_c64* out, void* stream);


/* ----------------------------------------------------------------------------------------
 * Workspace. Iterative calls take a caller-owned device workspace (ws, ws_bytes) whose size
 * comes from the matching *_workspace query; the library allocates nothing on these paths.
 * A workspace smaller than the query returns ED_ERR_WORKSPACE.
 * ---------------------------------------------------------------------------------------- */

/* ----------------------------------------------------------------------------------------
 * ed_lanczos_ground: lowest eigenpair of a Hermitian model, matrix-free. The paper obtains the
 * ground state from the full H with eigh/eigsh (Sec. ed:sec:statics); here the same Lanczos
 * recurrence that underlies the Krylov step (Sec. ed:sec:krylov) runs on H psi directly:
 *   v_1 = v0/|v0|; w = H v_j; beta_j = |w| after orthogonalisation; T = V^H H V is the projected
 *   matrix. reorth selects how w is orthogonalised:
 *   ED_REORTH_FULL: against every stored v_i by classical Gram-Schmidt applied twice (past the
 *     first step of a cycle the first pass takes only v_{j-1}, v_j, whose projections the
 *     three-term recurrence supplies, and the second pass the whole basis);
 *   ED_REORTH_PARTIAL: against v_{j-1}, v_j and, by one Gram-Schmidt pass, the kept Ritz vectors
 *     of the last restart; estimates of the overlaps with the other vectors follow Simon's
 *     recurrence (on the full projected matrix), and a vector whose estimate exceeds 1e-12 is
 *     re-orthogonalised, with its successor, against the vectors concerned. The first step of a
 *     cycle stays full (its projections on the kept vectors are the restarted matrix's arrow).
 *   When the basis reaches max_basis vectors it is restarted thick (Wu & Simon): the n_keep
 *   lowest Ritz vectors and the last residual vector are kept and the recurrence continues.
 *   Convergence: beta_j |s_j| <= tol for the lowest Ritz pair (theta, s) (the residual norm
 *   |H psi - theta psi| of the unit Ritz vector), or an invariant subspace (beta_j <= 1e-14 |theta|).
 *   With ED_REORTH_FULL, max_basis > max_iter (no restart possible), L <= 16, no long-range rules
 *   and max_iter <= 511, the recurrence runs device-resident: one cooperative launch performs
 *   every product and both Gram-Schmidt passes (grid barriers between the phases) and tests
 *   convergence on the device every 8 products, so it may take up to 7 products more than the
 *   per-product test; info->device_resident reports it.
 * v0      device, D amplitudes, any nonzero vector (not modified)
 * E0      host, lowest Ritz value; psi0 device, D amplitudes, unit norm (global phase arbitrary)
 * info    host (may be NULL): iterations (H psi products), restarts, explicit residual
 *         |H psi0 - E0 psi0| recomputed at the end, converged flag
 * Returns ED_ERR_NOCONV (with E0, psi0, info filled) if max_iter products were not enough.
 * Workspace: ed_lanczos_workspace = (max_basis + 1 + n_keep) D complex + scratch.
 * Limits: 2 <= max_basis <= 512, 0 <= n_keep < max_basis (0 means min(10, max_basis/2)).
 * ---------------------------------------------------------------------------------------- */
typedef enum { ED_REORTH_FULL = 0, ED_REORTH_PARTIAL = 1 } ed_reorth;

typedef struct {
    int max_iter;
    int max_basis;
    int n_keep;
    double tol;
    int reorth;  /* ed_reorth */
} ed_lanczos_params;

typedef struct {
    int iters;
    int restarts;
    double residual;
    int converged;
    int extra_reorth;  /* re-orthogonalisations triggered by the estimates (reorth = PARTIAL) */
    int device_resident; /* 1 if the recurrence ran in one device-resident launch (see above) */
} ed_lanczos_info;

ed_status ed_lanczos_workspace(const ed_model* model, const ed_lanczos_params* params, size_t* bytes);
ed_status ed_lanczos_ground(const ed_model* model, const ed_c64* v0, const ed_lanczos_params* params,
                            double* E0, ed_c64* psi0, ed_lanczos_info* info, void* ws, size_t ws_bytes,
                            void* stream);

/* ----------------------------------------------------------------------------------------
 * ed_krylov_evolve: n_steps Krylov time steps psi(t+dt) = |psi| V_m exp(-i dt T_m) e_1
 * (Sec. ed:sec:krylov): a new Krylov basis of the current state every step, xi_i = [exp(-i dt T_m)]_{i,1}.
 * hermitian = 1: Lanczos, T_m real symmetric tridiagonal (closed systems);
 * hermitian = 0: Arnoldi, T_m upper Hessenberg (non-Hermitian generators, Sec. ed:sec:Liouville).
 * Stopping (the paper names a tolerance and a maximal basis size): the a-posteriori estimate
 * |psi| beta_m |[exp(-i dt T_m)]_{m,1}| <= tol, an invariant subspace (beta_m <= 1e-14 |T_m|), or
 * m = m_max. fixed_m > 0 forces exactly min(fixed_m, m_max) vectors unless the space is invariant.
 * reorth = 1 orthogonalises every new vector against the whole basis by classical Gram-Schmidt,
 * with a second pass when the first removed more than half of the squared norm (the DGKS test
 * with eta = 1/sqrt(2); info->reorth_skipped counts the second passes found unnecessary);
 * reorth = 0 against the previous two (the three-term recurrence with local re-projection;
 * Hermitian only). Arnoldi (hermitian = 0) needs reorth = 1.
 * psi     device, D amplitudes, in place: psi(0) on entry, psi(n_steps dt) on exit; no
 *         renormalisation (the norm drift is measured).
 * obs     arrays, each may be NULL: sz[(n_steps+1) * L] = <sigma^z_k>/<psi|psi> for sites
 *         k = 1..L at t = 0, dt, ..., energy[n_steps+1] = <psi|H|psi>/<psi|psi>,
 *         norm[n_steps+1] = |psi|. Host arrays when obs->on_device = 0; device arrays when it
 *         is 1 (the values are staged on the host during the call and copied to the device
 *         arrays before it returns).
 * info    host (may be NULL).
 * Workspace: ed_krylov_workspace = (m_max + 1) D complex + scratch. Limits: 1 <= m_max <= 64.
 * ---------------------------------------------------------------------------------------- */
typedef struct {
    int m_max;
    double tol;
    int fixed_m;
    int reorth;
    int hermitian;
} ed_krylov_params;

typedef struct {
    double* sz;
    double* energy;
    double* norm;
    int on_device; /* 0: the arrays are host memory; 1: device memory */
} ed_observe;

typedef struct {
    int steps;
    int total_m;
    int max_m;
    double max_err;
    int reorth_skipped;  /* second Gram-Schmidt passes skipped by the DGKS test (reorth = 1) */
} ed_krylov_info;

ed_status ed_krylov_workspace(const ed_model* model, const ed_krylov_params* params, size_t* bytes);
ed_status ed_krylov_evolve(const ed_model* model, ed_c64* psi, double dt, int n_steps,
                           const ed_krylov_params* params, const ed_observe* obs, ed_krylov_info* info,
                           void* ws, size_t ws_bytes, void* stream);

/* ----------------------------------------------------------------------------------------
 * ed_trotter_evolve: n_steps Suzuki-Trotter time steps (Sec. ed:sec:trotter). H = H_o + H_e,
 * H_o = the bond terms (k, k+1) with k odd (1-based sites), H_e = those with k even; the site
 * terms of each site are shared by the bonds that contain it, weight 1/2 each, or 1 for a site
 * in a single bond (sites 1 and L of the open chain).
 *   order 2: exp(-i dt/2 H_e) exp(-i dt H_o) exp(-i dt/2 H_e)              (Eq. ed:eq:trotter2)
 *   order 4: the eleven layers of Eq. ed:eq:trotter4, constants of Eq. ed:eq:trotter4c.
 * A layer is the product of the commuting two-site propagators exp(-i t h_k) (formed on the host
 * from the model's folded operators, which need not be Hermitian), applied in place.
 * psi     device, D amplitudes, in place: psi(0) on entry, psi(n_steps dt) on exit.
 * obs     as for ed_krylov_evolve (host arrays of n_steps + 1 entries, each may be NULL);
 *         energy = <psi|H|psi>/<psi|psi> costs one H psi per record and needs the workspace of
 *         ed_trotter_workspace(model, with_energy = 1, ...).
 * Workspace: ed_trotter_workspace bytes (scratch, two state vectors when with_energy = 1, and a
 *         50 KiB table of the gate matrices and their tile bits, copied in at the start of the
 *         call, which synchronises the stream once before the first pass).
 * Errors: ED_ERR_ARG (null model/psi/ws, order not 2 or 4, n_steps < 0, dt not finite),
 * ED_ERR_WORKSPACE. Synchronises stream.
 * ---------------------------------------------------------------------------------------- */
ed_status ed_trotter_workspace(const ed_model* model, int with_energy, size_t* bytes);
ed_status ed_trotter_evolve(const ed_model* model, ed_c64* psi, double dt, int n_steps, int order,
                            const ed_observe* obs, void* ws, size_t ws_bytes, void* stream);

/* ----------------------------------------------------------------------------------------
 * ed_trotter_passes: the number of in-place passes over the state that one ed_trotter_evolve
 * step of the given order makes (Sec. ed:sec:trotter), each reading and writing the state once.
 * The step's layers are applied in runs of four consecutive layers; a run streams the state
 * through LDS tiles (the 12 low bits, then windows of 8 bits above 4 contiguous low bits) and a
 * pass applies, layer by layer, every gate its tile holds whose earlier-layer neighbours are
 * already applied. passes host. No device work.
 * Errors: ED_ERR_ARG (null model/passes, order not 2 or 4), ED_ERR_UNSUPPORTED (long-range or
 * Liouville models).
 * ---------------------------------------------------------------------------------------- */
ed_status ed_trotter_passes(const ed_model* model, int order, int* passes);

/* ----------------------------------------------------------------------------------------
 * ed_measure: norm and all-site <sigma^z> of a state in one read pass (Sec. ed:sec:meas: the diagonal of
 * every single-site reduced density matrix). psi device; sz host [L] (site order k = 1..L,
 * normalised by <psi|psi>), norm host (may be NULL). Synchronises stream.
 * Workspace: ed_measure_workspace bytes.
 * ---------------------------------------------------------------------------------------- */
ed_status ed_measure_workspace(int L, size_t* bytes);
ed_status ed_measure(const ed_c64* psi, int L, double* sz, double* norm, void* ws, size_t ws_bytes,
                     void* stream);

/* ----------------------------------------------------------------------------------------
 * ed_measure_noalloc: the same measurement as ed_measure, for callers that cannot allocate
 * device memory or pass a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation). Its partial sums live in a fixed 1 MiB + 4 KiB array of
 * device memory inside the library, one copy per GPU, resolved on the first call on each device
 * and kept until the process ends; the call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine).
 * psi device, D = 2^L amplitudes; sz host [L]; norm host (may be NULL). Synchronises stream.
 * Results equal those of ed_measure bit for bit (same kernels, grid and summation order).
 * Limits: 1 <= L <= 30, else ED_ERR_ARG with a message naming the limit.
 * Concurrency: every call on one GPU shares that GPU's array; calls that overlap in time on the
 * same GPU (other threads, other streams) race and must be serialised by the caller.
 * ---------------------------------------------------------------------------------------- */
ed_status ed_measure_noalloc(const ed_c64* psi, int L, double* sz, double* norm, void* stream);

/* ----------------------------------------------------------------------------------------
 * ed_entropy: bond entropy S(l) = -sum_j Lambda_j log Lambda_j (natural log, 0 log 0 = 0) of the
 * bipartition sites 1..l | l+1..L (Sec. ed:sec:meas, bond entropy). Lambda_j are the eigenvalues of
 * rho_l = M M^dagger / <psi|psi>, M = psi reshaped to 2^l x 2^(L-l) row-major (no copy is made).
 * The Gram matrix of the smaller side is formed on the FP64 matrix cores, reduced to
 * tridiagonal form by Householder steps on the GPU, and its eigenvalues are found by bisection
 * on Sturm counts on the GPU (absolute accuracy a few eps |rho|). When every amplitude has a zero
 * imaginary part (a real state), rho is real symmetric and the Gram matrix and the reduction run
 * in real arithmetic: the same steps without their zero imaginary parts (half the bytes per
 * Householder sweep, a quarter of the matrix-core products). A NaN imaginary part counts as
 * nonzero.
 * psi        device, D amplitudes (any nonzero norm)
 * S          host; spectrum host (may be NULL): min(2^l, 2^(L-l)) eigenvalues, descending.
 * Limits: 0 <= l_cut <= L, min(l_cut, L - l_cut) <= 14. Synchronises stream.
 * Workspace: ed_entropy_workspace (the Gram matrix, 16 * 4^min(l, L-l) bytes, plus vectors).
 * ed_entropy_ex: the same, and real_arith (host, may be NULL) is set to 1 when the real
 * arithmetic ran, else 0.
 * ---------------------------------------------------------------------------------------- */
ed_status ed_entropy_workspace(int L, int l_cut, size_t* bytes);
ed_status ed_entropy(const ed_c64* psi, int L, int d, int l_cut, double* S, double* spectrum, void* ws,
                     size_t ws_bytes, void* stream);
ed_status ed_entropy_ex(const ed_c64* psi, int L, int d, int l_cut, double* S, double* spectrum, int* real_arith,
                        void* ws, size_t ws_bytes, void* stream);

/* ----------------------------------------------------------------------------------------
 * Liouville space (Sec. ed:sec:Liouville, Eqs. ed:eq:lioutrafo, ed:eq:liousuperket, App. F). The density
 * matrix rho (D x D, D = 2^L) of the Lindblad equation (Eq. ed:eq:lindbladme)
 *   d rho/dt = -i [H, rho] + sum_nu (L_nu rho L_nu^dagger - 1/2 {L_nu^dagger L_nu, rho}),
 * with L_nu = sqrt(rates[z][k-1]) J_z on site k, is stored as the superket |rho>> of D^2 entries,
 * row-major: entry j D + k is rho_jk (the row index is the high L bits). A D x D operator product
 * A rho B becomes (A (x) B^T)|rho>>.
 *
 * ed_liouville_create: a model of 2L bits for i Lcal, where d|rho>>/dt = Lcal |rho>>:
 *   i Lcal = H_eff (x) 1 - 1 (x) H_eff^* + i sum_nu L_nu (x) L_nu^*,
 *   H_eff = H - (i/2) sum_nu L_nu^dagger L_nu.
 * Then ed_apply_H(model, rho, out) gives out = i Lcal |rho>>, and ed_krylov_evolve with
 * hermitian = 0 (Arnoldi, reorth = 1) propagates |rho(t + dt)>> = exp(dt Lcal)|rho(t)>>; its
 * observables are then those of rho: sz [n_steps+1][L] = tr(sigma^z_k rho)/tr(rho) and norm =
 * tr(rho) (energy is not available). Lanczos, Trotter, trajectories and the adjoint return
 * ED_ERR_UNSUPPORTED for such a model.
 * H         host descriptor of a Hermitian H on L sites (no InfiniteFunc rules), 2 <= L <= 15.
 * jump_op   host [n_jump][2][2] complex row-major (J_z); rates host [n_jump][L] (>= 0).
 * The local part (H_eff on the row bits, -H_eff^* on the column bits) runs in the streaming passes
 * of H psi; the jump sandwiches L_nu (x) L_nu^* couple row and column bits of one site, L bits
 * apart, and are applied by one gather pass after them.
 * Errors: ED_ERR_ARG, ED_ERR_NUMERIC, ED_ERR_UNSUPPORTED (L > 15, InfiniteFunc rules), ED_ERR_HIP.
 * ---------------------------------------------------------------------------------------- */
ed_status ed_liouville_create(const ed_model_desc* H, int n_jump, const ed_c64* jump_op, const double* rates,
                              ed_model** out);
/* L of the system whose superket the model acts on (0 for a Hamiltonian model). */
ed_status ed_model_liouville_sites(const ed_model* model, int* L);

/* ed_liouville_measure: tr(rho) and <sigma^z_k> = tr(sigma^z_k rho)/tr(rho), k = 1..L, of a
 * superket rho (device, 4^L entries); sz host [L], trace host (may be NULL). Synchronises stream.
 * Workspace: ed_measure_workspace bytes (any L). */
ed_status ed_liouville_measure(const ed_c64* rho, int L, double* sz, double* trace, void* ws, size_t ws_bytes,
                               void* stream);

/* ----------------------------------------------------------------------------------------
 * ed_rdm: every single-site and every two-site reduced density matrix of a pure state (Sec. ed:sec:meas:
 * rho of the kept sites is the sum over the traced sites of psi psi^*, the kept legs in front,
 * e.g. rho_1 = [[sum A A^*, sum A B^*], [sum B A^*, sum B B^*]] for psi = [A][B]). Not normalised:
 * Tr rho = <psi|psi>.
 * psi   device, 2^L amplitudes (site 1 = most significant bit, index 0 = up).
 * rho1  device [L][2][2] complex row-major (rho_k for k = 1..L), or NULL.
 * rho2  device [L(L-1)/2][4][4] complex row-major, or NULL: rho_{k,j} for every pair k < j in
 *       lexicographic order (pair (k, j) at (k-1)L - (k-1)k/2 + j-k-1); row index 2 i_k + i_j.
 *       Both triangles are written (the lower as the conjugate of the upper).
 * The state is streamed in LDS tiles that hold 12 of its index bits; each pass evaluates the pairs
 * of its tile bits (C(m, 2) passes for all pairs, m = ceil((L - 4) / 4); then rho_k is the partial
 * trace of a nearest-neighbour pair). With rho2 NULL, rho_k is evaluated directly, every site of
 * a tile at once (ceil((L - 4) / 8) passes).
 * Limits: 2 <= L <= 30. Asynchronous on stream; deterministic (fixed reduction order).
 * Workspace: ed_rdm_workspace(L) bytes (the pair table, 64 L(L-1) bytes, plus per-workgroup sums,
 * about 35 MiB; the single-site path uses part of it).
 * Errors: ED_ERR_ARG (psi or ws NULL, L outside 2..30), ED_ERR_WORKSPACE, ED_ERR_HIP.
 * ---------------------------------------------------------------------------------------- */
ed_status ed_rdm_workspace(int L, size_t* bytes);
ed_status ed_rdm(const ed_c64* psi, int L, ed_c64* rho1, ed_c64* rho2, void* ws, size_t ws_bytes, void* stream);

/* Pairs of index bits (p < q) that ed_rdm evaluates for this L when rho2 is requested, in pass
 * order, with the pass of each. Writes min(count, max_pairs) entries of pairs [2 per pair] and
 * pass_of, and returns count (-1 for L outside 2..30). Host only. */
int ed_rdm_plan_pairs(int L, int* pairs, int max_pairs, int* pass_of);

/* Index bits that ed_rdm evaluates for this L when only rho1 is requested, in pass order, with
 * the pass of each (bit b is site L - b). Writes min(count, max_bits) entries of bits and pass_of
 * and returns count (= L; -1 for L outside 2..30). Host only. */
int ed_rdm_plan_sites(int L, int* bits, int max_bits, int* pass_of);

/* ----------------------------------------------------------------------------------------
 * ed_trace_distances: D(a_m, b_m) = 1/2 Tr |a_m - b_m|, |A| = sqrt(A^dagger A) (Sec. ed:sec:conv, the
 * distance of the error measures eps_local and eps_corr), for count pairs of n x n matrices.
 * a, b  host [count][n][n] complex row-major, meant Hermitian (only the Hermitian part of a - b
 *       enters); out host [count]. D is half the sum of the absolute eigenvalues of a - b, taken
 *       by Jacobi rotations of its real symmetric 2n x 2n form.
 * Limits: 1 <= n <= 64. Errors: ED_ERR_ARG, ED_ERR_NUMERIC (non-finite entry), ED_ERR_NOCONV.
 * ---------------------------------------------------------------------------------------- */
ed_status ed_trace_distances(int n, int count, const ed_c64* a, const ed_c64* b, double* out);

/* ----------------------------------------------------------------------------------------
 * Quantum trajectories (Sec. ed:sec:QT) of the Lindblad equation with one jump operator per site,
 * L_nu = sqrt(rate_nu) J on site nu, and H_eff = H - (i/2) sum_nu L_nu^dagger L_nu built inside.
 * Per trajectory: draw r; evolve the unnormalised state under H_eff (Krylov steps of length dt,
 * Arnoldi basis, stopping tolerance tol, at most m_max vectors) until |psi|^2 = r, the crossing
 * time being solved exactly inside the step; draw r_kappa, pick kappa with
 * P_{kappa-1} < r_kappa <= P_kappa, P the normalised cumulative sum of
 * p_nu = <psi|L_nu^dagger L_nu|psi> over sites nu = 1..L; apply L_kappa, renormalise, repeat.
 * Random numbers: trajectory t uses Philox4x64-10 with key (seed, t); draw n is word n%4 of
 * counter block (n/4 + 1, 0, 0, 0) mapped to ((w >> 11) + 1) 2^-53 in (0, 1]; draws alternate
 * threshold r, then (at each jump) r_kappa and the next r.
 * desc:  models[n_models] Hermitian parts H (one per chain length, L <= 16); rates[m] host [L_m];
 *        psi0[m] device initial states; model_of_traj host [n_traj]; jump_op host 2x2 row-major,
 *        J^dagger J must be diagonal (lowering, raising, number, dephasing) else UNSUPPORTED.
 * out:   sz host [n_traj][n_out][L_max] = <sigma^z_k>/<psi|psi> at t = n dt out_stride,
 *        n = 0..n_out-1 with n_out = n_steps/out_stride + 1 (sites k = 1..L_t, zero padded);
 *        n_jumps host [n_traj] (may be NULL); jump_t / jump_site host [n_traj][max_jumps]
 *        (may be NULL): time and site index nu-1 of the first max_jumps jumps.
 * ed_trajectories_batch runs every trajectory in one persistent kernel launch (replayed from a
 * hipGraph when stream is not NULL); ed_trajectories_plain runs the same algorithm one trajectory
 * at a time from the host (the per-instance baseline). Both synchronise stream. The effective
 * Hamiltonians' tables are built on the first call with a given H, rates and jump operator (on
 * the current device) and kept for later calls, which then allocate nothing (at most 64 are kept;
 * the oldest is dropped first).
 * ---------------------------------------------------------------------------------------- */
typedef struct {
    int n_models;
    const ed_model* const* models;
    const ed_c64* jump_op;
    const double* const* rates;
    const ed_c64* const* psi0;
    int n_traj;
    const int* model_of_traj;
    double dt;
    int n_steps;
    int out_stride;
    uint64_t seed;
} ed_traj_desc;

typedef struct {
    int m_max;
    double tol;
    int max_jumps;
} ed_traj_params;

typedef struct {
    double* sz;
    int* n_jumps;
    double* jump_t;
    int* jump_site;
} ed_traj_out;

typedef struct {
    long long total_jumps;
    long long total_krylov;
    int blocks;
    long long unconverged_steps;  /* Krylov steps that stopped at m_max with the error estimate above tol */
    int graph_replayed;           /* 1 if the batched launch replayed the stream's executable graph */
    double busy_max_ms;           /* batched launch: the longest, shortest and mean time a workgroup */
    double busy_min_ms;           /* spent on its list of trajectories (wall clock); 0 for the plain */
    double busy_mean_ms;          /* path */
} ed_traj_info;

ed_status ed_trajectories_workspace(const ed_traj_desc* desc, const ed_traj_params* params, size_t* bytes);
ed_status ed_trajectories_batch(const ed_traj_desc* desc, const ed_traj_params* params, const ed_traj_out* out,
                                ed_traj_info* info, void* ws, size_t ws_bytes, void* stream);
ed_status ed_trajectories_plain_workspace(const ed_traj_desc* desc, const ed_traj_params* params, size_t* bytes);
ed_status ed_trajectories_plain(const ed_traj_desc* desc, const ed_traj_params* params, const ed_traj_out* out,
                                ed_traj_info* info, void* ws, size_t ws_bytes, void* stream);

/* ed_stream_copy: dst[i] = src[i] for n amplitudes (device arrays, not overlapping), one amplitude
 * per thread with streaming stores: a plain device copy that measures the practical HBM streaming
 * rate against which the benchmarks' kernels are compared. Asynchronous on stream. */
ed_status ed_stream_copy(const ed_c64* src, ed_c64* dst, int64_t n, void* stream);

/* Raw 64-bit words n = 0..count-1 of the trajectory random stream of key (seed, id), written to
 * device memory out (for checking the generator against its published definition). Async. */
ed_status ed_philox_words(uint64_t seed, uint64_t id, uint64_t* out, int64_t count, void* stream);

/* ----------------------------------------------------------------------------------------
 * Adjoint gradient of a final-time observable with respect to piecewise-constant bond couplings.
 * Evolution: psi_s = exp(-i H_s slice_len) psi_{s-1}, s = 1..n_slices, with
 *   H_s = sum_b J[s-1][b] h_b + (site terms of tmpl),  h_b = the bond operator of tmpl on bond b
 *   (sites b+1, b+2, b = 0..L-2, as folded from tmpl's bond rules);
 * each slice is propagated by `substeps` Krylov steps (Sec. ed:sec:krylov; Lanczos with local
 * re-projection, m_fixed vectors if > 0, else adaptive with tol, at most m_max).
 * Loss = <psi_S|O|psi_S>, O = sum_k obs_w[k-1] sigma^z_k. The gradient is back-propagated:
 * lam_S = O psi_S, lam_{s-1} = exp(+i H_s slice_len) lam_s, and
 *   dLoss/dJ[s][b] = 2 int_0^slice_len Im <mu(tau)|h_b|phi(tau)> dtau,
 *   phi(tau) = exp(-i H_s tau) psi_{s-1}, mu(tau) = exp(-i H_s tau) lam_{s-1},
 * by Gauss-Legendre quadrature with quad_nodes nodes per sub-step. psi_s are kept at slice
 * boundaries (checkpoints) and recomputed inside slices.
 * J host [n_slices][L-1]; psi0 device; obs_w host [L]; loss host; grad host [n_slices][L-1].
 * Limits: L <= 24. Synchronises stream. ed_evolve_loss runs the forward pass only (loss), with
 * the same discretisation: the per-parameter baseline for finite differences.
 * ---------------------------------------------------------------------------------------- */
typedef struct {
    int substeps;
    int quad_nodes;
    int m_max;
    int m_fixed;
    double tol;
} ed_adjoint_params;

ed_status ed_adjoint_workspace(const ed_model* tmpl, int n_slices, const ed_adjoint_params* params, size_t* bytes);
ed_status ed_evolve_adjoint(const ed_model* tmpl, int n_slices, double slice_len, const double* J, const ed_c64* psi0,
                            const double* obs_w, const ed_adjoint_params* params, double* loss, double* grad, void* ws,
                            size_t ws_bytes, void* stream);
ed_status ed_evolve_loss_workspace(const ed_model* tmpl, const ed_adjoint_params* params, size_t* bytes);
ed_status ed_evolve_loss(const ed_model* tmpl, int n_slices, double slice_len, const double* J, const ed_c64* psi0,
                         const double* obs_w, const ed_adjoint_params* params, double* loss, void* ws, size_t ws_bytes,
                         void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ED_H */
