"""Benchmark of the exact-diagonalisation hot path on one MI355X.

Headline (the JSON line's value): matrix-free H psi (ed_apply_H) on the open transverse-field
Ising chain, L = 28, g = 0.5 (2^28 complex128 amplitudes, 4 GiB per vector), reported as
algorithmic GB/s = 32 B per amplitude (read psi once, write H psi once) / time per product,
and as a fraction of the 8 TB/s HBM peak. A step is one H psi over the whole state; the state
is resident in HBM and the time comes from HIP events on the stream the library launches on.

The JSON line also carries the bytes the counters saw per H psi over the same time and the rate of
a plain 4 GiB device copy on the box ("hbm_measured").

Beside it, each remaining row of the hot path is run once on its synthetic workload and reported
under "rows": an H psi sweep over L = 20..28 (TFIM and XXZ), Lanczos ground state (TFIM L = 14,
with the oracle's textbook Lanczos timed beside it), Lanczos + half-chain entropy (XXZ L = 26),
the L = 28 Krylov quench (100 steps), the same quench with the Suzuki-Trotter propagators of order
4 and 2, the long-range Ising chain H_LRQI at L = 28 (H psi and a Krylov quench), 4096 batched
quantum trajectories against the plain per-trajectory path, the reduced density matrices at
L = 28, the L = 14 Liouville-space evolution (2^28 superket), and the adjoint gradient (L = 20)
against finite differences of the forward-only path. The CPU oracle is timed on a bounded sample
of the headline workload (its CSR product at L = 22 for about 10 s).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def host_info():
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu": cpu, "omp_threads": os.environ.get("OMP_NUM_THREADS")}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


HPSI_SOURCES = ["paper_1802_10052_amd/csrc/apply_h.hip", "paper_1802_10052_amd/csrc/hpsi_device.h",
                "paper_1802_10052_amd/csrc/model.cpp", "paper_1802_10052_amd/csrc/ed_internal.h"]
TRAFFIC_PROFILE = "profiles/hpsi_tile_L28_tfim.md"


def measured_traffic(plan_desc):
    """HBM bytes (read + written) per H psi of the plan `plan_desc` from the committed rocprofv3
    counter summary, if it was taken on the H psi kernels as they are now (same source hash) and
    lists that plan; otherwise None. Summary lines: "source-hash: <hex>" and
    "traffic-bytes-per-apply[<plan description>]: <bytes>"."""
    import hashlib
    try:
        h = hashlib.sha256()
        for f in HPSI_SOURCES:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        cur = h.hexdigest()[:16]
        rec, traffic = None, None
        key = f"traffic-bytes-per-apply[{plan_desc}]:"
        for line in open(os.path.join(ROOT, TRAFFIC_PROFILE)):
            if line.startswith("source-hash:"):
                rec = line.split(":", 1)[1].strip()
            if line.startswith(key):
                traffic = float(line[len(key):])
        return traffic if rec == cur else None
    except OSError:
        return None


def cpu_baseline(L=22, budget_s=10.0, max_reps=200):
    """The oracle's explicit sparse H psi (scipy CSR matvec, single-threaded) at L = 22, repeated
    for about budget_s seconds (the CSR build is not timed)."""
    import edinputs as E
    from oracle import hamiltonian as OH
    H = OH.hamiltonian_sparse(E.tfim(L, 0.5))
    psi = E.random_state(L, 11)
    H @ psi
    reps = 0
    t0 = time.perf_counter()
    while reps < max_reps and (reps == 0 or time.perf_counter() - t0 < budget_s):
        H @ psi
        reps += 1
    dt = (time.perf_counter() - t0) / reps
    return {"value": round(32.0 * (1 << L) / dt / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"scipy CSR H psi (oracle, {H.nnz} nonzeros), TFIM g=0.5 L={L} (2^{L} amplitudes), {reps} "
                      f"products of {dt * 1e3:.1f} ms ({reps * dt:.1f} s); same 32 B/amplitude accounting as the "
                      f"headline; the L=28 product would need a ~190 GB CSR matrix"}


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max((i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas"), default=None)
    except ImportError:
        return None


def _oracle_traj_task(args):
    """One worker of the trajectory oracle timing: n trajectories of one length, `steps` steps."""
    L, ids, steps = args
    try:  # one core per worker: the products are small, threads would only contend
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except ImportError:
        pass
    import edinputs as E
    from oracle import hamiltonian as OH
    from oracle import trajectories as OT
    H = OH.hamiltonian_sparse(E.xxz(L, 1.0, 1.0))
    jumps = OT.lowering_jumps(L, 0.1)
    psi0 = E.product_state(L, E.neel_index(L))
    t0 = time.perf_counter()
    for tr in ids:
        OT.trajectory(H, jumps, psi0, 0.01, steps, 10, 4, tr, m_max=20, tol=1e-10)
    return L, len(ids) * steps, time.perf_counter() - t0


def oracle_trajectories():
    """Quantum trajectories of every chain length on the host, one worker process (one BLAS thread)
    per length. Runs before the process touches the GPU, so the workers start from a process
    without GPU state."""
    import multiprocessing as mp
    tasks = [(L, [2 * k, 2 * k + 1], 10) for k, L in enumerate((8, 10, 12, 14, 16))]
    workers = max(1, min(16, os.cpu_count() or 1, len(tasks)))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_traj_task, tasks)
    wall = time.perf_counter() - t0
    return {"oracle_cores": workers, "oracle_wall_s": round(wall, 3),
            "oracle_ms_per_trajectory_step": {f"L{L}": round(1e3 * sec / n, 2) for L, n, sec in res},
            "sample": "2 trajectories per length, 10 steps of dt = 0.01, one process (one BLAS thread) per length"}


def oracle_rows(P, E, torch, dev, traj_oracle=None):
    """The oracle timed on the host beside the workloads it can finish in seconds, each next to the
    GPU path at the same size: XXZ ground state (ARPACK on the explicit sparse H, the paper's
    statics) and its half-chain entropy (SVD) at L = 18; the transverse-field Ising quench (textbook
    Krylov steps on the sparse H) at L = 18; quantum trajectories of every chain length over a
    process pool; the adjoint gradient from the dense eigendecomposition at L = 10 (5 slices)."""
    import numpy as np
    from oracle import adjoint as OA
    from oracle import hamiltonian as OH
    from oracle import krylov as OK
    from oracle import lanczos as OL
    from oracle import observables as OO
    info = {"nproc": os.cpu_count(), "blas_threads": _blas_threads()}
    out = {"host": info}
    # ground state + entropy, L = 18
    L = 18
    desc = E.xxz(L, 1.0, 0.5, E.random_fields(L, 2))
    t0 = time.perf_counter()
    H = OH.hamiltonian_sparse(desc)
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    e_or, psi_or = OL.ground_state_eigsh(H, tol=1e-14)
    t_eigsh = time.perf_counter() - t0
    t0 = time.perf_counter()
    s_or = OO.bond_entropy(psi_or, L, L // 2)
    t_svd = time.perf_counter() - t0
    m = P.Model(desc)
    v0 = E.random_state_device(L, 3, dev)
    P.lanczos_ground(m, v0, tol=1e-10, max_iter=1000, max_basis=24, n_keep=5, reorth="partial")
    with Timer(torch, None) as tg:
        e_g, psi_g, _ = P.lanczos_ground(m, v0, tol=1e-10, max_iter=1000, max_basis=24, n_keep=5, reorth="partial")
    with Timer(torch, None) as te:
        s_g = P.entropy(psi_g, L, L // 2)
    out["xxz_ground_entropy_L18"] = {
        "oracle_build_s": round(t_build, 3), "oracle_eigsh_s": round(t_eigsh, 3), "oracle_svd_entropy_s": round(t_svd, 4),
        "oracle_cores": "eigsh: 1 (sparse matvec) + BLAS", "gpu_lanczos_s": round(tg.s, 4), "gpu_entropy_s": round(te.s, 4),
        "E0_rel_diff": abs(e_g - e_or) / abs(e_or), "S_rel_diff": abs(s_g - s_or) / abs(s_or)}
    del m, v0, psi_g, H
    # quench, L = 18, 10 steps
    L, steps = 18, 10
    desc = E.tfim(L, 0.5)
    H = OH.hamiltonian_sparse(desc)
    psi = E.product_state(L, 0)
    t0 = time.perf_counter()
    for _ in range(steps):
        psi, _m = OK.krylov_step(lambda v: H @ v, psi, 0.05, m_max=20, tol=1e-10)
    t_or = (time.perf_counter() - t0) / steps
    m = P.Model(desc)
    g = torch.zeros(1 << L, dtype=torch.complex128, device=dev)
    g[0] = 1.0
    P.krylov_evolve(m, g.clone(), 0.05, 2, m_max=20, tol=1e-10)
    with Timer(torch, None) as tq:
        P.krylov_evolve(m, g, 0.05, steps, m_max=20, tol=1e-10)
    out["tfim_quench_L18"] = {"steps": steps, "oracle_ms_per_step": round(1e3 * t_or, 2), "oracle_cores": 1,
                              "gpu_ms_per_step": round(1e3 * tq.s / steps, 3),
                              "final_state_overlap_err": float(1 - abs(np.vdot(psi, g.cpu().numpy())) /
                                                               (np.linalg.norm(psi) * torch.linalg.vector_norm(g).item()))}
    del m, g, H
    if traj_oracle is not None:
        out["trajectories"] = traj_oracle
    # adjoint gradient, L = 10: the oracle's dense eigendecomposition gradient on the first 5 of the
    # 50 slices (its cost is per slice), the GPU on the same 5 slices
    L, S = 10, 5
    tmpl = E.xxz_bond_scaled(L, 0.5, np.ones(L - 1))
    J = E.adjoint_couplings(50, L - 1, 5)[:S]
    psi0 = E.product_state(L, E.neel_index(L))
    w = np.array([(-1) ** k for k in range(L)], np.float64) / L
    t0 = time.perf_counter()
    lo, go = OA.gradient_eig(tmpl, J, psi0, 0.1, w)
    t_or = time.perf_counter() - t0
    m = P.Model(tmpl)
    p0 = torch.from_numpy(psi0).to(dev)
    P.evolve_adjoint(m, J, p0, 0.1, w, substeps=2, quad_nodes=8)
    with Timer(torch, None) as ta:
        lg, gg = P.evolve_adjoint(m, J, p0, 0.1, w, substeps=2, quad_nodes=8)
    out["adjoint_L10"] = {"slices": S, "n_params": int(S * (L - 1)), "oracle_s": round(t_or, 3),
                          "oracle_s_per_slice": round(t_or / S, 3), "oracle_cores": info["blas_threads"],
                          "gpu_s": round(ta.s, 4),
                          "grad_max_abs_diff_over_max": float(np.max(np.abs(gg - go)) / np.max(np.abs(go)))}
    return out


class Timer:
    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.t0 = time.perf_counter()
        return self

    def __exit__(self, *a):
        self.torch.cuda.synchronize()
        self.s = time.perf_counter() - self.t0


def row_hpsi_sweep(P, E, torch, dev, reps=10):
    """H psi over L = 20..28 for the transverse-field Ising chain (g = 0.5) and the XXZ chain
    (Delta = 0.5, h ~ U[-0.5, 0.5]): tuned plan, passes, ms per product and algorithmic GB/s."""
    out = {"workload": "apply_H, TFIM g=0.5 and XXZ Delta=0.5 h~U[-0.5,0.5], L=20..28, tuned plans"}
    for L in (20, 22, 24, 26, 28):
        for name, desc in (("tfim", E.tfim(L, 0.5)), ("xxz", E.xxz(L, 1.0, 0.5, E.random_fields(L, 2)))):
            m = P.Model(desc)
            psi = E.random_state_device(L, 11, dev)
            o = torch.empty_like(psi)
            best, _ = m.tune(psi, o, reps=2)
            P.apply_H(m, psi, o)
            with Timer(torch, None) as t:
                for _ in range(reps):
                    P.apply_H(m, psi, o)
            ms = 1e3 * t.s / reps
            out[f"{name}{L}"] = {"ms": round(ms, 4), "GBps": round(32.0 * (1 << L) / (ms * 1e-3) / 1e9, 1),
                                 "passes": m.passes, "plan": m.describe_plan(best)}
            del psi, o, m
            torch.cuda.empty_cache()
    return out


def row_lanczos_L14(P, E, torch, dev):
    from tests import closed_forms as CF
    L = 14
    m = P.Model(E.tfim(L, 1.0))
    v0 = torch.from_numpy(E.random_state(L, 1)).to(dev)
    P.lanczos_ground(m, v0, tol=1e-10, max_iter=200)
    with Timer(torch, None) as t:
        e0, psi, info = P.lanczos_ground(m, v0, tol=1e-10, max_iter=200)
    ref = CF.tfim_bdg_ground_energy(L, 1.0, 1.0)
    # the oracle beside it: textbook Lanczos on the explicit CSR matrix (one core for the matvecs)
    import edinputs
    from oracle import hamiltonian as OH
    from oracle import lanczos as OL
    H = OH.hamiltonian_sparse(edinputs.tfim(L, 1.0))
    t0 = time.perf_counter()
    e_or = OL.lanczos_ground(lambda v: H @ v, edinputs.random_state(L, 1), tol=1e-10, max_iter=200)[0]
    t_or = time.perf_counter() - t0
    return {"workload": "TFIM g=1 L=14 Lanczos, full reorthogonalisation, tol 1e-10", "seconds": round(t.s, 4),
            "iters": info["iters"], "E0": e0, "rel_err_vs_free_fermion": abs(e0 - ref) / abs(ref),
            "residual": info["residual"], "oracle_seconds": round(t_or, 3),
            "oracle_E0_rel_diff": abs(e_or - e0) / abs(e0)}


def row_lanczos_entropy_L26(P, E, torch, dev):
    import numpy as np
    L = 26
    desc = E.xxz(L, 1.0, 0.5, E.random_fields(L, 2))
    m = P.Model(desc)
    # a real start vector: the Hamiltonian is real, so every Lanczos vector and the ground state
    # stay exactly real, and the entropy takes the real-arithmetic reduction
    v0 = E.random_state_device(L, 3, dev, real=True)
    with Timer(torch, None) as t:
        e0, psi, info = P.lanczos_ground(m, v0, tol=1e-10, max_iter=1000, max_basis=24, n_keep=5, reorth="partial")
    del v0
    torch.cuda.empty_cache()
    rec = {"workload": "XXZ J=1 Delta=0.5 h~U[-0.5,0.5] L=26, Lanczos from a real random vector with at most 24 "
                       "stored vectors (thick restart keeping 5 Ritz vectors, partial reorthogonalisation), tol "
                       "1e-10, half-chain entropy 2^13 x 2^13",
           "lanczos_seconds": round(t.s, 3), "iters": info["iters"], "restarts": info["restarts"],
           "extra_reorth": info["extra_reorth"], "E0": e0, "residual": info["residual"],
           "converged": info["converged"]}
    try:
        with Timer(torch, None) as te:
            S, inf = P.entropy(psi, L, L // 2, info=True)
        rec.update({"entropy": S, "entropy_seconds": round(te.s, 3), "entropy_real_arith": inf["real_arith"]})
        # the same state times a global phase: same entropy, complex arithmetic
        psi *= complex(np.cos(0.7), np.sin(0.7))
        with Timer(torch, None) as tc:
            Sc, infc = P.entropy(psi, L, L // 2, info=True)
        rec.update({"entropy_seconds_complex_arith": round(tc.s, 3),
                    "entropy_complex_arith_rel_diff": abs(Sc - S) / abs(S), "complex_real_arith": infc["real_arith"]})
    except Exception as e:
        rec["entropy_error"] = f"{type(e).__name__}: {e}"
    return rec


def row_quench_L28(P, E, torch, dev, steps=100):
    L = 28
    m = P.Model(E.tfim(L, 0.5))
    psi = torch.zeros(1 << L, dtype=torch.complex128, device=dev)
    psi[0] = 1.0
    with Timer(torch, None) as t:
        _, obs, info = P.krylov_evolve(m, psi, 0.05, steps, m_max=20, tol=1e-10, reorth=0)
    e = obs["energy"]
    _SHARED["quench28_sz"] = obs["sz"]
    r1, r2 = P.rdm(psi, L)
    _SHARED["quench28_rdm"] = (r1.cpu().numpy(), r2.cpu().numpy())
    return {"workload": f"TFIM g=0.5 L=28 quench from all up, dt=0.05, {steps} Krylov steps, m<=20, tol 1e-10",
            "seconds": round(t.s, 3), "ms_per_step": round(1e3 * t.s / steps, 2), "total_krylov": info["total_m"],
            "max_m": info["max_m"], "energy_drift": float(abs(e - e[0]).max() / abs(e[0])),
            "norm_drift": float(abs(obs["norm"] - 1).max()), "sz_final_site1": float(obs["sz"][-1, 0])}


_SHARED = {}


def row_trotter_L28(P, E, torch, dev, steps=100):
    """The L = 28 quench of the Krylov row with the Suzuki-Trotter propagators (Sec. ed:sec:trotter):
    orders 4 and 2, per-step time, the algorithmic bandwidth of the gate passes (each pass reads and
    writes the state once: 32 B per amplitude; the library reports the passes of a step, runs of
    four layers fused) and the largest difference of <sigma^z_k>(t) from the Krylov run when that
    row ran before."""
    import numpy as np
    L, dt = 28, 0.05
    m = P.Model(E.tfim(L, 0.5))
    out = {"workload": f"TFIM g=0.5 L=28 quench from all up, dt=0.05, {steps} Trotter steps (order 4 and 2)"}
    layers = {4: 11, 2: 3}
    for order in (4, 2):
        npass = P.trotter_passes(m, order)
        psi = torch.zeros(1 << L, dtype=torch.complex128, device=dev)
        psi[0] = 1.0
        with Timer(torch, None) as t:
            _, obs = P.trotter_evolve(m, psi, dt, steps, order=order)
        per_step = t.s / steps
        nbytes = npass * 32.0 * (1 << L)
        r = {"seconds": round(t.s, 3), "ms_per_step": round(1e3 * per_step, 2), "layers": layers[order],
             "passes_per_step": npass,
             "gate_pass_GBps": round(nbytes / per_step / 1e9, 1), "norm_drift": float(abs(obs["norm"] - 1).max()),
             "sz_final_site1": float(obs["sz"][-1, 0])}
        ref = _SHARED.get("quench28_sz")
        if ref is not None:
            r["max_abs_sz_diff_vs_krylov"] = float(np.abs(obs["sz"] - ref).max())
        ref = _SHARED.get("quench28_rdm")
        if ref is not None:  # the error measures of the convergence study, Krylov as the reference
            g1, g2 = P.rdm(psi, L)
            r["eps_local_vs_krylov"] = P.eps_local(g1, ref[0])
            r["eps_corr_vs_krylov"] = P.eps_corr(g2, ref[1])
        out[f"order{order}"] = r
        del psi
    return out


def row_lrqi_L28(P, E, torch, dev, reps=10, steps=20):
    """The long-range quantum Ising chain H_LRQI (App. A InfiniteFunc rule, f(r) = 1/r^alpha,
    phi = pi/4, alpha = 1.5) at L = 28: the tuned H psi with its O(L^2) diagonal fused into the
    first pass (same 32 B per amplitude accounting as the headline), and a Krylov quench from all
    up, the paper's case for Krylov over Trotter (Trotter layers do not cover long-range terms)."""
    import numpy as np
    L = 28
    m = P.Model(E.lrqi(L, np.pi / 4, 1.5))
    psi = E.random_state_device(L, 11, dev)
    out = torch.empty_like(psi)
    best, plan_ms = m.tune(psi, out, reps=3)
    P.apply_H(m, psi, out)
    with Timer(torch, None) as t:
        for _ in range(reps):
            P.apply_H(m, psi, out)
    ms = 1e3 * t.s / reps
    rec = {"workload": f"H_LRQI phi=pi/4 alpha=1.5 L=28: apply_H ({reps} products) and a quench from all up, "
                       f"dt=0.05, {steps} Krylov steps, m<=20, tol 1e-10",
           "apply_ms": round(ms, 3), "apply_GBps": round(32.0 * (1 << L) / (ms * 1e-3) / 1e9, 1),
           "plan": m.describe_plan(best)}
    del psi, out
    torch.cuda.empty_cache()
    psi = torch.zeros(1 << L, dtype=torch.complex128, device=dev)
    psi[0] = 1.0
    with Timer(torch, None) as t:
        _, obs, info = P.krylov_evolve(m, psi, 0.05, steps, m_max=20, tol=1e-10, reorth=0)
    e = obs["energy"]
    rec.update({"quench_seconds": round(t.s, 3), "quench_ms_per_step": round(1e3 * t.s / steps, 2),
                "total_krylov": info["total_m"], "max_m": info["max_m"],
                "energy_drift": float(abs(e - e[0]).max() / max(1.0, abs(e[0]))),
                "norm_drift": float(abs(obs["norm"] - 1).max()), "sz_final_site1": float(obs["sz"][-1, 0])})
    return rec


def row_rdm_L28(P, E, torch, dev, reps=3):
    """All single-site and all two-site reduced density matrices (Sec. ed:sec:meas) of a random L = 28
    state: 378 pairs in 15 LDS-tiled passes. Algorithmic work: the 6 upper off-diagonal entries of
    each pair's 4x4 matrix are complex multiply-adds over the 2^(L-2) quads of amplitudes (48
    flops per quad and pair); the 4 diagonal entries are marginals of |psi|^2, summed once per
    amplitude and pass (4 flops). The products are not a dense contraction, so the bound is the
    FP64 vector peak (78.6 TFLOP/s). Also timed: the single-site matrices alone (every site's 2x2
    matrix directly, 3 passes over the state, each reading it once: HBM-bound)."""
    L = 28
    psi = E.random_state_device(L, 12, dev)
    pairs, pass_of = P.rdm_plan(L)
    passes = int(pass_of.max()) + 1
    P.rdm(psi, L)
    with Timer(torch, None) as t:
        for _ in range(reps):
            P.rdm(psi, L)
    ms = 1e3 * t.s / reps
    flops = 48.0 * len(pairs) * float(1 << (L - 2)) + 4.0 * passes * float(1 << L)
    P.rdm(psi, L, two_site=False)
    with Timer(torch, None) as t1:
        for _ in range(reps):
            P.rdm(psi, L, two_site=False)
    ms1 = 1e3 * t1.s / reps
    passes1 = int(P.rdm_plan_sites(L)[1].max()) + 1
    gbs1 = passes1 * 16.0 * float(1 << L) / (ms1 * 1e-3) / 1e9  # each pass streams the state once
    tf = flops / (ms * 1e-3) / 1e12
    return {"workload": "rho_k for all 28 sites and rho_{k,j} for all 378 pairs of a random L=28 state",
            "all_pairs_ms": round(ms, 2), "all_pairs_TFLOPs": round(tf, 2),
            "frac_fp64_vector_peak": round(tf / 78.6, 4), "passes": passes,
            "single_site_only_ms": round(ms1, 2), "single_site_passes": passes1,
            "single_site_GBps": round(gbs1, 1), "single_site_frac_hbm_peak": round(gbs1 / 8000.0, 4)}


def row_liouville_L14(P, E, torch, dev, reps=5, steps=10):
    """Liouville-space evolution (Sec. ed:sec:Liouville) of the dissipative XXZ chain of the trajectory row
    (J = 1, Delta = 1, gamma = 0.1 sigma^- on every site) at L = 14: the density matrix as a 2^28
    superket (4 GiB). Reported: one product i Lcal |rho>> (the tuned streaming passes of the local
    part plus the jump gather pass; GB/s on the headline's 32 B per amplitude), and Arnoldi time
    steps from the Neel state with the exact decay identity sum_k <sigma^z_k>(t) = L (e^{-gamma t} - 1)
    and the trace as checks."""
    import numpy as np
    L, gamma, dt = 14, 0.1, 0.05
    sm = np.array([[0, 0], [1, 0]], np.complex128)
    m = P.Liouville(E.xxz(L, 1.0, 1.0), [sm], np.full((1, L), gamma))
    D2 = 1 << (2 * L)
    x = E.random_state_device(2 * L, 3, dev)
    out = torch.empty_like(x)
    best, _ = m.tune(x, out, reps=2)
    P.apply_H(m, x, out)
    with Timer(torch, None) as t:
        for _ in range(reps):
            P.apply_H(m, x, out)
    ms = 1e3 * t.s / reps
    del x, out
    torch.cuda.empty_cache()
    rho = torch.zeros(D2, dtype=torch.complex128, device=dev)
    n = E.neel_index(L)
    rho[n * (1 << L) + n] = 1.0
    with Timer(torch, None) as te:
        _, obs, info = P.krylov_evolve(m, rho, dt, steps, m_max=30, tol=1e-10, hermitian=False)
    tt = dt * np.arange(steps + 1)
    ident = float(np.abs(obs["sz"].sum(axis=1) - L * (np.exp(-gamma * tt) - 1)).max())
    return {"workload": f"dissipative XXZ (Delta=1, gamma=0.1 sigma^-) L=14 as a 2^28 superket: i Lcal |rho>> "
                        f"({reps} products) and {steps} Arnoldi steps of dt={dt} from the Neel state (m<=30, tol 1e-10)",
            "apply_ms": round(ms, 3), "apply_GBps": round(32.0 * D2 / (ms * 1e-3) / 1e9, 1),
            "plan": m.describe_plan(best), "evolve_seconds": round(te.s, 3),
            "ms_per_step": round(1e3 * te.s / steps, 1), "total_krylov": info["total_m"], "max_m": info["max_m"],
            "second_gs_passes_skipped": info["reorth_skipped"],
            "decay_identity_max_err": ident, "trace_drift": float(np.abs(obs["norm"] - 1).max())}


def row_trajectories(P, E, torch, dev, n_traj=4096, plain_sample=10):
    import numpy as np
    lengths = [8, 10, 12, 14, 16]
    gamma = 0.1
    models = [P.Model(E.xxz(L, 1.0, 1.0)) for L in lengths]
    rates = [np.full(L, gamma) for L in lengths]
    psi0 = [torch.from_numpy(E.product_state(L, E.neel_index(L))).to(dev) for L in lengths]
    mo = np.array([t % 5 for t in range(n_traj)], np.int32)
    dt, steps, stride, seed = 0.01, 500, 10, 4
    with Timer(torch, None) as t:
        res = P.trajectories(models, E.SMINUS, rates, psi0, mo, dt, steps, stride, seed, m_max=20, tol=1e-10)
    n_out = steps // stride + 1
    times = np.arange(n_out) * dt * stride
    # ensemble check: mean of sum_k sz_k = -2 <jumps>  -> L (exp(-gamma t) - 1) per length
    ens = {}
    for i, L in enumerate(lengths):
        sel = mo == i
        tot = res["sz"][sel][:, :, :L].sum(axis=2)
        mean = tot.mean(axis=0)
        sem = tot.std(axis=0, ddof=1) / np.sqrt(sel.sum()) + 1e-12
        z = np.abs(mean - L * (np.exp(-gamma * times) - 1)) / sem
        ens[f"L{L}"] = round(float(z.max()), 3)
    # plain per-trajectory path on a sample (two of each length), time per trajectory-step
    ids = np.concatenate([np.where(mo == i)[0][:plain_sample // 5] for i in range(5)])
    sub = mo[ids]
    with Timer(torch, None) as tp:
        rp = P.trajectories(models, E.SMINUS, rates, psi0, sub, dt, steps, stride, seed, m_max=20, tol=1e-10,
                            plain=True)
    # the plain path's trajectory t of the sample has id t, not ids[t]: compare cost only
    traj_steps_batched = n_traj * steps
    plain_per_len = tp.s / len(ids)
    est_plain = plain_per_len * n_traj
    return {"workload": "4096 dissipative XXZ trajectories (J=1, Delta=1, gamma=0.1 sigma^- on every site), "
                        "L in {8..16} mixed, Neel start, dt=0.01, T=5, one persistent launch",
            "batched_seconds": round(t.s, 3), "trajectory_steps_per_s": round(traj_steps_batched / t.s, 1),
            "total_jumps": res["info"]["total_jumps"], "blocks": res["info"]["blocks"],
            "unconverged_krylov_steps": res["info"]["unconverged_steps"],
            "workgroup_busy_ms": {k: round(v, 1) for k, v in res["info"]["busy_ms"].items()},
            "plain_sample_trajectories": int(len(ids)), "plain_sample_seconds": round(tp.s, 3),
            "plain_estimated_seconds_4096": round(est_plain, 1),
            "speedup_vs_plain": round(est_plain / t.s, 2),
            "ensemble_max_z_sum_sz": ens}


def row_trajectories_L16(P, E, torch, dev, n_traj=512, steps=20):
    """The L = 16 slice of the trajectory workload on its own (the chain length that dominates its
    cost): 512 trajectories, 20 steps of dt = 0.01, one persistent launch. For profiling."""
    import numpy as np
    L, gamma = 16, 0.1
    m = P.Model(E.xxz(L, 1.0, 1.0))
    psi0 = torch.from_numpy(E.product_state(L, E.neel_index(L))).to(dev)
    mo = np.zeros(n_traj, np.int32)
    with Timer(torch, None) as t:
        res = P.trajectories([m], E.SMINUS, [np.full(L, gamma)], [psi0], mo, 0.01, steps, 10, 4, m_max=20, tol=1e-10)
    return {"workload": f"{n_traj} dissipative XXZ trajectories at L={L} (J=1, Delta=1, gamma=0.1), Neel start, "
                        f"dt=0.01, {steps} steps, one persistent launch",
            "seconds": round(t.s, 4), "trajectory_steps_per_s": round(n_traj * steps / t.s, 1),
            "krylov_vectors_per_step": round(res["info"]["total_krylov"] / (n_traj * steps), 3),
            "unconverged_krylov_steps": res["info"]["unconverged_steps"],
            "total_jumps": res["info"]["total_jumps"], "blocks": res["info"]["blocks"]}


def row_adjoint(P, E, torch, dev, fd_sample=4):
    import numpy as np
    L, S = 20, 50
    tmpl = E.xxz_bond_scaled(L, 0.5, np.ones(L - 1))
    J = E.adjoint_couplings(S, L - 1, 5)
    psi0 = torch.from_numpy(E.product_state(L, E.neel_index(L))).to(dev)
    w = np.array([(-1) ** k for k in range(L)], np.float64) / L
    m = P.Model(tmpl)
    kw = dict(substeps=2, m_fixed=20, m_max=30)
    P.evolve_adjoint(m, J, psi0, 0.1, w, quad_nodes=8, **kw)
    with Timer(torch, None) as t:
        loss, g = P.evolve_adjoint(m, J, psi0, 0.1, w, quad_nodes=8, **kw)
    # plain path: central differences need 2 forward runs per parameter (1900 in total)
    h = 1e-6
    errs = []
    with Timer(torch, None) as tf:
        for k in range(fd_sample):
            s, b = [(49, 9), (0, 0), (25, 18), (10, 3)][k]
            Jp, Jm = J.copy(), J.copy()
            Jp[s, b] += h
            Jm[s, b] -= h
            fd = (P.evolve_loss(m, Jp, psi0, 0.1, w, **kw) - P.evolve_loss(m, Jm, psi0, 0.1, w, **kw)) / (2 * h)
            errs.append(abs(g[s, b] - fd) / max(abs(fd), 1e-3 * np.max(np.abs(g))))
    per_forward = tf.s / (2 * fd_sample)
    est_fd = per_forward * 2 * S * (L - 1)
    return {"workload": "XXZ L=20 Delta=0.5, 50 slices x 0.1, J~U[0.5,1.5], Neel, staggered magnetisation",
            "adjoint_seconds": round(t.s, 3), "loss": loss, "n_params": int(S * (L - 1)),
            "forward_seconds": round(per_forward, 4), "fd_estimated_seconds": round(est_fd, 1),
            "speedup_vs_fd": round(est_fd / t.s, 1), "fd_sample_max_rel_err": float(max(errs))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=28)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain device copy of the 4 GiB state first (known bytes, for scaling "
                         "the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--plan", default=None,
                    help="use the H psi plan with this description (ed_model_plan_describe) instead of tuning")
    ap.add_argument("--rows", default="all",
                    help="comma list of hpsi_sweep,lanczos14,lanczos26,quench28,trotter28,lrqi28,rdm28,liouville14,traj,adjoint (the 'all' set) and traj16 "
                         "(the L=16 trajectory slice, for profiling); 'none' or 'all'")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for --gpus {args.gpus}); the multi-GPU layout is a design note, "
              f"not a measured path", file=sys.stderr)
        sys.exit(2)

    traj_oracle = None
    if not args.no_cpu_baseline and args.rows != "none":
        log("bench: oracle trajectories (host, before the GPU is used)")
        try:
            traj_oracle = oracle_trajectories()
        except Exception as e:  # reported, not hidden
            traj_oracle = {"error": f"{type(e).__name__}: {e}"}

    import torch
    import edinputs as E
    import paper_1802_10052_amd as P

    dev = "cuda:0"
    L = args.L
    D = 1 << L
    model = P.Model(E.tfim(L, 0.5))
    psi = E.random_state_device(L, 11, dev)
    out = torch.empty_like(psi)
    stream = torch.cuda.current_stream()
    # the practical HBM rate on this machine: the library's plain streaming copy of the state (one
    # amplitude per thread; reads and writes 4 GiB), and torch's copy_ beside it
    def copy_rate(fn):
        fn()
        torch.cuda.synchronize()
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        for _ in range(5):
            fn()
        c1.record(stream)
        torch.cuda.synchronize()
        return 32.0 * D / (c0.elapsed_time(c1) / 5 * 1e-3) / 1e9
    copy_gbs = copy_rate(lambda: P.stream_copy(psi, out))
    torch_copy_gbs = copy_rate(lambda: out.copy_(psi))
    if args.copy_calibration:
        P.stream_copy(psi, out)
        torch.cuda.synchronize()
        log(f"bench: calibration copy (ed_stream_copy) of {16 * D} bytes read + {16 * D} bytes written")
    if args.plan is None:
        best, plan_ms = model.tune(psi, out, reps=3)
        log(f"bench: tuned H psi plan {best} of {len(plan_ms)}")
        for i, t in enumerate(plan_ms):
            log(f"bench:   plan {i:2d} {t:8.3f} ms  {model.describe_plan(i)}")
    else:
        descs = [model.describe_plan(i) for i in range(model.plans[0])]
        if args.plan not in descs:
            print(f"bench.py: no H psi plan '{args.plan}' for L={L}; candidates: {descs}", file=sys.stderr)
            sys.exit(2)
        best, plan_ms = descs.index(args.plan), []
        model.select_plan(best)
        log(f"bench: H psi plan {best} ({args.plan}), not tuned")
    log(f"bench: apply_H L={L}, {model.passes} passes, warmup {args.warmup}, steps {args.steps}")
    for _ in range(args.warmup):
        P.apply_H(model, psi, out)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        P.apply_H(model, psi, out)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    gbs = 32.0 * D / (ms * 1e-3) / 1e9
    traffic = measured_traffic(model.describe_plan(best)) if L == 28 else None
    rec = {
        "metric": "H·ψ GB/s (% HBM peak) at L=28",
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"apply_H, open transverse-field Ising chain g=0.5, L={L} "
                               f"(2^{L} complex128 amplitudes, seeded complex-normal state)",
                   "L": L, "passes": model.passes, "launches_per_step": model.passes,
                   "plan": best, "plan_desc": model.describe_plan(best),
                   "plan_ms": [round(t, 4) for t in plan_ms]},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic},
        # bytes actually moved (rocprofv3 counters of the same plan) per time, and a plain copy
        "hbm_measured": {"GBps": round(traffic / (ms * 1e-3) / 1e9, 1) if traffic else None,
                         "frac": round(traffic / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4) if traffic else None,
                         "copy_GBps": round(copy_gbs, 1), "copy_frac": round(copy_gbs / PEAK_HBM_GBS, 4),
                         "copy_kernel": "ed_stream_copy (one amplitude per thread, streaming stores)",
                         "torch_copy_GBps": round(torch_copy_gbs, 1)},
        "host": host_info(),
        "wall_s": round(wall, 3),
    }
    del psi, out
    torch.cuda.empty_cache()
    rows = {"lanczos14": row_lanczos_L14, "lanczos26": row_lanczos_entropy_L26, "quench28": row_quench_L28,
            "traj": row_trajectories, "adjoint": row_adjoint, "traj16": row_trajectories_L16,
            "trotter28": row_trotter_L28, "lrqi28": row_lrqi_L28, "rdm28": row_rdm_L28, "liouville14": row_liouville_L14,
            "hpsi_sweep": row_hpsi_sweep}
    default_rows = ["hpsi_sweep", "lanczos14", "lanczos26", "quench28", "trotter28", "lrqi28", "rdm28", "liouville14", "traj",
                    "adjoint"]
    pick = default_rows if args.rows == "all" else ([] if args.rows == "none" else args.rows.split(","))
    rec["rows"] = {}
    for name in pick:
        log(f"bench: row {name}")
        try:
            rec["rows"][name] = rows[name](P, E, torch, dev)
        except Exception as e:  # a failing row is reported, not hidden
            rec["rows"][name] = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("bench: cpu baseline")
        rec["cpu_baseline"] = cpu_baseline()
        if args.rows != "none":
            log("bench: oracle rows")
            try:
                rec["oracle_rows"] = oracle_rows(P, E, torch, dev, traj_oracle)
            except Exception as e:  # reported, not hidden
                rec["oracle_rows"] = {"error": f"{type(e).__name__}: {e}"}
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
