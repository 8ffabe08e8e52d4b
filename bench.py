"""Benchmark of the exact-diagonalisation hot path on one MI355X.

Headline: matrix-free H psi (ed_apply_H) on the L = 28 transverse-field Ising chain (g = 0.5,
complex128 state of 2^28 amplitudes, 4 GiB), reported as algorithmic GB/s = 32 B/amplitude
(read psi once, write H psi once) / kernel time, and as a fraction of the 8 TB/s HBM peak.
A step is one H psi over the whole state. Timing uses HIP events on the stream the library
launches on, after warm-up, with the state resident in HBM.
"""
import argparse
import json
import os
import platform
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


def cpu_baseline(L=20, reps=60):
    """The oracle's explicit sparse H psi (scipy CSR matvec, single-threaded) at L = 20."""
    import numpy as np
    import edinputs as E
    from oracle import hamiltonian as OH
    H = OH.hamiltonian_sparse(E.tfim(L, 0.5))
    psi = E.random_state(L, 11)
    H @ psi
    t0 = time.perf_counter()
    for _ in range(reps):
        y = H @ psi
    dt = (time.perf_counter() - t0) / reps
    return {"value": 32.0 * (1 << L) / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"scipy CSR H psi, TFIM g=0.5 L={L} (2^{L} amplitudes), {reps} products, "
                      f"{dt * 1e3:.1f} ms each; same 32 B/amplitude accounting"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=28)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is a design "
              f"note, not a measured path", file=sys.stderr)
        sys.exit(2)

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
        "config": {"workload": f"apply_H TFIM g=0.5 open chain L={L} (2^{L} complex128 amplitudes)",
                   "L": L, "passes": model.passes},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None},
        "host": host_info(),
        "wall_s": round(wall, 3),
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline()
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
