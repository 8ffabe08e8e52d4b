"""MI355X-native exact-diagonalisation hot path (Jaschke & Carr, arXiv:1802.10052).

Python face of libed.so: device memory and streams come from torch; the product H psi and all
the methods built on it run in the library's HIP kernels. Names follow the C ABI (include/ed.h).
"""
import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import EdError, call, lib

__all__ = ["Model", "apply_H", "lanczos_ground", "krylov_evolve", "measure", "entropy", "Liouville", "superket", "liouville_measure", "rdm", "rdm_plan", "rdm_plan_sites", "trace_distances", "eps_local", "eps_corr", "trajectories", "philox_words", "evolve_adjoint", "evolve_loss", "AdjointEvolve", "EdError", "lib"]


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def _check_state(t, D, name="psi"):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if t.numel() != D or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with {D} elements")


class Model:
    """Handle on an immutable rule-set Hamiltonian (site, bond and diagonal InfiniteFunc rules).

    desc: any object with L, site_ops (n,2,2), site_coef (n,L), bond_ops (m,4,4),
    bond_coef (m,L-1) and optionally inf_ops / inf_ops2 (r,2,2), inf_coef (r,L), inf_f (r,L-1)
    (e.g. edinputs.ModelDesc). The handle lives on the current device.
    """

    def __init__(self, desc):
        self.L = int(desc.L)
        L = self.L
        io = getattr(desc, "inf_ops", None)
        ni = 0 if io is None else len(np.asarray(io).reshape(-1, 2, 2))
        self._keep = [np.ascontiguousarray(desc.site_ops, np.complex128),
                      np.ascontiguousarray(desc.site_coef, np.float64),
                      np.ascontiguousarray(desc.bond_ops, np.complex128),
                      np.ascontiguousarray(desc.bond_coef, np.float64),
                      np.ascontiguousarray(np.asarray(io if ni else np.zeros((0, 2, 2))).reshape(-1, 2, 2), np.complex128),
                      np.ascontiguousarray(np.asarray(desc.inf_ops2 if ni else np.zeros((0, 2, 2))).reshape(-1, 2, 2),
                                           np.complex128),
                      np.ascontiguousarray(np.asarray(desc.inf_coef if ni else np.zeros((0, L))).reshape(ni, L),
                                           np.float64),
                      np.ascontiguousarray(np.asarray(desc.inf_f if ni else np.zeros((0, L - 1))).reshape(ni, L - 1),
                                           np.float64)]
        so, sc, bo, bc, i1, i2, ic, fr = self._keep
        d = _lib.ModelDescC(self.L, 2, len(so), so.ctypes.data, sc.ctypes.data,
                            len(bo), bo.ctypes.data, bc.ctypes.data,
                            ni, i1.ctypes.data, i2.ctypes.data, ic.ctypes.data, fr.ctypes.data)
        h = C.c_void_p()
        call("ed_model_create", C.byref(d), C.byref(h))
        self._h = h
        self.D = 1 << self.L

    @property
    def handle(self):
        return self._h

    @property
    def passes(self):
        n = C.c_int()
        call("ed_model_passes", self._h, C.byref(n))
        return n.value

    @property
    def plans(self):
        """(number of candidate H psi pass plans, selected index)."""
        n, sel = C.c_int(), C.c_int()
        call("ed_model_plans", self._h, C.byref(n), C.byref(sel))
        return n.value, sel.value

    def select_plan(self, index):
        call("ed_model_select_plan", self._h, int(index))

    def describe_plan(self, index=None):
        """One-line description of candidate plan `index` (default: the selected one)."""
        if index is None:
            index = self.plans[1]
        buf = C.create_string_buffer(256)
        call("ed_model_plan_describe", self._h, int(index), buf, 256)
        return buf.value.decode()

    @property
    def plan_key(self):
        """The model's key in the tuned-plan cache (ed_model_plan_key)."""
        buf = C.create_string_buffer(512)
        call("ed_model_plan_key", self._h, buf, 512)
        return buf.value.decode()

    def tune(self, psi, out=None, reps=3, stream=None):
        """Time every candidate H psi plan on psi (ed_model_tune) and keep the fastest.
        Returns (best index, list of ms per product)."""
        _check_state(psi, self.D)
        if out is None:
            out = torch.empty_like(psi)
        n = self.plans[0]
        times = (C.c_float * max(n, 1))()
        best = C.c_int()
        call("ed_model_tune", self._h, _dptr(psi), _dptr(out), int(reps), _stream_ptr(stream), C.byref(best), times)
        return best.value, [times[i] for i in range(n)]

    def close(self):
        if getattr(self, "_h", None):
            lib().ed_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Liouville(Model):
    """Handle on the Liouvillian of a Lindblad equation (ed_liouville_create): a model of 2L bits
    whose apply_H gives i Lcal |rho>> for the row-major superket |rho>> (entry j 2^L + k = rho_jk),
    and whose krylov_evolve (Arnoldi) propagates exp(dt Lcal). desc: the Hermitian H on L sites;
    jump_ops: list of 2x2 operators J_z; rates: [n_jump, L] array of gamma (L_nu = sqrt(gamma) J on
    site k). `sites` is L; `L` is the superket's bit count 2L."""

    def __init__(self, desc, jump_ops, rates):
        self.sites = int(desc.L)
        Ls = self.sites
        self._keep = [np.ascontiguousarray(desc.site_ops, np.complex128),
                      np.ascontiguousarray(desc.site_coef, np.float64),
                      np.ascontiguousarray(desc.bond_ops, np.complex128),
                      np.ascontiguousarray(desc.bond_coef, np.float64),
                      np.ascontiguousarray(np.asarray(jump_ops, np.complex128).reshape(-1, 2, 2)),
                      np.ascontiguousarray(np.asarray(rates, np.float64).reshape(-1, Ls))]
        so, sc, bo, bc, jo, rt = self._keep
        if len(jo) != len(rt):
            raise ValueError("one rate row per jump operator")
        d = _lib.ModelDescC(Ls, 2, len(so), so.ctypes.data, sc.ctypes.data, len(bo), bo.ctypes.data, bc.ctypes.data,
                            0, None, None, None, None)
        h = C.c_void_p()
        call("ed_liouville_create", C.byref(d), len(jo), jo.ctypes.data if len(jo) else None,
             rt.ctypes.data if len(jo) else None, C.byref(h))
        self._h = h
        self.L = 2 * Ls
        self.D = 1 << self.L


def superket(rho):
    """|rho>> of a [D, D] density matrix (tensor or array): the row-major flattening."""
    if not hasattr(rho, "reshape"):
        rho = np.asarray(rho)
    return rho.reshape(-1)


def liouville_measure(rho, L, stream=None):
    """(sz[L] = tr(sigma^z_k rho)/tr(rho), tr(rho)) of a device superket (ed_liouville_measure)."""
    _check_state(rho, 1 << (2 * L), "rho")
    nb = C.c_size_t()
    call("ed_measure_workspace", int(L), C.byref(nb))
    ws = _workspace(nb.value, rho.device)
    sz = np.zeros(L)
    tr = C.c_double()
    call("ed_liouville_measure", _dptr(rho), int(L), sz.ctypes.data, C.byref(tr), _dptr(ws), nb.value,
         _stream_ptr(stream))
    return sz, tr.value


def apply_H(model, psi, out=None, stream=None):
    """out = H psi (asynchronous on the current torch stream)."""
    _check_state(psi, model.D)
    if out is None:
        out = torch.empty_like(psi)
    _check_state(out, model.D, "out")
    call("ed_apply_H", model.handle, _dptr(psi), _dptr(out), _stream_ptr(stream))
    return out


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def plan_cache_load(path):
    """Merge a tuned-plan file into the process's plan cache; returns the number of entries."""
    n = C.c_int()
    call("ed_plan_cache_load", str(path).encode(), C.byref(n))
    return n.value


def plan_cache_save(path):
    call("ed_plan_cache_save", str(path).encode())


def plan_cache_get(key):
    """The cached plan description for key, or None."""
    buf = C.create_string_buffer(512)
    code = lib().ed_plan_cache_get(key.encode(), buf, 512)
    return buf.value.decode() if code == 0 else None


def plan_cache_put(key, plan):
    call("ed_plan_cache_put", key.encode(), plan.encode())


def plan_cache_clear():
    call("ed_plan_cache_clear")


REORTH = {"full": 0, "partial": 1}


def lanczos_ground(model, v0, tol=1e-10, max_iter=200, max_basis=None, n_keep=0, reorth="full", stream=None):
    """Lowest eigenpair (E0, psi0, info) of a Hermitian model by matrix-free Lanczos with thick
    restart (ed_lanczos_ground); reorth "full" (classical Gram-Schmidt twice against the whole basis
    every step) or "partial" (three-term recurrence, the kept Ritz vectors every step, the rest when
    the orthogonality estimates ask for it). info is a dict."""
    _check_state(v0, model.D, "v0")
    mb = max_iter + 1 if max_basis is None else max_basis
    mb = max(2, min(mb, 512))
    p = _lib.LanczosParams(int(max_iter), int(mb), int(n_keep), float(tol), REORTH[reorth])
    nb = C.c_size_t()
    call("ed_lanczos_workspace", model.handle, C.byref(p), C.byref(nb))
    ws = _workspace(nb.value, v0.device)
    psi0 = torch.empty_like(v0)
    e0 = C.c_double()
    info = _lib.LanczosInfo()
    code = lib().ed_lanczos_ground(model.handle, _dptr(v0), C.byref(p), C.byref(e0), _dptr(psi0),
                                   C.byref(info), _dptr(ws), nb.value, _stream_ptr(stream))
    d = {"iters": info.iters, "restarts": info.restarts, "residual": info.residual,
         "converged": bool(info.converged), "extra_reorth": info.extra_reorth,
         "device_resident": bool(info.device_resident), "status": _lib.STATUS.get(code, code)}
    if code not in (0, -7):
        _lib.check("ed_lanczos_ground", code)
    return e0.value, psi0, d


def _observe(shapes, device):
    """Output arrays of an evolve call: numpy arrays, or with device set float64 tensors there
    (ed_observe.on_device = 1). Returns (dict, Observe)."""
    if device is None:
        obs = {k: np.zeros(v) for k, v in shapes.items()}
        ptr = {k: a.ctypes.data for k, a in obs.items()}
    else:
        obs = {k: torch.zeros(v, dtype=torch.float64, device=device) for k, v in shapes.items()}
        ptr = {k: a.data_ptr() for k, a in obs.items()}
    o = _lib.Observe(ptr.get("sz"), ptr.get("energy"), ptr.get("norm"), 0 if device is None else 1)
    return obs, o


def krylov_evolve(model, psi, dt, n_steps, m_max=20, tol=1e-10, fixed_m=0, reorth=0, hermitian=True,
                  observe=True, stream=None, device_obs=False):
    """Krylov time evolution of psi in place (ed_krylov_evolve). Returns (psi, obs, info) with obs
    holding numpy arrays sz [(n_steps+1), L], energy [n_steps+1], norm [n_steps+1] (with
    device_obs=True, float64 tensors on psi's device, written through device pointers). For a
    Liouville model (hermitian=False): sz [(n_steps+1), sites] of rho, norm = tr(rho), no energy."""
    odev = psi.device if device_obs else None
    _check_state(psi, model.D)
    if isinstance(model, Liouville):
        p = _lib.KrylovParams(int(m_max), float(tol), int(fixed_m), 1, 0)
        if hermitian:
            raise ValueError("a Liouville model evolves with hermitian=False (Arnoldi)")
        nb = C.c_size_t()
        call("ed_krylov_workspace", model.handle, C.byref(p), C.byref(nb))
        ws = _workspace(nb.value, psi.device)
        obs, o = None, None
        if observe:
            obs, o = _observe({"sz": (n_steps + 1, model.sites), "norm": (n_steps + 1,)}, odev)
        info = _lib.KrylovInfo()
        call("ed_krylov_evolve", model.handle, _dptr(psi), float(dt), int(n_steps), C.byref(p),
             C.byref(o) if o is not None else None, C.byref(info), _dptr(ws), nb.value, _stream_ptr(stream))
        return psi, obs, {"steps": info.steps, "total_m": info.total_m, "max_m": info.max_m, "max_err": info.max_err,
                          "reorth_skipped": info.reorth_skipped}
    p = _lib.KrylovParams(int(m_max), float(tol), int(fixed_m), int(reorth if hermitian else 1), int(bool(hermitian)))
    nb = C.c_size_t()
    call("ed_krylov_workspace", model.handle, C.byref(p), C.byref(nb))
    ws = _workspace(nb.value, psi.device)
    obs = None
    o = None
    if observe:
        obs, o = _observe({"sz": (n_steps + 1, model.L), "energy": (n_steps + 1,), "norm": (n_steps + 1,)}, odev)
    info = _lib.KrylovInfo()
    call("ed_krylov_evolve", model.handle, _dptr(psi), float(dt), int(n_steps), C.byref(p),
         C.byref(o) if o is not None else None, C.byref(info), _dptr(ws), nb.value, _stream_ptr(stream))
    return psi, obs, {"steps": info.steps, "total_m": info.total_m, "max_m": info.max_m, "max_err": info.max_err,
                      "reorth_skipped": info.reorth_skipped}


def trotter_evolve(model, psi, dt, n_steps, order=4, observe=True, energy=False, stream=None, device_obs=False):
    """Suzuki-Trotter time evolution of psi in place (ed_trotter_evolve, order 2 or 4). Returns
    (psi, obs) with obs holding numpy arrays sz [(n_steps+1), L], norm [n_steps+1] and, with
    energy=True, energy [n_steps+1] (with device_obs=True, float64 tensors on psi's device)."""
    _check_state(psi, model.D)
    nb = C.c_size_t()
    call("ed_trotter_workspace", model.handle, int(bool(energy)), C.byref(nb))
    ws = _workspace(nb.value, psi.device)
    obs = None
    o = None
    if observe or energy:
        shapes = {"sz": (n_steps + 1, model.L), "norm": (n_steps + 1,)}
        if energy:
            shapes["energy"] = (n_steps + 1,)
        obs, o = _observe(shapes, psi.device if device_obs else None)
    call("ed_trotter_evolve", model.handle, _dptr(psi), float(dt), int(n_steps), int(order),
         C.byref(o) if o is not None else None, _dptr(ws), nb.value, _stream_ptr(stream))
    return psi, obs


def trotter_passes(model, order=4):
    """In-place passes over the state per Trotter step of the given order (ed_trotter_passes)."""
    n = C.c_int()
    call("ed_trotter_passes", model.handle, int(order), C.byref(n))
    return n.value


def measure(psi, L, stream=None):
    """(sz[L], norm) of a device state in one pass (ed_measure)."""
    _check_state(psi, 1 << L)
    nb = C.c_size_t()
    call("ed_measure_workspace", int(L), C.byref(nb))
    ws = _workspace(nb.value, psi.device)
    sz = np.zeros(L)
    nrm = C.c_double()
    call("ed_measure", _dptr(psi), int(L), sz.ctypes.data, C.byref(nrm), _dptr(ws), nb.value, _stream_ptr(stream))
    return sz, nrm.value


def stream_copy(src, dst, stream=None):
    """dst = src for two device complex128 tensors of equal size (ed_stream_copy)."""
    if src.numel() != dst.numel():
        raise ValueError("src and dst differ in size")
    call("ed_stream_copy", _dptr(src), _dptr(dst), int(src.numel()), _stream_ptr(stream))


def measure_noalloc(psi, L, stream=None):
    """(sz[L], norm) of a device state (ed_measure_noalloc: no workspace, nothing allocated)."""
    _check_state(psi, 1 << L)
    sz = np.zeros(L)
    nrm = C.c_double()
    call("ed_measure_noalloc", _dptr(psi), int(L), sz.ctypes.data, C.byref(nrm), _stream_ptr(stream))
    return sz, nrm.value


def entropy(psi, L, l_cut=None, spectrum=False, stream=None, info=False):
    """Bond entropy S(l_cut) (natural log) of a device state (ed_entropy); with spectrum=True
    also the Schmidt spectrum (descending numpy array); with info=True also a dict whose
    "real_arith" tells whether the state was real and the reduction ran in real arithmetic."""
    _check_state(psi, 1 << L)
    l = L // 2 if l_cut is None else int(l_cut)
    nb = C.c_size_t()
    call("ed_entropy_workspace", int(L), l, C.byref(nb))
    ws = _workspace(nb.value, psi.device)
    S = C.c_double()
    real = C.c_int(0)
    spec = np.zeros(1 << min(l, L - l)) if spectrum else None
    if info:
        call("ed_entropy_ex", _dptr(psi), int(L), 2, l, C.byref(S), spec.ctypes.data if spectrum else None,
             C.byref(real), _dptr(ws), nb.value, _stream_ptr(stream))
    else:
        call("ed_entropy", _dptr(psi), int(L), 2, l, C.byref(S), spec.ctypes.data if spectrum else None,
             _dptr(ws), nb.value, _stream_ptr(stream))
    out = (S.value, spec) if spectrum else (S.value,)
    if info:
        out = out + ({"real_arith": bool(real.value)},)
    return out if len(out) > 1 else out[0]


def rdm(psi, L, two_site=True, stream=None):
    """Reduced density matrices of a device state (ed_rdm): rho1 [L, 2, 2] (rho_k, k = 1..L) and,
    with two_site, rho2 [L(L-1)/2, 4, 4] (rho_{k,j} for all pairs k < j, lexicographic), both
    complex128 device tensors, not normalised (trace <psi|psi>). Asynchronous on the stream."""
    import torch
    _check_state(psi, 1 << L)
    nb = C.c_size_t()
    call("ed_rdm_workspace", int(L), C.byref(nb))
    ws = _workspace(nb.value, psi.device)
    rho1 = torch.empty((L, 2, 2), dtype=torch.complex128, device=psi.device)
    rho2 = torch.empty((L * (L - 1) // 2, 4, 4), dtype=torch.complex128, device=psi.device) if two_site else None
    call("ed_rdm", _dptr(psi), int(L), _dptr(rho1), _dptr(rho2) if two_site else None, _dptr(ws), nb.value,
         _stream_ptr(stream))
    return rho1, rho2


def rdm_plan(L):
    """The pairs of index bits ed_rdm evaluates for the two-site matrices, as (pairs [n, 2],
    pass index [n]) numpy arrays."""
    n = lib().ed_rdm_plan_pairs(int(L), None, 0, None)
    if n < 0:
        raise EdError("ed_rdm_plan_pairs", "ED_ERR_ARG", f"L={L}")
    pairs = np.zeros((n, 2), np.int32)
    pass_of = np.zeros(n, np.int32)
    lib().ed_rdm_plan_pairs(int(L), pairs.ctypes.data, n, pass_of.ctypes.data)
    return pairs, pass_of


def rdm_plan_sites(L):
    """The index bits ed_rdm evaluates for the single-site matrices alone, as (bits [L],
    pass index [L]) numpy arrays (bit b is site L - b)."""
    n = lib().ed_rdm_plan_sites(int(L), None, 0, None)
    if n < 0:
        raise EdError("ed_rdm_plan_sites", "ED_ERR_ARG", f"L={L}")
    bits = np.zeros(n, np.int32)
    pass_of = np.zeros(n, np.int32)
    lib().ed_rdm_plan_sites(int(L), bits.ctypes.data, n, pass_of.ctypes.data)
    return bits, pass_of


def trace_distances(a, b):
    """D = 1/2 Tr|a_m - b_m| for stacks of Hermitian n x n matrices (ed_trace_distances, host).
    a, b: arrays or tensors of shape [count, n, n] (or [n, n]); returns a numpy array [count]."""
    def host(x):
        if hasattr(x, "detach"):
            x = x.detach().cpu().numpy()
        return np.ascontiguousarray(np.asarray(x, np.complex128))
    A, B = host(a), host(b)
    if A.ndim == 2:
        A, B = A[None], B[None]
    if A.shape != B.shape or A.ndim != 3 or A.shape[1] != A.shape[2]:
        raise ValueError(f"shapes {A.shape} and {B.shape} are not two equal stacks of square matrices")
    out = np.zeros(A.shape[0])
    call("ed_trace_distances", int(A.shape[1]), int(A.shape[0]), A.ctypes.data, B.ctypes.data, out.ctypes.data)
    return out


def eps_local(rho1, rho1_ref):
    """The largest single-site trace distance (the error measure eps_local of the convergence study)."""
    return float(trace_distances(rho1, rho1_ref).max())


def eps_corr(rho2, rho2_ref):
    """The largest two-site trace distance over all pairs (eps_corr)."""
    return float(trace_distances(rho2, rho2_ref).max())


_TRAJ_STREAMS = {}


def _traj_stream(dev):
    """One stream per device for the batched trajectories, so that consecutive calls replay the
    stream's executable graph."""
    key = torch.device(dev)
    if key not in _TRAJ_STREAMS:
        _TRAJ_STREAMS[key] = torch.cuda.Stream(device=key)
    return _TRAJ_STREAMS[key]


def trajectories(models, jump_op, rates, psi0, model_of_traj, dt, n_steps, out_stride, seed,
                 m_max=20, tol=1e-10, max_jumps=64, plain=False, stream=None):
    """Quantum trajectories (ed_trajectories_batch, or ed_trajectories_plain with plain=True).

    models: list of Model (Hermitian parts, one per chain length); jump_op: 2x2 complex;
    rates: list of per-site rate arrays; psi0: list of complex128 device states;
    model_of_traj: int array. Returns dict with sz [n_traj, n_out, L_max], n_jumps, jump_t,
    jump_site and info. Runs on a dedicated non-default stream (so the batched launch is replayed
    from a hipGraph) and synchronises it."""
    nm = len(models)
    mh = (C.c_void_p * nm)(*[m.handle.value for m in models])
    J = np.ascontiguousarray(np.asarray(jump_op, np.complex128).reshape(2, 2))
    rk = [np.ascontiguousarray(r, np.float64) for r in rates]
    rp = (C.c_void_p * nm)(*[r.ctypes.data for r in rk])
    for i, p0 in enumerate(psi0):
        _check_state(p0, models[i].D, "psi0")
    pp = (C.c_void_p * nm)(*[p0.data_ptr() for p0 in psi0])
    mo = np.ascontiguousarray(model_of_traj, np.int32)
    nt = len(mo)
    d = _lib.TrajDesc(nm, C.cast(mh, C.POINTER(C.c_void_p)), J.ctypes.data, C.cast(rp, C.POINTER(C.c_void_p)),
                      C.cast(pp, C.POINTER(C.c_void_p)), nt, mo.ctypes.data, float(dt), int(n_steps),
                      int(out_stride), int(seed))
    p = _lib.TrajParams(int(m_max), float(tol), int(max_jumps))
    nb = C.c_size_t()
    name = "ed_trajectories_plain" if plain else "ed_trajectories_batch"
    call(name.replace("_plain", "_plain_workspace") if plain else "ed_trajectories_workspace",
         C.byref(d), C.byref(p), C.byref(nb))
    dev = psi0[0].device
    ws = _workspace(nb.value, dev)
    Lmax = max(m.L for m in models)
    n_out = n_steps // out_stride + 1
    sz = np.zeros((nt, n_out, Lmax))
    nj = np.zeros(nt, np.int32)
    mj = max(int(max_jumps), 1)
    jt = np.zeros((nt, mj))
    js = np.zeros((nt, mj), np.int32)
    o = _lib.TrajOut(sz.ctypes.data, nj.ctypes.data, jt.ctypes.data, js.ctypes.data)
    info = _lib.TrajInfo()
    st = stream if stream is not None else _traj_stream(dev)
    st.wait_stream(torch.cuda.current_stream(dev))
    call(name, C.byref(d), C.byref(p), C.byref(o), C.byref(info), _dptr(ws), nb.value, _stream_ptr(st))
    return {"sz": sz, "n_jumps": nj, "jump_t": jt, "jump_site": js,
            "info": {"total_jumps": info.total_jumps, "total_krylov": info.total_krylov, "blocks": info.blocks,
                     "unconverged_steps": info.unconverged_steps, "graph_replayed": bool(info.graph_replayed),
                     "busy_ms": {"max": info.busy_max_ms, "min": info.busy_min_ms, "mean": info.busy_mean_ms}}}


def philox_words(seed, ident, count, device="cuda:0", stream=None):
    """Raw 64-bit words 0..count-1 of the trajectory random stream of key (seed, ident)."""
    out = torch.empty(int(count), dtype=torch.int64, device=device)
    call("ed_philox_words", int(seed), int(ident), _dptr(out), int(count), _stream_ptr(stream))
    torch.cuda.synchronize(device)
    return out.cpu().numpy().view(np.uint64)


def _adj_params(substeps, quad_nodes, m_max, m_fixed, tol):
    return _lib.AdjointParams(int(substeps), int(quad_nodes), int(m_max), int(m_fixed), float(tol))


def evolve_adjoint(template, J, psi0, slice_len, obs_w, substeps=2, quad_nodes=8, m_max=30, m_fixed=0, tol=1e-13,
                   stream=None):
    """(loss, grad) of <psi_S|sum_k w_k sz_k|psi_S> w.r.t. the sliced bond couplings J [S, L-1]
    (ed_evolve_adjoint)."""
    J = np.ascontiguousarray(J, np.float64)
    S = J.shape[0]
    w = np.ascontiguousarray(obs_w, np.float64)
    _check_state(psi0, template.D, "psi0")
    p = _adj_params(substeps, quad_nodes, m_max, m_fixed, tol)
    nb = C.c_size_t()
    call("ed_adjoint_workspace", template.handle, S, C.byref(p), C.byref(nb))
    ws = _workspace(nb.value, psi0.device)
    loss = C.c_double()
    grad = np.zeros_like(J)
    call("ed_evolve_adjoint", template.handle, S, float(slice_len), J.ctypes.data, _dptr(psi0), w.ctypes.data,
         C.byref(p), C.byref(loss), grad.ctypes.data, _dptr(ws), nb.value, _stream_ptr(stream))
    return loss.value, grad


def evolve_loss(template, J, psi0, slice_len, obs_w, substeps=2, m_max=30, m_fixed=0, tol=1e-13, ws=None,
                stream=None):
    """Forward-only loss with the same discretisation (ed_evolve_loss)."""
    J = np.ascontiguousarray(J, np.float64)
    w = np.ascontiguousarray(obs_w, np.float64)
    p = _adj_params(substeps, 1, m_max, m_fixed, tol)
    nb = C.c_size_t()
    call("ed_evolve_loss_workspace", template.handle, C.byref(p), C.byref(nb))
    if ws is None or ws.numel() < nb.value:
        ws = _workspace(nb.value, psi0.device)
    loss = C.c_double()
    call("ed_evolve_loss", template.handle, J.shape[0], float(slice_len), J.ctypes.data, _dptr(psi0), w.ctypes.data,
         C.byref(p), C.byref(loss), _dptr(ws), nb.value, _stream_ptr(stream))
    return loss.value


class AdjointEvolve(torch.autograd.Function):
    """Loss(J) = <psi_S|O|psi_S> as a differentiable function of the couplings J [S, L-1]
    (float64 CPU tensor). forward runs the forward propagation only (ed_evolve_loss); backward runs
    ed_evolve_adjoint (forward with slice-boundary checkpoints, then the costate sweep) and returns
    grad_out * dLoss/dJ, so a caller that needs only the loss never pays for the gradient."""

    @staticmethod
    def forward(ctx, J, template, psi0, slice_len, obs_w, substeps=2, quad_nodes=8, m_max=30, m_fixed=0, tol=1e-13):
        Jn = J.detach().cpu().numpy()
        loss = evolve_loss(template, Jn, psi0, slice_len, obs_w, substeps, m_max, m_fixed, tol)
        ctx.save_for_backward(J.detach().cpu())
        ctx.args = (template, psi0, slice_len, obs_w, substeps, quad_nodes, m_max, m_fixed, tol)
        return torch.tensor(loss, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        (J,) = ctx.saved_tensors
        template, psi0, slice_len, obs_w, substeps, quad_nodes, m_max, m_fixed, tol = ctx.args
        _, grad = evolve_adjoint(template, J.numpy(), psi0, slice_len, obs_w, substeps, quad_nodes, m_max, m_fixed,
                                 tol)
        return (grad_out * torch.from_numpy(grad), None, None, None, None, None, None, None, None, None)
