"""ctypes view of libed.so (the C ABI declared in include/ed.h).

Argument marshalling only: every step of the hot path runs in the library's HIP kernels. The
library must be built (paper_1802_10052_amd/build.py); importing without it fails loudly.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# ED_LIB names another build of the library (the sanitized one, for the host boundary tests)
LIB_PATH = os.environ.get("ED_LIB") or os.path.join(HERE, "libed.so")


class EdError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


class c64(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class ModelDescC(C.Structure):
    _fields_ = [("L", C.c_int), ("d", C.c_int),
                ("n_site", C.c_int), ("site_op", C.c_void_p), ("site_coef", C.c_void_p),
                ("n_bond", C.c_int), ("bond_op", C.c_void_p), ("bond_coef", C.c_void_p),
                ("n_inf", C.c_int), ("inf_op", C.c_void_p), ("inf_op2", C.c_void_p), ("inf_coef", C.c_void_p),
                ("inf_f", C.c_void_p)]


class LanczosParams(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("max_basis", C.c_int), ("n_keep", C.c_int), ("tol", C.c_double),
                ("reorth", C.c_int)]


class LanczosInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("residual", C.c_double), ("converged", C.c_int),
                ("extra_reorth", C.c_int), ("device_resident", C.c_int)]


class KrylovParams(C.Structure):
    _fields_ = [("m_max", C.c_int), ("tol", C.c_double), ("fixed_m", C.c_int), ("reorth", C.c_int),
                ("hermitian", C.c_int)]


class Observe(C.Structure):
    _fields_ = [("sz", C.c_void_p), ("energy", C.c_void_p), ("norm", C.c_void_p), ("on_device", C.c_int)]


class KrylovInfo(C.Structure):
    _fields_ = [("steps", C.c_int), ("total_m", C.c_int), ("max_m", C.c_int), ("max_err", C.c_double),
                ("reorth_skipped", C.c_int)]


class TrajDesc(C.Structure):
    _fields_ = [("n_models", C.c_int), ("models", C.POINTER(C.c_void_p)), ("jump_op", C.c_void_p),
                ("rates", C.POINTER(C.c_void_p)), ("psi0", C.POINTER(C.c_void_p)), ("n_traj", C.c_int),
                ("model_of_traj", C.c_void_p), ("dt", C.c_double), ("n_steps", C.c_int),
                ("out_stride", C.c_int), ("seed", C.c_uint64)]


class TrajParams(C.Structure):
    _fields_ = [("m_max", C.c_int), ("tol", C.c_double), ("max_jumps", C.c_int)]


class TrajOut(C.Structure):
    _fields_ = [("sz", C.c_void_p), ("n_jumps", C.c_void_p), ("jump_t", C.c_void_p), ("jump_site", C.c_void_p)]


class TrajInfo(C.Structure):
    _fields_ = [("total_jumps", C.c_longlong), ("total_krylov", C.c_longlong), ("blocks", C.c_int),
                ("unconverged_steps", C.c_longlong), ("graph_replayed", C.c_int), ("busy_max_ms", C.c_double),
                ("busy_min_ms", C.c_double), ("busy_mean_ms", C.c_double)]


class AdjointParams(C.Structure):
    _fields_ = [("substeps", C.c_int), ("quad_nodes", C.c_int), ("m_max", C.c_int), ("m_fixed", C.c_int),
                ("tol", C.c_double)]


ED_OK = 0
STATUS = {0: "ED_OK", -1: "ED_ERR_ARG", -2: "ED_ERR_UNSUPPORTED", -3: "ED_ERR_NODEVICE",
          -4: "ED_ERR_NOMEM", -5: "ED_ERR_WORKSPACE", -6: "ED_ERR_HIP", -7: "ED_ERR_NOCONV",
          -8: "ED_ERR_NUMERIC"}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libed.so is not built ({LIB_PATH}); run paper_1802_10052_amd/build.py")
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
        _load_default_plans(_lib)
    return _lib


# Tuned H psi plans shipped with the package (written by tune_plans.py on the target GPU); the
# environment variable ED_PLAN_CACHE names another file, or "none" to start with an empty cache.
DEFAULT_PLANS = os.path.join(HERE, "plan_cache.tsv")


def _load_default_plans(l):
    path = os.environ.get("ED_PLAN_CACHE", DEFAULT_PLANS)
    if path and path != "none" and os.path.exists(path):
        n = C.c_int()
        code = l.ed_plan_cache_load(path.encode(), C.byref(n))
        if code != 0:
            raise RuntimeError(f"plan cache {path}: {l.ed_last_error().decode(errors='replace')}")


def _fn(l, name, argtypes, restype=C.c_int):
    f = getattr(l, name)
    f.argtypes = argtypes
    f.restype = restype
    return f


def _declare(l):
    P = C.c_void_p
    _fn(l, "ed_last_error", [], C.c_char_p)
    _fn(l, "ed_version", [], C.c_char_p)
    _fn(l, "ed_model_create", [C.POINTER(ModelDescC), C.POINTER(P)])
    _fn(l, "ed_model_destroy", [P])
    _fn(l, "ed_model_dims", [P, C.POINTER(C.c_int), C.POINTER(C.c_int64)])
    _fn(l, "ed_model_passes", [P, C.POINTER(C.c_int)])
    _fn(l, "ed_apply_H", [P, P, P, P])
    _fn(l, "ed_model_plans", [P, C.POINTER(C.c_int), C.POINTER(C.c_int)])
    _fn(l, "ed_model_select_plan", [P, C.c_int])
    _fn(l, "ed_model_plan_describe", [P, C.c_int, C.c_char_p, C.c_int])
    _fn(l, "ed_model_tune", [P, P, P, C.c_int, P, C.POINTER(C.c_int), C.POINTER(C.c_float)])
    S = C.POINTER(C.c_size_t)
    _fn(l, "ed_lanczos_workspace", [P, C.POINTER(LanczosParams), S])
    _fn(l, "ed_lanczos_ground", [P, P, C.POINTER(LanczosParams), C.POINTER(C.c_double), P,
                                 C.POINTER(LanczosInfo), P, C.c_size_t, P])
    _fn(l, "ed_krylov_workspace", [P, C.POINTER(KrylovParams), S])
    _fn(l, "ed_krylov_evolve", [P, P, C.c_double, C.c_int, C.POINTER(KrylovParams), C.POINTER(Observe),
                                C.POINTER(KrylovInfo), P, C.c_size_t, P])
    _fn(l, "ed_trotter_workspace", [P, C.c_int, S])
    _fn(l, "ed_trotter_evolve", [P, P, C.c_double, C.c_int, C.c_int, C.POINTER(Observe), P, C.c_size_t, P])
    _fn(l, "ed_trotter_passes", [P, C.c_int, C.POINTER(C.c_int)])
    _fn(l, "ed_measure_workspace", [C.c_int, S])
    _fn(l, "ed_entropy_workspace", [C.c_int, C.c_int, S])
    TD, TP, TO, TI = C.POINTER(TrajDesc), C.POINTER(TrajParams), C.POINTER(TrajOut), C.POINTER(TrajInfo)
    _fn(l, "ed_trajectories_workspace", [TD, TP, S])
    _fn(l, "ed_trajectories_batch", [TD, TP, TO, TI, P, C.c_size_t, P])
    _fn(l, "ed_trajectories_plain_workspace", [TD, TP, S])
    _fn(l, "ed_trajectories_plain", [TD, TP, TO, TI, P, C.c_size_t, P])
    _fn(l, "ed_philox_words", [C.c_uint64, C.c_uint64, P, C.c_int64, P])
    AP = C.POINTER(AdjointParams)
    _fn(l, "ed_adjoint_workspace", [P, C.c_int, AP, S])
    _fn(l, "ed_evolve_adjoint", [P, C.c_int, C.c_double, P, P, P, AP, C.POINTER(C.c_double), P, P, C.c_size_t, P])
    _fn(l, "ed_evolve_loss_workspace", [P, AP, S])
    _fn(l, "ed_evolve_loss", [P, C.c_int, C.c_double, P, P, P, AP, C.POINTER(C.c_double), P, C.c_size_t, P])
    _fn(l, "ed_entropy", [P, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double), P, P, C.c_size_t, P])
    _fn(l, "ed_entropy_ex", [P, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double), P, C.POINTER(C.c_int), P,
                             C.c_size_t, P])
    _fn(l, "ed_measure", [P, C.c_int, P, P, P, C.c_size_t, P])
    _fn(l, "ed_measure_noalloc", [P, C.c_int, P, P, P])
    _fn(l, "ed_stream_copy", [P, P, C.c_int64, P])
    _fn(l, "ed_model_plan_key", [P, C.c_char_p, C.c_int])
    _fn(l, "ed_plan_cache_load", [C.c_char_p, C.POINTER(C.c_int)])
    _fn(l, "ed_plan_cache_save", [C.c_char_p])
    _fn(l, "ed_plan_cache_get", [C.c_char_p, C.c_char_p, C.c_int])
    _fn(l, "ed_plan_cache_put", [C.c_char_p, C.c_char_p])
    _fn(l, "ed_plan_cache_clear", [])
    _fn(l, "ed_liouville_create", [C.POINTER(ModelDescC), C.c_int, P, P, C.POINTER(P)])
    _fn(l, "ed_model_liouville_sites", [P, C.POINTER(C.c_int)])
    _fn(l, "ed_liouville_measure", [P, C.c_int, P, C.POINTER(C.c_double), P, C.c_size_t, P])
    _fn(l, "ed_rdm_workspace", [C.c_int, S])
    _fn(l, "ed_rdm", [P, C.c_int, P, P, P, C.c_size_t, P])
    _fn(l, "ed_rdm_plan_pairs", [C.c_int, P, C.c_int, P])
    _fn(l, "ed_rdm_plan_sites", [C.c_int, P, C.c_int, P])
    _fn(l, "ed_trace_distances", [C.c_int, C.c_int, P, P, P])


def check(name, code):
    if code != ED_OK:
        msg = lib().ed_last_error().decode(errors="replace")
        raise EdError(name, STATUS.get(code, code), msg)


def call(name, *args):
    check(name, getattr(lib(), name)(*args))
