"""ctypes declarations of the C ABI in include/ipmg.h (argument marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libipmg.so")

OK = 0
E_INVALID, E_DOMAIN, E_HIP, E_NOMEM, E_BREAKDOWN, E_NOT_CONVERGED, E_STALLED, E_STATE = range(-1, -9, -1)
OP_K, OP_Z = 0, 1


class Desc(C.Structure):
    _fields_ = [("dim", C.c_int), ("nel", C.c_int * 3), ("levels", C.c_int), ("E", C.c_double),
                ("nu", C.c_double), ("vcycle_fp32", C.c_int), ("nu_pre", C.c_int), ("nu_post", C.c_int),
                ("omega", C.c_double), ("pcg_flexible", C.c_int)]


class PCGInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("status", C.c_int), ("relres", C.c_double),
                ("true_relres", C.c_double), ("setup_ms", C.c_double), ("solve_ms", C.c_double),
                ("bu", C.c_double)]


class OCInfo(C.Structure):
    _fields_ = [("lam", C.c_double), ("volume", C.c_double), ("trials", C.c_int)]


class IPState(C.Structure):
    _fields_ = [("u", C.c_void_p), ("x", C.c_void_p), ("phi", C.c_void_p), ("psi", C.c_void_p),
                ("lam", C.c_double), ("s", C.c_double), ("r", C.c_double)]


class IPParams(C.Structure):
    _fields_ = [("V", C.c_double), ("xbar", C.c_double), ("sigma", C.c_double), ("tau_nwt", C.c_double),
                ("pcg_rtol", C.c_double), ("pcg_maxit", C.c_int), ("frac", C.c_double),
                ("step_all_blocks", C.c_int), ("stop_rule", C.c_int), ("kkt_tol", C.c_double),
                ("tau_ip", C.c_double), ("max_newton", C.c_int), ("accept_rtol", C.c_double)]


class IPInfo(C.Structure):
    _fields_ = [("alpha", C.c_double), ("nwt", C.c_double), ("gap", C.c_double), ("volume_res", C.c_double),
                ("compliance", C.c_double), ("pcg_iters", C.c_int), ("pcg_status", C.c_int),
                ("barrier_updated", C.c_int), ("converged", C.c_int), ("setup_ms", C.c_double),
                ("solve_ms", C.c_double), ("pcg_true_relres", C.c_double),
                ("pcg_retries", C.c_int)]


SIGNATURES = {
    "ipmg_create": (C.c_int, [C.POINTER(Desc), C.c_void_p, C.POINTER(C.c_void_p)]),
    "ipmg_destroy": (None, [C.c_void_p]),
    "ipmg_last_error": (C.c_char_p, [C.c_void_p]),
    "ipmg_status_string": (C.c_char_p, [C.c_int]),
    "ipmg_sizes": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                             C.POINTER(C.c_int64)]),
    "ipmg_dof_map": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "ipmg_slot_of": (C.c_int64, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
    "ipmg_element_matrix": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ipmg_set_density": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ipmg_apply_K": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ipmg_mg_setup": (C.c_int, [C.c_void_p, C.c_int]),
    "ipmg_level_damping": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "ipmg_vcycle": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "ipmg_apply_Z": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ipmg_pcg": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_int,
                           C.POINTER(PCGInfo)]),
    "ipmg_pcg_noalloc": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_int,
                                   C.POINTER(PCGInfo)]),
    "ipmg_pcg_noalloc_bytes": (C.c_int64, [C.c_void_p]),
    "ipmg_oc_update": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double,
                                 C.c_double, C.c_double, C.c_void_p, C.c_void_p, C.POINTER(OCInfo)]),
    "ipmg_filter": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_int]),
    "ipmg_simp_compliance": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double,
                                       C.c_int, C.c_void_p, C.c_void_p, C.POINTER(PCGInfo)]),
    "ipmg_element_sens": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]),
    "ipmg_ip_init": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(IPParams), C.POINTER(IPState),
                               C.POINTER(PCGInfo)]),
    "ipmg_ip_prepare": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(IPParams), C.POINTER(IPState),
                                  C.c_void_p]),
    "ipmg_ip_step": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(IPParams), C.POINTER(IPState),
                               C.POINTER(IPInfo)]),
    "ipmg_simp_ip_init": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(IPParams), C.c_double, C.c_double,
                                    C.POINTER(IPState), C.POINTER(PCGInfo)]),
    "ipmg_simp_ip_step": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(IPParams), C.c_double, C.c_double,
                                    C.POINTER(IPState), C.POINTER(IPInfo)]),
    "ipmg_profile_begin": (C.c_int, [C.c_void_p, C.c_uint, C.c_int]),
    "ipmg_profile_end": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
}

_lib = None


def load():
    """Load libipmg.so (built in-tree by paper_1606_06201_amd.build).  Raises if it is
    missing: there is no fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1606_06201_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
