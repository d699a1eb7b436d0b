"""ctypes loader for libadelia.so (the HIP library built from csrc/ for gfx950).

Argument marshalling only: every step of the computation runs in the library's kernels.
Loading fails loudly when the library has not been built; there is no fallback path.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadelia.so")

_lib = None

c_int = C.c_int
c_int32 = C.c_int32
c_double = C.c_double
c_size_t = C.c_size_t
c_ll = C.c_longlong
vp = C.c_void_p
i32p = C.c_void_p


class BtaShape(C.Structure):
    _fields_ = [("n", C.c_int32), ("b", C.c_int32), ("a", C.c_int32)]


class ModelDesc(C.Structure):
    _fields_ = [
        ("param", C.c_int32), ("k", C.c_int32), ("ns", C.c_int32), ("nt", C.c_int32),
        ("a", C.c_int32), ("n_obs", C.c_int32),
        ("c0_ptr", vp), ("c0_idx", vp), ("c0_val", vp),
        ("g1_ptr", vp), ("g1_idx", vp), ("g1_val", vp),
        ("g2_ptr", vp), ("g2_idx", vp), ("g2_val", vp),
        ("m0_diag", vp), ("m0_off", vp), ("m1_diag", vp), ("m1_off", vp),
        ("m2_diag", vp), ("m2_off", vp),
        ("obs_t", vp), ("obs_field", vp), ("obs_node", vp), ("obs_w", vp),
        ("X", vp), ("y", vp),
        ("sigma_prior", C.c_double), ("tip_prec", C.c_double),
    ]


class KernelStats(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("ms", C.c_double),
                ("flops", C.c_double), ("bytes", C.c_double)]


# name -> (restype, argtypes)
SIGNATURES = {
    "adelia_create": (c_int, [C.POINTER(vp), c_int]),
    "adelia_destroy": (c_int, [vp]),
    "adelia_strerror": (C.c_char_p, [c_int]),
    "adelia_version": (C.c_char_p, []),
    "adelia_last_error": (C.c_char_p, []),
    "adelia_dgemm": (c_int, [vp, c_int, c_int, c_int, c_int, c_int, c_double, vp, c_int, c_ll,
                             vp, c_int, c_ll, c_double, vp, c_int, c_ll, c_int, c_int, vp]),
    "adelia_bta_workspace_bytes": (c_size_t, [BtaShape, c_int]),
    "bta_factor": (c_int, [vp, BtaShape, vp, vp, vp, vp, vp, vp, vp, vp, vp, c_size_t, vp]),
    "bta_factor_noalloc": (c_int, [vp, BtaShape, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
    "adelia_bta_batched_workspace_bytes": (c_size_t, [c_int, C.POINTER(BtaShape), c_int]),
    "bta_factor_batched": (c_int, [vp, c_int, C.POINTER(BtaShape), C.POINTER(vp), C.POINTER(vp),
                                   C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                   vp, vp, vp, c_size_t, vp]),
    "bta_logdet": (c_int, [vp, BtaShape, vp, vp, vp, vp, c_size_t, vp]),
    "bta_solve": (c_int, [vp, BtaShape, vp, vp, vp, vp, vp, c_int, vp, c_size_t, vp]),
    "bta_selinv": (c_int, [vp, BtaShape, vp, vp, vp, vp, vp, vp, vp, vp, vp, c_size_t, vp]),
    "inla_model_create": (c_int, [vp, C.POINTER(ModelDesc), C.POINTER(vp)]),
    "inla_model_destroy": (c_int, [vp]),
    "inla_model_dim": (c_int, [vp]),
    "inla_workspace_bytes": (c_size_t, [vp, c_int, c_int]),
    "inla_objective": (c_int, [vp, vp, c_int32, vp, vp, vp, c_size_t, c_int, vp]),
    "inla_grad": (c_int, [vp, vp, vp, vp, vp, vp, c_size_t, c_int, vp]),
    "inla_grad_terms": (c_int, [vp, vp, vp, vp, vp, c_size_t, c_int, vp]),
    "inla_fd_grad": (c_int, [vp, vp, c_double, c_int32, vp, vp, vp, vp, c_size_t, vp]),
    "inla_grad_batched": (c_int, [vp, vp, c_int32, vp, vp, vp, vp, c_size_t, vp]),
    "inla_hessian": (c_int, [vp, vp, c_double, c_int32, vp, vp, vp, vp, vp, c_size_t, vp]),
    "inla_fd_hessian": (c_int, [vp, vp, c_double, c_int32, vp, vp, vp, vp, c_size_t, vp]),
    "inla_batch_create": (c_int, [vp, c_int, C.POINTER(vp), C.POINTER(vp)]),
    "inla_batch_destroy": (c_int, [vp]),
    "inla_batch_groups": (c_int, [vp]),
    "inla_batch_workspace_bytes": (c_size_t, [vp, c_int]),
    "inla_batch_objective": (c_int, [vp, vp, vp, vp, vp, c_size_t, vp]),
    "inla_batch_grad": (c_int, [vp, vp, vp, vp, vp, vp, c_size_t, vp]),
    "adelia_tune_set": (c_int, [c_int, c_int, c_int]),
    "adelia_tune_get": (c_int, [c_int, c_int]),
    "adelia_tune_clear": (c_int, []),
    "adelia_tune_save": (c_int, [C.c_char_p]),
    "adelia_tune_load": (c_int, [C.c_char_p]),
    "inla_autotune": (c_int, [vp, vp, c_int32, c_int, c_int, vp, c_size_t, vp, C.POINTER(c_int32)]),
    "inla_batch_autotune": (c_int, [vp, vp, c_int, c_int, vp, c_size_t, vp, C.POINTER(c_int32)]),
    "adelia_profile_start": (c_int, [vp, c_int]),
    "adelia_profile_stop": (c_int, [vp, C.POINTER(KernelStats), c_int, C.POINTER(c_int)]),
}


def lib():
    """Load (once) and return the library handle; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2605_06392_amd.build` "
            "(or __graft_entry__.build()); there is no CPU fallback")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


class AdeliaError(RuntimeError):
    pass


def check(code, what=""):
    if code != 0:
        msg = lib().adelia_strerror(code).decode()
        extra = lib().adelia_last_error().decode()
        raise AdeliaError(f"{what} failed with code {code}: {msg}" + (f" ({extra})" if extra else ""))
