"""ctypes declarations of libofks.so (the C ABI in include/ofks.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libofks.so")

OFKS_OK = 0
OFKS_NOT_CONVERGED = 1
PRECOND = {"none": 0, "paper": 1, "learned": 2, "graph": 3}
STEP = {"bb2": 0, "bb1": 1, "abb1": 2, "abb2": 3, "fixed": 4}
PRECISION = {"f64": 0, "f32": 1}

_c_double = ctypes.c_double
_c_int32 = ctypes.c_int32


class Params(ctypes.Structure):
    _fields_ = [
        ("beta", _c_double),
        ("eta0", _c_double),
        ("tol", _c_double),
        ("step_rule", _c_int32),
        ("precond", _c_int32),
        ("pcg_iters", _c_int32),
        ("precision", _c_int32),
        ("precond_lambda", _c_int32),
        ("max_iter", _c_int32),
        ("occupation", _c_double),
        ("scf", _c_int32),
        ("energy_every", _c_int32),
        ("refine_tol", _c_double),
        ("poisson_rtol", _c_double),
        ("poisson_max_iter", _c_int32),
        ("fallback_window", _c_int32),
        ("fallback_hold", _c_int32),
        ("fallback_rule", _c_int32),
        ("use_graphs", _c_int32),
        ("algorithm", _c_int32),
        ("spmm_mode", _c_int32),
        ("fallback_stall", _c_int32),
        ("poisson_adapt", _c_double),
        ("graph_sweeps", _c_int32),
    ]


class IterStats(ctypes.Structure):
    _fields_ = [
        ("k", _c_int32),
        ("precond_used", _c_int32),
        ("precision", _c_int32),
        ("fell_back", _c_int32),
        ("energy", _c_double),
        ("kkt", _c_double),
        ("fea", _c_double),
        ("rel", _c_double),
        ("eta", _c_double),
        ("ms", _c_double),
    ]


# (name, restype, argtypes)
P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int32
SIGNATURES = [
    ("ofks_default_params", None, [ctypes.POINTER(Params)]),
    ("ofks_create", I32, [ctypes.POINTER(P), P]),
    ("ofks_destroy", I32, [P]),
    ("ofks_last_error", ctypes.c_char_p, [P]),
    ("ofks_mesh_load", I32, [P, I64, P, I64, P, P]),
    ("ofks_nuclei_set", I32, [P, I32, P, P]),
    ("ofks_assemble", I32, [P]),
    ("ofks_csr_info", I32, [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]),
    ("ofks_iterate_info", I32, [P, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32)]),
    ("ofks_csr_get", I32, [P, P, P, P, P, P]),
    ("ofks_csr_load", I32, [P, I64, I64, P, P, P, P, P]),
    ("ofks_set_params", I32, [P, ctypes.POINTER(Params)]),
    ("ofks_workspace_size", I32, [P, I32, ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]),
    ("ofks_set_workspace", I32, [P, P, ctypes.c_size_t]),
    ("ofks_set_x0", I32, [P, I32, P, I32]),
    ("ofks_step", I32, [P, I32, ctypes.POINTER(IterStats), ctypes.POINTER(I32), ctypes.POINTER(I32)]),
    ("ofks_residual", I32, [P, ctypes.POINTER(_c_double), ctypes.POINTER(_c_double), ctypes.POINTER(_c_double)]),
    ("ofks_energy", I32, [P, P]),
    ("ofks_postprocess", I32, [P, P]),
    ("ofks_get_x", I32, [P, P]),
    ("ofks_get_density", I32, [P, P]),
    ("ofks_update_density", I32, [P]),
    ("ofks_state_size", I32, [P, ctypes.POINTER(ctypes.c_size_t)]),
    ("ofks_state_get", I32, [P, P, ctypes.c_size_t]),
    ("ofks_state_set", I32, [P, P, ctypes.c_size_t]),
    ("ofks_spmm", I32, [P, I32, P, P, P]),
    ("ofks_spmm_ex", I32, [P, I32, I32, I32, P, P, P, P]),
    ("ofks_gram", I32, [P, I32, P, P, P, P, P]),
    ("ofks_gram_noalloc", I32, [P, I32, P, P, P, P, P]),
    ("ofks_precondition", I32, [P, I32, P, P, P]),
    ("ofks_build_hamiltonian", I32, [P, I32, P, P, P, P, P, P]),
    ("ofks_lp_set_weights", I32, [P, P, P]),
    ("ofks_lp_collect", I32, [P, I64, I32, P, I64]),
    ("ofks_lp_collected", I32, [P, ctypes.POINTER(I64)]),
    ("ofks_lp_train", I32, [P, P, I64, I32, ctypes.c_float, P, P, P]),
    ("ofks_lp_loss_grad", I32, [P, P, I64, P, P, ctypes.POINTER(_c_double), P]),
    ("ofks_lp_apply", I32, [P, I32, P, P, P]),
    ("ofks_lp_features", I32, [P, I32, P, P]),
    ("ofks_gl_set_weights", I32, [P, P, P]),
    ("ofks_gl_apply", I32, [P, I32, P, P, P]),
    ("ofks_gl_loss_grad", I32, [P, I32, P, P, ctypes.POINTER(_c_double), P]),
    ("ofks_gl_capture", I32, [P, P, I32, I64]),
    ("ofks_gl_captured", I32, [P, ctypes.POINTER(I32), P]),
    ("ofks_gl_train", I32, [P, I32, P, P, I32, I32, ctypes.c_float, P, P, P]),
    ("ofks_gl_feature_norm", I32, [P, P]),
    ("ofks_timing", I32, [P, I32]),
    ("ofks_timer_get", I32, [P, ctypes.c_char_p, ctypes.POINTER(_c_double), ctypes.POINTER(I64)]),
]

_lib = None


def load(path: str = None):
    """Loads the HIP library; raises if it has not been built.

    torch is imported first so that libofks.so binds to the HIP runtime that
    torch has already loaded: one runtime per process, shared streams and
    device memory."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime the library must share)
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2007_14228_amd.build`")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
