"""ctypes binding of libpr.so (the C ABI declared in include/pr.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels. Loading fails loudly when the built library is missing; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpr.so")

PR_OK, PR_EINVAL, PR_ENOMEM, PR_EDEVICE, PR_ENUMERIC, PR_EUNSUPPORTED = range(6)
PR_SPLIT_DIM, PR_SPLIT_DD = 0, 1
PR_FIE, PR_DR = 0, 1
PR_COEF_FACES, PR_COEF_NODAL_LOG = 0, 1
(PR_OPT_GRAPH, PR_OPT_FINE_CHUNK, PR_OPT_LANES, PR_OPT_BLOCKS_PER_PASS, PR_OPT_TWISTED, PR_OPT_GROUPED,
 PR_OPT_PARTITIONED, PR_OPT_PARTITIONED_USED) = (1, 2, 3, 4, 5, 6, 7, 8)

STATUS_NAMES = {0: "PR_OK", 1: "PR_EINVAL", 2: "PR_ENOMEM", 3: "PR_EDEVICE", 4: "PR_ENUMERIC",
                5: "PR_EUNSUPPORTED"}

_dp = C.POINTER(C.c_double)


class PrProblemDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
        ("T", C.c_double),
        ("n_slices", C.c_int), ("fine_steps", C.c_int), ("coarse_steps", C.c_int),
        ("fine", C.c_int), ("split", C.c_int), ("coef_mode", C.c_int),
        ("coef_x", C.c_void_p), ("coef_y", C.c_void_p),
        ("c", C.c_double),
        ("n_colors", C.c_int),
        ("rho", C.c_void_p),
        ("n_forcing", C.c_int),
        ("forcing_space", C.c_void_p),
        ("forcing_time_fine", C.c_void_p),
        ("forcing_time_coarse", C.c_void_p),
    ]


class PrInstanceLayout(C.Structure):
    _fields_ = [("u0_offset", C.c_size_t), ("slices_offset", C.c_size_t),
                ("states_offset", C.c_size_t), ("npts", C.c_int), ("n_slices", C.c_int)]


PROFILE_PHASES = 8
PHASE_NAMES = ["fine_sweep", "fine_transpose", "coarse_x", "coarse_y", "other", "coarse_sweep", "p6",
               "p7"]


class PrProfile(C.Structure):
    _fields_ = [("ms", C.c_double * PROFILE_PHASES), ("count", C.c_longlong * PROFILE_PHASES)]


class PrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libpr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2502_08370_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        vp, i, d = C.c_void_p, C.c_int, C.c_double
        sigs = {
            "pr_create_problem": [C.POINTER(PrProblemDesc), i, vp, C.POINTER(vp)],
            "pr_destroy_problem": [vp],
            "pr_query_layout": [vp, C.POINTER(PrInstanceLayout), C.POINTER(C.c_size_t)],
            "pr_num_instances": [vp, C.POINTER(i)],
            "pr_set_coefficients": [vp, i, vp, vp, vp],
            "pr_fine_propagate": [vp, vp, vp, vp],
            "pr_coarse_sweep": [vp, vp, vp, vp, vp, vp],
            "pr_parareal_iterate": [vp, vp, vp, i, d, C.POINTER(i), _dp, vp],
            "pr_sequential_fine": [vp, vp, vp, vp],
            "pr_adjoint": [vp, vp, vp, vp, vp, vp, vp],
            "pr_adjoint_noalloc": [vp, vp, vp, vp, vp, vp, vp],
            "pr_adjoint_parallel": [vp, vp, vp, vp, vp, vp, i, d, C.POINTER(i), vp],
            "pr_profile_control": [vp, i],
            "pr_profile_read": [vp, C.POINTER(PrProfile)],
            "pr_set_option": [vp, i, i],
            "pr_get_option": [vp, i, C.POINTER(i)],
            "pr_autotune": [vp, vp, C.POINTER(i), C.POINTER(i), C.POINTER(C.c_float)],
        }
        for name, args in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.pr_last_error.argtypes = []
        L.pr_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def check(status):
    if status != PR_OK:
        raise PrError(status, lib().pr_last_error().decode(errors="replace"))
    return status


def exported_symbols():
    """Names of the pr_* entry points this binding knows (all declared in pr.h)."""
    return ["pr_create_problem", "pr_destroy_problem", "pr_query_layout", "pr_num_instances",
            "pr_set_coefficients", "pr_fine_propagate", "pr_coarse_sweep", "pr_parareal_iterate",
            "pr_sequential_fine", "pr_adjoint", "pr_adjoint_noalloc", "pr_adjoint_parallel", "pr_profile_control",
            "pr_profile_read", "pr_set_option", "pr_get_option", "pr_autotune", "pr_last_error"]
