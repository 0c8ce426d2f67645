"""ctypes declarations of libsem's C ABI (include/sem.h).

Argument marshalling only: every computation runs inside libsem.so.  Loading
fails loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsem.so")

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p
c_char_p = ctypes.c_char_p

SEM_OK, SEM_EINVAL, SEM_ENOMEM, SEM_EDEVICE, SEM_ENOCONV, SEM_EBREAKDOWN, SEM_ENOTSUP = (
    0, -1, -2, -3, -4, -5, -6)
STATUS_NAMES = {0: "SEM_OK", -1: "SEM_EINVAL", -2: "SEM_ENOMEM", -3: "SEM_EDEVICE",
                -4: "SEM_ENOCONV", -5: "SEM_EBREAKDOWN", -6: "SEM_ENOTSUP"}
PREC = {"fp64": 0, "fp32": 1, "bf16_mfma": 2, "fp16_mfma": 3}
PRECOND = {"jacobi": 0, "chebyshev": 1, "pmg": 2, "chebyshev1": 3}
PMG_MAX_LEVELS = 8
SMOOTHER = {"jacobi": 0, "schwarz": 1}
MODE = {"cg": 0, "mixed_ir": 1}


class MeshDesc(ctypes.Structure):
    _fields_ = [("N", c_int32), ("E", c_int64), ("xyz", c_void_p), ("gid", c_void_p),
                ("dirichlet", c_void_p)]


class MeshInfo(ctypes.Structure):
    _fields_ = [("E", c_int64), ("n_local", c_int64), ("n_unique", c_int64),
                ("n_free", c_int64), ("n_shared", c_int64), ("N", c_int32),
                ("has_nullspace", c_int32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("mode", c_int32), ("precond", c_int32), ("precond_prec", c_int32),
                ("cheb_order", c_int32), ("lmax", c_double), ("rtol", c_double),
                ("max_iter", c_int32), ("fixed_iters", c_int32), ("inner_rtol", c_double),
                ("max_outer", c_int32), ("check_every", c_int32), ("profile", c_int32),
                ("residual_history", c_void_p)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("outer_iters", c_int32), ("operator_applies", c_int32),
                ("converged", c_int32), ("rel_res", c_double), ("time_ms", c_double),
                ("lmax", c_double), ("ax_ms", c_double), ("ax_launches", c_int32),
                ("pad_", c_int32)]


class PmgOpts(ctypes.Structure):
    _fields_ = [("n_levels", c_int32), ("orders", c_int32 * 8), ("smooth_order", c_int32),
                ("coarse_iters", c_int32), ("smoother", c_int32)]


ADV_RULE = {"collocation": 0, "dealias": 1}

# name -> (restype, argtypes)
SIGNATURES = {
    "sem_solve_opts_default": (None, [ctypes.POINTER(SolveOpts)]),
    "sem_gll": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p]),
    "sem_host_numbering": (c_int32, [c_int32, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p]),
    "sem_setup_mesh": (c_int32, [ctypes.POINTER(MeshDesc), c_void_p, ctypes.POINTER(c_void_p)]),
    "sem_free_mesh": (c_int32, [c_void_p]),
    "sem_get_info": (c_int32, [c_void_p, ctypes.POINTER(MeshInfo)]),
    "sem_get_geometry": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "sem_ax": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int32, c_void_p]),
    "sem_mass": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "sem_gs": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p]),
    "sem_mask": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p]),
    "sem_jacobi_inverse": (c_int32, [c_void_p, c_void_p, c_double, c_void_p, c_void_p]),
    "sem_cheb_apply": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int32,
                                 c_double, c_int32, c_void_p]),
    "sem_cheb_apply_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int32,
                                 c_double, c_int32, c_void_p]),
    "sem_pmg_opts_default": (None, [ctypes.POINTER(PmgOpts)]),
    "sem_setup_pmg": (c_int32, [c_void_p, ctypes.POINTER(MeshDesc), ctypes.POINTER(PmgOpts),
                                c_void_p]),
    "sem_pmg_info": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "sem_pmg_apply": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int32,
                                c_void_p]),
    "sem_host_coarse_mesh": (c_int32, [c_int32, c_int64, c_void_p, c_void_p, c_void_p, c_int32,
                                       c_void_p, c_void_p, c_void_p]),
    "sem_host_schwarz": (c_int32, [c_int32, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p]),
    "sem_advection_rule": (c_int32, [c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "sem_setup_advection": (c_int32, [c_void_p, ctypes.POINTER(MeshDesc), c_int32, c_void_p]),
    "sem_get_advection_factors": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "sem_advect": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "sem_advect_fields": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_void_p, c_void_p,
                                    c_int32, c_void_p]),
    "sem_lmax_estimate": (c_int32, [c_void_p, c_void_p, c_double, c_int32,
                                    ctypes.POINTER(c_double), c_void_p]),
    "sem_pcg_solve": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                                ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats), c_void_p]),
    "sem_ax_backward": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_void_p,
                                  c_void_p, c_void_p]),
    "sem_solve_backward": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                                     ctypes.POINTER(SolveOpts), c_void_p, c_void_p,
                                     ctypes.POINTER(SolveStats), c_void_p]),
    "sem_last_error": (c_char_p, []),
}

_lib = None


def load():
    """Load libsem.so (built in-tree); raises ImportError if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2501_13240_amd.build` "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
