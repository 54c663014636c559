"""ctypes loader of libmgpoisson.so (the C ABI of include/mg.h).

Argument marshalling only: every step of the solve runs in the HIP library.  The
library must have been built in-tree (python -m paper_1410_2240_amd.build); there is
no fallback path, so a missing library is an error.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmgpoisson.so")

MG_OK, MG_EINVAL, MG_EWORKSPACE, MG_EHIP, MG_ENOCONV, MG_EBREAKDOWN = 0, -1, -2, -3, -4, -5
MG_FP64, MG_MIXED, MG_KRYLOV, MG_COARSEN_DENSITY, MG_FROM_RHO = 0, 1, 2, 4, 8
MG_PREC_F64, MG_PREC_F32 = 0, 1
MG_PRE, MG_POST = 0, 1
MG_MAX_LANES = 16

ERROR_NAMES = {MG_EINVAL: "MG_EINVAL", MG_EWORKSPACE: "MG_EWORKSPACE", MG_EHIP: "MG_EHIP",
               MG_ENOCONV: "MG_ENOCONV", MG_EBREAKDOWN: "MG_EBREAKDOWN"}


class MgStats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("levels", ctypes.c_int),
                ("active_cells", ctypes.c_longlong), ("dropped_cells", ctypes.c_longlong),
                ("removed_mean", ctypes.c_double), ("final_relres", ctypes.c_double),
                ("seconds", ctypes.c_double), ("ws_bytes", ctypes.c_size_t)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_DIMS = ctypes.POINTER(ctypes.c_int)

# name -> (restype, argtypes); the same set of functions include/mg.h declares
SIGNATURES = {
    "mg_workspace_size": (ctypes.c_size_t, [_DIMS, _I]),
    "mg_coeffs_from_rho": (_I, [_P, _P, _DIMS, _P, _P, _P, _P]),
    "mg_setup": (_I, [ctypes.POINTER(_P), _P, ctypes.c_size_t, _P, _P, _P, _P, _DIMS, _D, _I, _P]),
    "mg_setup_from_rho": (_I, [ctypes.POINTER(_P), _P, ctypes.c_size_t, _P, _P, _DIMS, _D, _I, _P]),
    "mg_set_stream": (_I, [_P, _P]),
    "mg_solve": (_I, [_P, _P, _P, _I, _D, _I, ctypes.POINTER(_D), ctypes.POINTER(_I), ctypes.POINTER(MgStats)]),
    "mg_solve_static": (_I, [_P, _P, _P, _I, _D, _I, ctypes.POINTER(_D), ctypes.POINTER(_I), ctypes.POINTER(MgStats)]),
    "mg_lane_workspace_size": (ctypes.c_size_t, [_DIMS, _I]),
    "mg_add_lanes": (_I, [_P, _P, ctypes.c_size_t, _I]),
    "mg_apply": (_I, [_P, _P, _P, _I]),
    "mg_coeff_grad": (_I, [_P, _P, _P, _I, _P, _P, _P, _P]),
    "mg_divergence": (_I, [_P, _P, _P, _P, _P, _P, _P, _D, _P]),
    "mg_project": (_I, [_P, _P, _P, _P, _P, _P, _P, _D, _P]),
    "mg_cut_cells": (_I, [_P, _DIMS, _I, _P, _P, _P, _P, _P, _P]),
    "mg_cut_coeffs": (_I, [_P, _P, _P, _P, _P, _P, _DIMS, _P, _P, _P, _P, _P]),
    "mg_merge_rhs": (_I, [_P, _P, _P, _DIMS, _P]),
    "mg_merge_fill": (_I, [_P, _P, _DIMS, _P]),
    "mg_destroy": (None, [_P]),
    "mg_last_error": (ctypes.c_char_p, []),
    "mg_level_info": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_D)]),
    "mg_level_coeffs": (_I, [_P, _I, _P, _P, _P, _P]),
    "mg_smooth": (_I, [_P, _I, _I, _P, _P, _I, _I]),
    "mg_residual_restrict": (_I, [_P, _I, _I, _P, _P, _P]),
    "mg_prolong_add": (_I, [_P, _I, _I, _P, _P]),
    "mg_coarse_solve": (_I, [_P, _I, _P, _P]),
    "mg_vcycle": (_I, [_P, _I, _P, _P]),
}

_lib = None


def load():
    """Load the library once; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1410_2240_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def dims3(n: int):
    return (ctypes.c_int * 3)(n, n, n)


def last_error() -> str:
    msg = load().mg_last_error()
    return msg.decode() if msg else ""
