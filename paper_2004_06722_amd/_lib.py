"""ctypes declarations of libbp.so (include/bp.h). No fallback: if the
library is not built, loading raises."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbp.so")

BP_OK, BP_ERR_ARG, BP_ERR_MESH, BP_ERR_HIP = 0, -1, -2, -3
BP_ERR_NONFINITE, BP_ERR_BREAKDOWN, BP_ERR_OOM = -4, -5, -6
BP_QUAD_GL, BP_QUAD_GLL = 0, 1
BP_MASS, BP_STIFF, BP_HELM = 1, 3, 4
BP_FP64, BP_FP32 = 0, 1
BP_MASKED = 1
BP_SETUP_FP32 = 1
BP_SETUP_CALLER_ORDER = 2
BP_OPT_TIME_APPLY = 1
BP_OPT_MIXED_MODE = 2
BP_MIXED_RESTART, BP_MIXED_RELIABLE = 0, 1
BP_OPT_CG_VARIANT = 3
BP_OPT_CG_FUSE = 5
BP_CG_STANDARD, BP_CG_SINGLE_REDUCTION = 0, 1
BP_STATIC_WS_MB = 64

ERROR_NAMES = {BP_ERR_ARG: "BP_ERR_ARG", BP_ERR_MESH: "BP_ERR_MESH", BP_ERR_HIP: "BP_ERR_HIP",
               BP_ERR_NONFINITE: "BP_ERR_NONFINITE", BP_ERR_BREAKDOWN: "BP_ERR_BREAKDOWN",
               BP_ERR_OOM: "BP_ERR_OOM"}


class BpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class PcgStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer", ctypes.c_int), ("converged", ctypes.c_int),
                ("ncomp", ctypes.c_int), ("rel_res", ctypes.c_double * 8), ("ms", ctypes.c_double),
                ("apply_ms", ctypes.c_double), ("apply_count", ctypes.c_int), ("pad_", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {"iters": self.iters, "outer": self.outer, "converged": bool(self.converged),
                "rel_res": list(self.rel_res[: self.ncomp]), "ms": self.ms,
                "apply_ms": self.apply_ms, "apply_count": self.apply_count}


_vp, _i, _i64, _d, _u = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_uint

# name -> (restype, argtypes); the exported C ABI of include/bp.h
SIGNATURES = {
    "bp_version": (_i, []),
    "bp_rule": (_i, [_i, _i, _vp, _vp]),
    "bp_setup": (_i, [ctypes.POINTER(_vp), _i, _i, _i, _i, _i64, _i64, _vp, _vp, _vp, _u, _vp]),
    "bp_info": (_i, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "bp_set_coeff": (_i, [_vp, _vp, _vp]),
    "bp_set_helmholtz": (_i, [_vp, ctypes.c_double, _vp, _vp]),
    "bp_apply": (_i, [_vp, _i, _i, _vp, _vp, _u, _vp]),
    "bp_apply_local": (_i, [_vp, _i, _i, _vp, _vp, _vp]),
    "bp_diag": (_i, [_vp, _i, _vp, _u, _vp]),
    "bp_pcg_solve": (_i, [_vp, _i, _vp, _vp, _d, _i, _i, ctypes.POINTER(PcgStats), _vp]),
    "bp_pcg_solve_static": (_i, [_vp, _i, _vp, _vp, _d, _i, _i, ctypes.POINTER(PcgStats), _vp]),
    "bp_pcg_solve_mixed": (_i, [_vp, _vp, _vp, _d, _d, _i, _i, ctypes.POINTER(PcgStats), _vp]),
    "bp_grad_kappa": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "bp_mass_misfit": (_i, [_vp, _vp, _vp, _vp, ctypes.POINTER(_d), _vp]),
    "bp_set_option": (_i, [_vp, _i, _i]),
    "bp_destroy": (_i, [_vp]),
    "bp_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libbp.so once; raise ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built (run: python -m paper_2004_06722_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != BP_OK:
        msg = load().bp_last_error().decode(errors="replace")
        raise BpError(rc, msg)
