"""MI355X-native bake-off library (BP1-BP6 hot path).

The compute path is libbp.so (HIP kernels for gfx950 behind the C ABI in
include/bp.h); this package holds its build script, the ctypes binding, a
torch.autograd wrapper of the variable-coefficient solve, and the byte/flop
model used to report roofline fractions. Importing the package does not load
the library; Operator(...) does, and raises if it is not built.
"""
from ._lib import (BP_FP32, BP_FP64, BP_MASS, BP_QUAD_GL, BP_QUAD_GLL, BP_STIFF, BpError)

__all__ = ["BP_FP32", "BP_FP64", "BP_MASS", "BP_QUAD_GL", "BP_QUAD_GLL", "BP_STIFF",
           "BpError", "Operator", "rule", "bp_quadrature"]


def __getattr__(name):
    if name in ("Operator", "rule", "bp_quadrature", "MASS", "STIFF", "GL", "GLL"):
        from . import bp
        return getattr(bp, name)
    raise AttributeError(name)
