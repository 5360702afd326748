"""Python binding of the bake-off library: argument marshalling only.

Every computation runs in libbp.so's HIP kernels; torch supplies device
memory (tensors) and the current HIP stream. Vectors with several components
are component-major tensors [ncomp, nglobal].
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (BP_FP32, BP_FP64, BP_HELM, BP_MASKED, BP_MASS, BP_QUAD_GL, BP_QUAD_GLL,
                   BP_SETUP_CALLER_ORDER, BP_SETUP_FP32, BP_STIFF, PcgStats, check)

MASS, STIFF, HELM = BP_MASS, BP_STIFF, BP_HELM
GL, GLL = BP_QUAD_GL, BP_QUAD_GLL


def rule(n: int, quad: int):
    """The library's 1D rule: (points, weights) as numpy arrays."""
    lib = _lib.load()
    x = np.zeros(n)
    w = np.zeros(n)
    check(lib.bp_rule(n, quad, x.ctypes.data, w.ctypes.data))
    return x, w


def bp_quadrature(bp: int, p: int):
    """(q, quad) that Table "bps" assigns to BPj at order p."""
    if bp in (1, 2, 3, 4):
        return p + 2, GL
    if bp in (5, 6):
        return p + 1, GLL
    raise ValueError(bp)


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Operator:
    """A mesh + order + quadrature on the current HIP device (bp_setup)."""

    def __init__(self, p: int, q: int, quad: int, elem_dofs, node_xyz, nglobal: int,
                 dirichlet=None, ncomp: int = 1, fp32: bool = False, caller_order: bool = False):
        self._lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        ed = np.ascontiguousarray(elem_dofs, dtype=np.int64)
        xyz = np.ascontiguousarray(node_xyz, dtype=np.float64)
        p1 = p + 1
        if ed.ndim != 2 or ed.shape[1] != p1 ** 3:
            raise ValueError("elem_dofs must be [nelem, (p+1)^3]")
        if xyz.shape != (ed.shape[0], p1 ** 3, 3):
            raise ValueError("node_xyz must be [nelem, (p+1)^3, 3]")
        dr = None
        if dirichlet is not None:
            dr = np.ascontiguousarray(dirichlet, dtype=np.uint8)
            if dr.shape != (nglobal,):
                raise ValueError("dirichlet must be [nglobal]")
        self.p, self.q, self.quad, self.ncomp = p, q, quad, ncomp
        self.nelem, self.nglobal = ed.shape[0], int(nglobal)
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p()
        check(self._lib.bp_setup(ctypes.byref(h), p, q, quad, ncomp, self.nelem, self.nglobal,
                                 ed.ctypes.data, xyz.ctypes.data,
                                 None if dr is None else dr.ctypes.data,
                                 (BP_SETUP_FP32 if fp32 else 0)
                                 | (BP_SETUP_CALLER_ORDER if caller_order else 0), _stream()))
        self._h = h

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize()
            self._lib.bp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------
    def _vec(self, t: torch.Tensor, dtype=torch.float64, name="vector") -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a device tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}")
        if t.numel() != self.nglobal * self.ncomp or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with nglobal*ncomp entries")
        return t

    def new_vector(self, dtype=torch.float64) -> torch.Tensor:
        """Zero vector; component-major [ncomp, nglobal] when ncomp > 1."""
        shape = (self.nglobal,) if self.ncomp == 1 else (self.ncomp, self.nglobal)
        return torch.zeros(shape, dtype=dtype, device=self.device)

    def apply(self, which: int, u: torch.Tensor, out: torch.Tensor | None = None,
              masked: bool = True) -> torch.Tensor:
        """w = [mask] Q^T A_L Q [mask] u (bp_apply); FP32 if u is float32."""
        prec = BP_FP32 if u.dtype == torch.float32 else BP_FP64
        self._vec(u, u.dtype, "u")
        w = torch.empty_like(u) if out is None else self._vec(out, u.dtype, "out")
        check(self._lib.bp_apply(self._h, which, prec, _ptr(u), _ptr(w),
                                 BP_MASKED if masked else 0, _stream()))
        return w

    def apply_local(self, which: int, uL: torch.Tensor,
                    out: torch.Tensor | None = None) -> torch.Tensor:
        """w_L = A_L u_L or B_L u_L per element, no gather or scatter
        (bp_apply_local). uL: [ncomp][nelem][(p+1)^3] (any shape with that many
        contiguous entries); FP32 if uL is float32."""
        prec = BP_FP32 if uL.dtype == torch.float32 else BP_FP64
        nl = self.ncomp * self.nelem * (self.p + 1) ** 3
        for t, name in ((uL, "uL"), (out, "out")):
            if t is None:
                continue
            if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
                raise TypeError(f"{name} must be a device tensor")
            if t.dtype != uL.dtype or t.numel() != nl or not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous {uL.dtype} with "
                                 "ncomp*nelem*(p+1)^3 entries")
        w = torch.empty_like(uL) if out is None else out
        check(self._lib.bp_apply_local(self._h, which, prec, _ptr(uL), _ptr(w), _stream()))
        return w

    def diag(self, which: int, masked: bool = True) -> torch.Tensor:
        d = torch.empty(self.nglobal, dtype=torch.float64, device=self.device)
        check(self._lib.bp_diag(self._h, which, _ptr(d), BP_MASKED if masked else 0, _stream()))
        return d

    def set_option(self, option: int, value: int):
        check(self._lib.bp_set_option(self._h, option, value))

    def set_cg_variant(self, single_reduction: bool):
        """PCG recurrences of pcg_solve: standard (two reduction phases per
        iteration) or single-reduction (Chronopoulos-Gear)."""
        self.set_option(_lib.BP_OPT_CG_VARIANT, _lib.BP_CG_SINGLE_REDUCTION if single_reduction
                        else _lib.BP_CG_STANDARD)

    def set_coeff(self, kappa: torch.Tensor | None):
        if kappa is not None:
            if kappa.dtype != torch.float64 or kappa.device.type != "cuda" or \
                    kappa.numel() != self.nelem * self.q ** 3 or not kappa.is_contiguous():
                raise ValueError("kappa must be a contiguous float64 device tensor [nelem, q^3]")
        check(self._lib.bp_set_coeff(self._h, _ptr(kappa), _stream()))

    def set_helmholtz(self, beta: float = 0.0, beta_q: torch.Tensor | None = None):
        """beta of H = A + B_beta for which=HELM (bp_set_helmholtz): a constant,
        or beta_q [nelem, q^3] at the quadrature points."""
        if beta_q is not None:
            if beta_q.dtype != torch.float64 or beta_q.device.type != "cuda" or \
                    beta_q.numel() != self.nelem * self.q ** 3 or not beta_q.is_contiguous():
                raise ValueError("beta_q must be a contiguous float64 device tensor [nelem, q^3]")
        check(self._lib.bp_set_helmholtz(self._h, float(beta), _ptr(beta_q), _stream()))

    def pcg_solve(self, b: torch.Tensor, x: torch.Tensor | None = None, which: int = STIFF,
                  rtol: float = 1e-8, maxit: int = 1000, fixed_iters: bool = False):
        """Jacobi-PCG (bp_pcg_solve). Returns (x, stats dict)."""
        self._vec(b, name="b")
        x = torch.zeros_like(b) if x is None else self._vec(x, name="x")
        st = PcgStats()
        check(self._lib.bp_pcg_solve(self._h, which, _ptr(b), _ptr(x), float(rtol), int(maxit),
                                     1 if fixed_iters else 0, ctypes.byref(st), _stream()))
        return x, st.as_dict()

    def pcg_solve_mixed(self, b: torch.Tensor, x: torch.Tensor | None = None,
                        outer_rtol: float = 1e-10, inner_rtol: float = 1e-5,
                        max_outer: int = 50, max_inner: int = 2000, reliable: bool = False):
        """FP32-inner solve with FP64 corrections (bp_pcg_solve_mixed): restarted
        defect correction, or with reliable=True one FP32 CG with FP64 residual
        replacement whenever its residual has dropped by inner_rtol."""
        self._vec(b, name="b")
        x = torch.zeros_like(b) if x is None else self._vec(x, name="x")
        check(self._lib.bp_set_option(self._h, _lib.BP_OPT_MIXED_MODE,
                                      _lib.BP_MIXED_RELIABLE if reliable else
                                      _lib.BP_MIXED_RESTART))
        st = PcgStats()
        check(self._lib.bp_pcg_solve_mixed(self._h, _ptr(b), _ptr(x), float(outer_rtol),
                                           float(inner_rtol), int(max_outer), int(max_inner),
                                           ctypes.byref(st), _stream()))
        return x, st.as_dict()

    def grad_kappa(self, lam: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
        self._vec(lam, name="lam")
        self._vec(u, name="u")
        g = torch.empty((self.nelem, self.q ** 3), dtype=torch.float64, device=self.device)
        check(self._lib.bp_grad_kappa(self._h, _ptr(lam), _ptr(u), _ptr(g), _stream()))
        return g

    def mass_misfit(self, u: torch.Tensor, u_target: torch.Tensor, grad: bool = True):
        """L = 1/2 sum_c (u - u_t)_c^T M (u - u_t)_c with the unmasked mass
        matrix, and M (u - u_t) (None without grad); bp_mass_misfit."""
        self._vec(u, name="u")
        self._vec(u_target, name="u_target")
        g = torch.empty_like(u) if grad else None
        loss = ctypes.c_double(0.0)
        check(self._lib.bp_mass_misfit(self._h, _ptr(u), _ptr(u_target),
                                       _ptr(g) if g is not None else None, ctypes.byref(loss),
                                       _stream()))
        return loss.value, g
