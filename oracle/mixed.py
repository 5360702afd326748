"""Single-precision inner PCG inside FP64 defect correction (oracle).

Not in the paper (all its runs are FP64); this is the precision extension of
the hot path: the outer loop forms the FP64 residual r = b - A x, stops when
||r||/||b|| <= outer_rtol, otherwise solves A d = r approximately with a
Jacobi-PCG whose operator, geometric factors and vectors are float32 (dot
products accumulated in float64), and updates x += d in float64.
The inner PCG is the same algorithm as pcg.pcg.

reliable_cg is the second variant: one FP32 Jacobi-PCG whose search
direction is kept for the whole solve, with the FP64 update x += x32 and the
FP64 residual r = b - A x substituted for the recursive FP32 residual
whenever the latter has dropped by the factor delta since the last
substitution ("reliable updates", residual replacement). Keeping p keeps the
Krylov space that a restarted inner solve discards.
"""
from __future__ import annotations

import numpy as np

from .geometry import G_PAIRS, tensor_apply, tensor_apply_t
from .operators import STIFF, Discretization
from .pcg import pcg


def apply_stiff_f32(disc: Discretization, u32: np.ndarray) -> np.ndarray:
    """Masked stiffness apply with every operand in float32."""
    r = disc.rule
    q, p1 = r.q, r.p1
    J, D = r.J.astype(np.float32), r.D.astype(np.float32)
    G = disc.G_effective().astype(np.float32).reshape(disc.E, 6, q, q, q)
    m = disc.mask.astype(np.float32)
    uL = (u32 * m)[disc.elem_dofs].reshape(disc.E, p1, p1, p1)
    grads = [tensor_apply(J, J, D, uL), tensor_apply(J, D, J, uL),
             tensor_apply(D, J, J, uL)]
    comp = {}
    for n, (a, b) in enumerate(G_PAIRS):
        comp[(a, b)] = comp[(b, a)] = G[:, n]
    v = [sum(comp[(a, b)] * grads[b] for b in range(3)) for a in range(3)]
    wL = (tensor_apply_t(J, J, D, v[0]) + tensor_apply_t(J, D, J, v[1])
          + tensor_apply_t(D, J, J, v[2]))
    w = np.zeros(disc.nglobal, dtype=np.float32)
    np.add.at(w, disc.elem_dofs.reshape(-1), wL.reshape(-1).astype(np.float32))
    return w * m


def pcg_f32(disc: Discretization, b32, dinv32, rtol, maxit):
    """Jacobi-PCG with float32 vectors/apply and float64 dot products."""
    dot = lambda a, c: float(np.dot(a.astype(np.float64), c.astype(np.float64)))
    x = np.zeros_like(b32)
    r = b32.copy()
    z = dinv32 * r
    p = z.copy()
    rz = dot(r, z)
    bn = np.sqrt(dot(b32, b32)) or 1.0
    it = 0
    while it < maxit and np.sqrt(dot(r, r)) > rtol * bn:
        w = apply_stiff_f32(disc, p)
        pw = dot(p, w)
        alpha = rz / pw if pw != 0 else 0.0
        x = x + np.float32(alpha) * p
        r = r - np.float32(alpha) * w
        z = dinv32 * r
        rz_new = dot(r, z)
        beta = rz_new / rz if rz != 0 else 0.0
        p = z + np.float32(beta) * p
        rz = rz_new
        it += 1
    return x, it


def defect_correction(disc: Discretization, b, outer_rtol=1e-10, inner_rtol=1e-5,
                      max_outer=30, max_inner=1000):
    """Returns (x, info) with info = dict(outer, inner_iters list, rel_res list)."""
    b = np.asarray(b, dtype=np.float64)
    dinv32 = disc.jacobi_inverse(STIFF).astype(np.float32)
    x = np.zeros_like(b)
    bn = np.linalg.norm(b) or 1.0
    rel, inner = [], []
    for _ in range(max_outer + 1):
        r = b - disc.apply(STIFF, x)
        rel.append(float(np.linalg.norm(r) / bn))
        if rel[-1] <= outer_rtol or len(inner) == max_outer:
            break
        d, k = pcg_f32(disc, r.astype(np.float32), dinv32, inner_rtol, max_inner)
        inner.append(k)
        x = x + d.astype(np.float64)
    return x, {"outer": len(inner), "inner_iters": inner, "rel_res": rel}


def reliable_cg(disc: Discretization, b, rtol=1e-10, delta=1e-2, max_updates=100,
                max_iters=100000):
    """Returns (x, info) with info = dict(iters, updates, rel_res list)."""
    dot = lambda a, c: float(np.dot(a.astype(np.float64), c.astype(np.float64)))
    b = np.asarray(b, dtype=np.float64)
    dinv32 = disc.jacobi_inverse(STIFF).astype(np.float32)
    x = np.zeros_like(b)
    bn = np.linalg.norm(b) or 1.0
    r64 = b - disc.apply(STIFF, x)
    rel = [float(np.linalg.norm(r64) / bn)]
    r = r64.astype(np.float32)
    x32 = np.zeros_like(r)
    z = dinv32 * r
    p = z.copy()
    rz = dot(r, z)
    ref = dot(r, r)
    it = updates = 0
    while rel[-1] > rtol and it < max_iters and updates < max_updates:
        w = apply_stiff_f32(disc, p)
        pw = dot(p, w)
        alpha = rz / pw if pw != 0 else 0.0
        x32 = x32 + np.float32(alpha) * p
        r = r - np.float32(alpha) * w
        z = dinv32 * r
        rz_new = dot(r, z)
        it += 1
        if dot(r, r) <= delta * delta * ref or it == max_iters:
            # reliable update: FP64 solution and true residual; p is kept
            x = x + x32.astype(np.float64)
            x32[:] = 0
            r64 = b - disc.apply(STIFF, x)
            rel.append(float(np.linalg.norm(r64) / bn))
            updates += 1
            r = r64.astype(np.float32)
            z = dinv32 * r
            rz_new = dot(r, z)
            ref = dot(r, r)
            if rel[-1] <= rtol:
                break
        beta = rz_new / rz if rz != 0 else 0.0
        p = z + np.float32(beta) * p
        rz = rz_new
    return x, {"iters": it, "updates": updates, "rel_res": rel}


def solve_fp64(disc: Discretization, b, rtol):
    """Reference FP64 Jacobi-PCG to the same tolerance."""
    dinv = disc.jacobi_inverse(STIFF)
    return pcg(lambda v: disc.apply(STIFF, v), b, dinv, rtol=rtol, maxit=100000)
