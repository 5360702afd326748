"""Jacobi-preconditioned conjugate gradients (oracle).

Section 3: each BP is CG on the assembled BK system with a diagonal (Jacobi)
preconditioner; section 2: timings cover a fixed number of iterations (100).
The paper prints no CG listing. This is the textbook Hestenes-Stiefel form
that the Nek5000 ax routine of Appendix A1 serves (it returns w = A p and
rho = p.w): x0 = 0, r = b, z = D^-1 r, p = z, then per iteration
  w = A p; alpha = (r.z)/(p.w); x += alpha p; r -= alpha w;
  z = D^-1 r; beta = (r.z)_new/(r.z); p = z + beta p.
Readings where the paper is silent: a zero (r.z) or (p.w) gives
alpha = beta = 0 so a fixed-iteration run keeps its work constant; the
stopping test is ||r||_2 / ||b||_2 <= rtol on the unpreconditioned residual;
with several components each has its own scalars.
"""
from __future__ import annotations

import numpy as np


def _dot(a, b):
    return np.sum(a * b, axis=0)


def _safe_div(num, den):
    num = np.asarray(num, dtype=np.float64)
    den = np.asarray(den, dtype=np.float64)
    out = np.zeros(np.broadcast(num, den).shape)
    return np.divide(num, den, out=out, where=den != 0)


def pcg(apply_A, b, dinv, x0=None, rtol=0.0, maxit=100, fixed_iters=False,
        record=None):
    """Solve A x = b. Returns (x, info) with info = dict(iters, rel_res list).

    apply_A: callable on arrays shaped like b. dinv: [n] inverse diagonal.
    record: optional list; the iterate x after each iteration is appended.
    """
    b = np.asarray(b, dtype=np.float64)
    d = dinv.reshape((-1,) + (1,) * (b.ndim - 1))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_A(x) if x0 is not None else b.copy()
    z = d * r
    p = z.copy()
    rz = _dot(r, z)
    bnorm = np.sqrt(_dot(b, b))
    bnorm = np.where(bnorm == 0, 1.0, bnorm)
    rel = [float(np.max(np.sqrt(_dot(r, r)) / bnorm))]
    it = 0
    while it < maxit:
        if not fixed_iters and rel[-1] <= rtol:
            break
        w = apply_A(p)
        pw = _dot(p, w)
        alpha = _safe_div(rz, pw)
        x = x + alpha * p
        r = r - alpha * w
        z = d * r
        rz_new = _dot(r, z)
        beta = _safe_div(rz_new, rz)
        p = z + beta * p
        rz = rz_new
        it += 1
        rel.append(float(np.max(np.sqrt(_dot(r, r)) / bnorm)))
        if record is not None:
            record.append(x.copy())
    return x, {"iters": it, "rel_res": rel}


def pcg_single_reduction(apply_A, b, dinv, x0=None, rtol=0.0, maxit=100, fixed_iters=False,
                         record=None):
    """Jacobi-PCG with one reduction phase per iteration (Chronopoulos-Gear
    recurrences): the same iterates as pcg in exact arithmetic. With u = D^-1 r
    and w = A u it carries s = A p by recurrence, so that gamma = (r, u) and
    delta = (u, w) come from the same pass:
        p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s, u = D^-1 r,
        w = A u, gamma' = (r, u), delta = (u, w), beta = gamma'/gamma,
        alpha = gamma' / (delta - beta gamma' / alpha).
    Arguments and return value as pcg."""
    b = np.asarray(b, dtype=np.float64)
    d = dinv.reshape((-1,) + (1,) * (b.ndim - 1))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_A(x) if x0 is not None else b.copy()
    u = d * r
    w = apply_A(u)
    gamma = _dot(r, u)
    delta = _dot(u, w)
    alpha = _safe_div(gamma, delta)
    beta = np.zeros_like(gamma)
    p = np.zeros_like(b)
    s = np.zeros_like(b)
    bnorm = np.sqrt(_dot(b, b))
    bnorm = np.where(bnorm == 0, 1.0, bnorm)
    rel = [float(np.max(np.sqrt(_dot(r, r)) / bnorm))]
    it = 0
    while it < maxit:
        if not fixed_iters and rel[-1] <= rtol:
            break
        p = u + beta * p
        s = w + beta * s
        x = x + alpha * p
        r = r - alpha * s
        u = d * r
        w = apply_A(u)
        gamma_new = _dot(r, u)
        delta = _dot(u, w)
        beta = _safe_div(gamma_new, gamma)
        alpha = _safe_div(gamma_new, delta - beta * _safe_div(gamma_new, alpha))
        gamma = gamma_new
        it += 1
        rel.append(float(np.max(np.sqrt(_dot(r, r)) / bnorm)))
        if record is not None:
            record.append(x.copy())
    return x, {"iters": it, "rel_res": rel}
