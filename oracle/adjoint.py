"""Variable-coefficient Poisson solve and its adjoint gradient (oracle).

Section 4, eq. (hm1)-(ip1): a(v,u) = int mu grad v . grad u with a variable
coefficient mu (called kappa here), sampled at the quadrature points, so the
element operator is eq. (bk5x) with G_q replaced by kappa_q G_q.
The adjoint is not in the paper. For A(kappa) u = b (masked, SPD) and the loss
L = 1/2 sum_batch (u - u_t)^T M (u - u_t):
  A lambda = M (u - u_t)     (A is symmetric, so the adjoint uses A itself)
  dL/dkappa_q = - sum_batch (D lambda)_q^T G_q (D u)_q   (= -w_q Jac_q grad lambda . grad u)
  dL/db = lambda.
"""
from __future__ import annotations

import numpy as np

from .geometry import G_PAIRS, tensor_apply
from .operators import MASS, STIFF, Discretization
from .pcg import pcg


def solve(disc: Discretization, b, rtol=1e-13, maxit=100000, x0=None):
    dinv = disc.jacobi_inverse(STIFF)
    x, info = pcg(lambda v: disc.apply(STIFF, v), b, dinv, x0=x0, rtol=rtol, maxit=maxit)
    return x, info


def loss(disc: Discretization, u, u_target):
    d = np.asarray(u) - np.asarray(u_target)
    return 0.5 * float(np.sum(d * disc.apply(MASS, d, masked=False)))


def loss_grad_u(disc: Discretization, u, u_target):
    return disc.apply(MASS, np.asarray(u) - np.asarray(u_target), masked=False)


def grad_kappa(disc: Discretization, lam, u) -> np.ndarray:
    """-sum_batch (D lam)_q^T G_q (D u)_q, [E, q^3]; lam, u masked vectors."""
    r = disc.rule
    q = r.q
    J, D = r.J, r.D
    m = disc.mask.reshape((-1,) + (1,) * (np.ndim(u) - 1))
    lL = disc.gather(np.asarray(lam) * m)
    uL = disc.gather(np.asarray(u) * m)
    gl = [tensor_apply(J, J, D, lL), tensor_apply(J, D, J, lL), tensor_apply(D, J, J, lL)]
    gu = [tensor_apply(J, J, D, uL), tensor_apply(J, D, J, uL), tensor_apply(D, J, J, uL)]
    extra = np.ndim(u) - 1
    G = disc.G.reshape((disc.E, 6, q, q, q) + (1,) * extra)
    out = np.zeros((disc.E, q, q, q) + np.shape(u)[1:])
    for n, (a, b) in enumerate(G_PAIRS):
        t = gl[a] * gu[b]
        if a != b:
            t = t + gl[b] * gu[a]
        out += G[:, n] * t
    out = -out
    if extra:
        out = out.sum(axis=tuple(range(4, 4 + extra)))
    return out.reshape(disc.E, q ** 3)


def loss_and_grad(disc: Discretization, b, u_target, rtol=1e-13):
    """Forward solve, loss, adjoint solve and gradients (kappa, b)."""
    u, _ = solve(disc, b, rtol)
    L = loss(disc, u, u_target)
    g_u = loss_grad_u(disc, u, u_target) * disc.mask.reshape((-1,) + (1,) * (np.ndim(u) - 1))
    lam, _ = solve(disc, g_u, rtol)
    return L, grad_kappa(disc, lam, u), lam, u
