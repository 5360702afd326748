"""Isoparametric geometry and geometric factors (oracle).

Section 4, eq. (xijk): x^e(r,s,t) = sum_ijk x^e_ijk h_i(r) h_j(s) h_k(t).
Section 5, eq. (gij): [G_mm']_abc = sum_l (dr_m/dx_l)(dr_m'/dx_l) Jac rho_a rho_b rho_c,
stored as the 6 symmetric components in the order 11, 12, 13, 22, 23, 33.
Section 5, eq. (mass): B~ = diag(rho_a rho_b rho_c Jac).

Local node arrays are [E, p1, p1, p1] indexed [e, k, j, i] (i fastest in the
flat id); quadrature arrays are [E, q, q, q] indexed [e, c, b, a] with a the
point along r.
"""
from __future__ import annotations

import numpy as np

from .quadrature import Rule

# order of the 6 stored components of the symmetric G
G_PAIRS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def tensor_apply(Ak, Aj, Ai, u):
    """(Ak (x) Aj (x) Ai) u for u [E, k, j, i, ...] -> [E, c, b, a, ...].

    Section 5, eq. (tens1): sum_k Ak[c,k] sum_j Aj[b,j] sum_i Ai[a,i] u[k,j,i].
    """
    t = np.einsum("ai,ekji...->ekja...", Ai, u)
    t = np.einsum("bj,ekja...->ekba...", Aj, t)
    return np.einsum("ck,ekba...->ecba...", Ak, t)


def tensor_apply_t(Ak, Aj, Ai, v):
    """(Ak (x) Aj (x) Ai)^T v for v [E, c, b, a, ...] -> [E, k, j, i, ...]."""
    t = np.einsum("ck,ecba...->ekba...", Ak, v)
    t = np.einsum("bj,ekba...->ekja...", Aj, t)
    return np.einsum("ai,ekja...->ekji...", Ai, t)


def jacobian(rule: Rule, node_xyz: np.ndarray) -> np.ndarray:
    """dx_l/dr_m at the quadrature points: [E, q, q, q, 3 (l), 3 (m)]."""
    p1 = rule.p1
    E = node_xyz.shape[0]
    X = node_xyz.reshape(E, p1, p1, p1, 3)
    J, D = rule.J, rule.D
    dr = tensor_apply(J, J, D, X)   # derivative along r (index i)
    ds = tensor_apply(J, D, J, X)   # along s (index j)
    dt = tensor_apply(D, J, J, X)   # along t (index k)
    return np.stack([dr, ds, dt], axis=-1)


def quad_weights3(rule: Rule) -> np.ndarray:
    """rho_a rho_b rho_c as [q, q, q] indexed [c, b, a]."""
    r = rule.rho
    return r[:, None, None] * r[None, :, None] * r[None, None, :]


def geometric_factors(rule: Rule, node_xyz: np.ndarray):
    """Return (G [E, 6, q^3], Btilde [E, q^3], Jac [E, q^3]).

    Raises ValueError naming the element if Jac <= 0 at any point.
    """
    E = node_xyz.shape[0]
    q = rule.q
    Jm = jacobian(rule, node_xyz)
    det = np.linalg.det(Jm)
    bad = np.nonzero((det <= 0).reshape(E, -1).any(axis=1))[0]
    if bad.size:
        raise ValueError(f"non-positive Jacobian in element {int(bad[0])}")
    inv = np.linalg.inv(Jm)            # inv[..., m, l] = dr_m/dx_l
    wq = quad_weights3(rule)[None]
    G = np.empty((E, 6, q, q, q))
    for n, (m, mp) in enumerate(G_PAIRS):
        G[:, n] = np.einsum("...l,...l->...", inv[..., m, :], inv[..., mp, :]) * det * wq
    Bt = det * wq
    return G.reshape(E, 6, q ** 3), Bt.reshape(E, q ** 3), det.reshape(E, q ** 3)


def quad_points(rule: Rule, node_xyz: np.ndarray) -> np.ndarray:
    """Physical coordinates of the quadrature points: [E, q^3, 3]."""
    p1 = rule.p1
    E = node_xyz.shape[0]
    X = node_xyz.reshape(E, p1, p1, p1, 3)
    J = rule.J
    return tensor_apply(J, J, J, X).reshape(E, rule.q ** 3, 3)
