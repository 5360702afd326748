"""Quadrature rules and 1D Lagrange matrices (oracle).

Paper section 3 (Table "bps"): nodal points are the p+1 Gauss-Lobatto-Legendre
(GLL) points; quadrature uses q = p+2 Gauss-Legendre (GL) points for BP1-BP4
and the q = p+1 GLL points for BP5-BP6. Section 5, eq. (bk5x): J^ and D^ are
the q x p1 matrices that interpolate and differentiate the Lagrange basis on
the GLL nodes at the quadrature points; for collocated GLL quadrature J^ = I.

The paper does not say how the points are found. Here: Newton iteration on
the Legendre three-term recurrence from Chebyshev starting guesses.
"""
from __future__ import annotations

import numpy as np


def legendre(n: int, x: np.ndarray):
    """P_n(x) and P_n'(x) by the three-term recurrence.

    (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1};
    P'_{k+1} = (k+1) P_k + x P'_k.
    """
    x = np.asarray(x, dtype=np.float64)
    p_prev, p_cur = np.ones_like(x), x.copy()
    d_prev, d_cur = np.zeros_like(x), np.ones_like(x)
    if n == 0:
        return p_prev, d_prev
    for k in range(1, n):
        p_next = ((2 * k + 1) * x * p_cur - k * p_prev) / (k + 1)
        d_next = (k + 1) * p_cur + x * d_cur
        p_prev, p_cur = p_cur, p_next
        d_prev, d_cur = d_cur, d_next
    return p_cur, d_cur


def gauss_legendre(q: int):
    """q-point Gauss-Legendre rule: roots of P_q, weights 2/((1-x^2) P_q'^2)."""
    if q < 1:
        raise ValueError("q >= 1 required")
    j = np.arange(q)
    x = -np.cos(np.pi * (j + 0.75) / (q + 0.5))
    for _ in range(100):
        P, dP = legendre(q, x)
        dx = P / dP
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    _, dP = legendre(q, x)
    w = 2.0 / ((1.0 - x * x) * dP * dP)
    return x, w


def gauss_lobatto_legendre(p1: int):
    """p1-point GLL rule: +-1 and the roots of P_p', weights 2/(p(p+1) P_p^2)."""
    if p1 < 2:
        raise ValueError("GLL needs at least 2 points")
    p = p1 - 1
    x = -np.cos(np.pi * np.arange(p1) / p)
    interior = x[1:-1].copy()
    for _ in range(100):
        if interior.size == 0:
            break
        P, dP = legendre(p, interior)
        # Legendre ODE: (1-x^2) P'' = 2x P' - p(p+1) P
        d2P = (2.0 * interior * dP - p * (p + 1) * P) / (1.0 - interior ** 2)
        dx = dP / d2P
        interior = interior - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    x = np.concatenate([[-1.0], interior, [1.0]])
    P, _ = legendre(p, x)
    w = 2.0 / (p * (p + 1) * P * P)
    return x, w


def lagrange_matrix(nodes: np.ndarray, points: np.ndarray) -> np.ndarray:
    """J[a, j] = h_j(points[a]), h_j the Lagrange polynomial on `nodes`.

    Plain product definition: h_j(x) = prod_{m != j} (x - x_m) / (x_j - x_m).
    """
    n = len(nodes)
    out = np.ones((len(points), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                out[:, j] *= (points - nodes[m]) / (nodes[j] - nodes[m])
    return out


def lagrange_deriv_matrix(nodes: np.ndarray, points: np.ndarray) -> np.ndarray:
    """D[a, j] = h_j'(points[a]).

    Product rule: h_j'(x) = sum_{l != j} 1/(x_j - x_l) prod_{m != j,l} (x - x_m)/(x_j - x_m).
    """
    n = len(nodes)
    out = np.zeros((len(points), n))
    for j in range(n):
        for l in range(n):
            if l == j:
                continue
            term = np.full(len(points), 1.0 / (nodes[j] - nodes[l]))
            for m in range(n):
                if m != j and m != l:
                    term *= (points - nodes[m]) / (nodes[j] - nodes[m])
            out[:, j] += term
    return out


class Rule:
    """Nodes, quadrature and 1D matrices for order p with q points.

    quad = "gll" (collocated, q must equal p+1) or "gl".
    Attributes: xi (p1 GLL nodes), eta, rho (q quadrature points/weights),
    J (q x p1 interpolation), D (q x p1 derivative).
    """

    def __init__(self, p: int, q: int, quad: str):
        self.p, self.p1, self.q, self.quad = p, p + 1, q, quad
        self.xi, self.xi_w = gauss_lobatto_legendre(p + 1)
        if quad == "gll":
            self.eta, self.rho = gauss_lobatto_legendre(q)
        elif quad == "gl":
            self.eta, self.rho = gauss_legendre(q)
        else:
            raise ValueError(quad)
        if quad == "gll" and q == p + 1:
            # collocation: interpolation is the identity (section 5)
            self.eta = self.xi
            self.J = np.eye(q)
        else:
            self.J = lagrange_matrix(self.xi, self.eta)
        self.D = lagrange_deriv_matrix(self.xi, self.eta)


def bp_rule(bp: int, p: int) -> Rule:
    """The rule Table "bps" assigns to BPj: GL q=p+2 for BP1-4, GLL q=p+1 for BP5-6."""
    if bp in (1, 2, 3, 4):
        return Rule(p, p + 2, "gl")
    if bp in (5, 6):
        return Rule(p, p + 1, "gll")
    raise ValueError(bp)
