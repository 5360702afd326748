"""Brute-force assembled matrices for tiny meshes (oracle).

Section 4: A = Q^T A_L Q with A_L = blockdiag(A^e). Each element matrix is
formed explicitly from Kronecker products of the 1D matrices (section 5:
D1 = J^(x)J^(x)D^, D2 = J^(x)D^(x)J^, D3 = D^(x)J^(x)J^, J = J^(x)J^(x)J^),
A^e = sum_mm' D_m^T diag(G_mm') D_m', B^e = J^T diag(B~) J and, for the Helmholtz
operator of eq. (hm2), A^e + J^T diag(beta B~) J, then summed
into a scipy.sparse matrix. This path shares nothing with the sum-factorised
one in operators.py except the geometric factors.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .geometry import G_PAIRS
from .operators import HELM, MASS, STIFF, Discretization


def kron_derivatives(rule):
    J, D = rule.J, rule.D
    D1 = np.kron(J, np.kron(J, D))
    D2 = np.kron(J, np.kron(D, J))
    D3 = np.kron(D, np.kron(J, J))
    Jf = np.kron(J, np.kron(J, J))
    return (D1, D2, D3), Jf


def element_matrices(disc: Discretization, which: int, G=None) -> np.ndarray:
    """Dense element matrices [E, p1^3, p1^3]."""
    (D1, D2, D3), Jf = kron_derivatives(disc.rule)
    Ds = (D1, D2, D3)
    n = disc.rule.p1 ** 3
    out = np.zeros((disc.E, n, n))
    if which in (MASS, HELM):
        Bt = disc.Bt if which == MASS else disc.beta * disc.Bt
        for e in range(disc.E):
            out[e] = Jf.T @ (Bt[e][:, None] * Jf)
        if which == MASS:
            return out
    G = disc.G_effective() if G is None else G
    for e in range(disc.E):
        for c, (m, mp) in enumerate(G_PAIRS):
            blk = Ds[m].T @ (G[e, c][:, None] * Ds[mp])
            out[e] += blk if m == mp else blk + blk.T
    return out


def assemble(disc: Discretization, which: int, masked: bool = True, G=None):
    """Assembled sparse matrix Q^T A_L Q (optionally P (.) P with P = mask)."""
    Ae = element_matrices(disc, which, G)
    n = disc.rule.p1 ** 3
    rows = np.repeat(disc.elem_dofs, n, axis=1).reshape(-1)
    cols = np.tile(disc.elem_dofs, (1, n)).reshape(-1)
    A = sp.coo_matrix((Ae.reshape(-1), (rows, cols)),
                      shape=(disc.nglobal, disc.nglobal)).tocsr()
    if masked:
        P = sp.diags(disc.mask)
        A = (P @ A @ P).tocsr()
    return A


def d_stiffness_d_kappa(disc: Discretization, e: int, qpt: int) -> np.ndarray:
    """Element matrix of dA/dkappa_q for quadrature point qpt of element e."""
    (D1, D2, D3), _ = kron_derivatives(disc.rule)
    Ds = (D1, D2, D3)
    n = disc.rule.p1 ** 3
    out = np.zeros((n, n))
    for c, (m, mp) in enumerate(G_PAIRS):
        g = disc.G[e, c, qpt]
        blk = np.outer(Ds[m][qpt], Ds[mp][qpt]) * g
        out += blk if m == mp else blk + blk.T
    return out
