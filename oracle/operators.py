"""Matrix-free mass and stiffness operators (oracle).

Section 4: w = Q^T A_L Q u, with Q the Boolean global-to-local map (gather),
Q^T its transpose (scatter-add) and A_L = blockdiag(A^e).
Section 5, eq. (bk5x): A^e u^e = [D1;D2;D3]^T G^e [D1;D2;D3] u^e with
D1 = J^(x)J^(x)D^, D2 = J^(x)D^(x)J^, D3 = D^(x)J^(x)J^.
Section 5, eq. (mass): B^e u^e = J^T B~^e J u^e, J = J^(x)J^(x)J^.
Section 4, eq. (hm2) with (ip1)-(ip2): the Helmholtz operator H = A + B_beta,
where B_beta is the mass matrix with beta(x) at the quadrature points
(B~ -> beta_q B~); HELM selects it.
Appendix A1 (Nek5000 ax): Dirichlet values are removed by a mask after the
assembly; "masked" here means w = mask * A (mask * u).

Vectors are [nglobal] (one component) or [nglobal, ncomp].
"""
from __future__ import annotations

import numpy as np

from .geometry import G_PAIRS, geometric_factors, tensor_apply, tensor_apply_t
from .quadrature import Rule

MASS, STIFF, HELM = 1, 3, 4


class Discretization:
    """Mesh + rule + precomputed geometric factors (section 3: precomputed).

    elem_dofs [E, p1^3] int, node_xyz [E, p1^3, 3], dirichlet [nglobal] flags
    or None (no Dirichlet nodes). kappa [E, q^3] scales G (variable mu of
    eq. (hm1)); None means 1. beta (a number or [E, q^3] values at the
    quadrature points) is the beta of eq. (hm1) used by HELM; None means 0.
    """

    def __init__(self, rule: Rule, elem_dofs, node_xyz, nglobal: int,
                 dirichlet=None, kappa=None, beta=None):
        self.rule = rule
        self.elem_dofs = np.asarray(elem_dofs, dtype=np.int64)
        self.E = self.elem_dofs.shape[0]
        self.nglobal = int(nglobal)
        self.G, self.Bt, self.jac = geometric_factors(rule, node_xyz)
        if dirichlet is None:
            self.mask = np.ones(self.nglobal)
        else:
            self.mask = 1.0 - np.asarray(dirichlet, dtype=np.float64)
        self.kappa = None if kappa is None else np.asarray(kappa, dtype=np.float64)
        if beta is None:
            self.beta = np.zeros((self.E, rule.q ** 3))
        else:
            self.beta = np.broadcast_to(np.asarray(beta, dtype=np.float64),
                                        (self.E, rule.q ** 3)).copy()

    # -- Q and Q^T --------------------------------------------------------
    def gather(self, u):
        """u_L = Q u: [E, p1, p1, p1, ...] (section 4)."""
        p1 = self.rule.p1
        uL = u[self.elem_dofs]
        return uL.reshape((self.E, p1, p1, p1) + u.shape[1:])

    def scatter(self, wL, ncomp_shape):
        """w = Q^T w_L: sum of local contributions per global node."""
        flat = wL.reshape((self.E * self.rule.p1 ** 3,) + ncomp_shape)
        out = np.zeros((self.nglobal,) + ncomp_shape)
        np.add.at(out, self.elem_dofs.reshape(-1), flat)
        return out

    # -- local operators --------------------------------------------------
    def G_effective(self):
        if self.kappa is None:
            return self.G
        return self.G * self.kappa[:, None, :]

    def stiff_local(self, uL, G=None):
        """w_L = A_L u_L by sum factorisation, eq. (bk5x) and (tens1)."""
        r = self.rule
        q = r.q
        G = self.G_effective() if G is None else G
        J, D = r.J, r.D
        grads = [tensor_apply(J, J, D, uL), tensor_apply(J, D, J, uL),
                 tensor_apply(D, J, J, uL)]
        extra = uL.shape[4:]
        Gq = G.reshape((self.E, 6, q, q, q) + (1,) * len(extra))
        comp = {}
        for n, (m, mp) in enumerate(G_PAIRS):
            comp[(m, mp)] = comp[(mp, m)] = Gq[:, n]
        v = [sum(comp[(m, mp)] * grads[mp] for mp in range(3)) for m in range(3)]
        return (tensor_apply_t(J, J, D, v[0]) + tensor_apply_t(J, D, J, v[1])
                + tensor_apply_t(D, J, J, v[2]))

    def mass_local(self, uL, Bt=None):
        """w_L = B_L u_L = J^T B~ J u_L, eq. (mass) (Bt replaces B~ if given)."""
        r = self.rule
        q = r.q
        J = r.J
        extra = uL.shape[4:]
        Bt = self.Bt if Bt is None else Bt
        Bq = Bt.reshape((self.E, q, q, q) + (1,) * len(extra))
        return tensor_apply_t(J, J, J, Bq * tensor_apply(J, J, J, uL))

    def helm_local(self, uL):
        """w_L = (A_L + B_beta,L) u_L: eq. (hm2), the stiffness of eq. (bk5x)
        plus the mass of eq. (mass) with beta_q B~ at the points."""
        return self.stiff_local(uL) + self.mass_local(uL, self.beta * self.Bt)

    def local(self, which: int, uL):
        if which == STIFF:
            return self.stiff_local(uL)
        if which == MASS:
            return self.mass_local(uL)
        if which == HELM:
            return self.helm_local(uL)
        raise ValueError("which must be MASS, STIFF or HELM")

    # -- assembled operators ----------------------------------------------
    def apply(self, which: int, u, masked: bool = True):
        """w = [mask] Q^T A_L Q [mask] u for which in {MASS, STIFF, HELM}."""
        u = np.asarray(u, dtype=np.float64)
        mshape = (self.nglobal,) + (1,) * (u.ndim - 1)
        m = self.mask.reshape(mshape)
        if masked:
            u = u * m
        uL = self.gather(u)
        wL = self.local(which, uL)
        w = self.scatter(wL, u.shape[1:])
        if masked:
            w = w * m
        return w

    def diag(self, which: int, masked: bool = True):
        """Diagonal of the assembled operator, diag(Q^T A_L Q).

        Stiffness: diagonal entry of sum_mm' D_m^T diag(G_mm') D_m' at node
        (i,j,k) is sum_abc sum_mm' G_mm'(a,b,c) phi_m phi_m', with
        phi_1 = D^[a,i] J^[b,j] J^[c,k], phi_2 = J^[a,i] D^[b,j] J^[c,k],
        phi_3 = J^[a,i] J^[b,j] D^[c,k]. Mass: sum_abc B~ J^[a,i]^2 J^[b,j]^2 J^[c,k]^2.
        Masked: Dirichlet rows are set to 0.
        """
        if which == HELM:
            d = self.diag(STIFF, masked)
            saved, self.Bt = self.Bt, self.beta * self.Bt
            try:
                return d + self.diag(MASS, masked)
            finally:
                self.Bt = saved
        r = self.rule
        q, p1 = r.q, r.p1
        J, D = r.J, r.D
        if which == MASS:
            B = self.Bt.reshape(self.E, q, q, q)
            J2 = J * J
            dL = np.einsum("ecba,ai,bj,ck->ekji", B, J2, J2, J2)
        else:
            G = self.G_effective().reshape(self.E, 6, q, q, q)
            # 1D factor of phi_m along direction d (0: a/i, 1: b/j, 2: c/k)
            fac = lambda m, d: D if m == d else J
            dL = np.zeros((self.E, p1, p1, p1))
            for n, (m, mp) in enumerate(G_PAIRS):
                term = np.einsum("ecba,ai,bj,ck->ekji", G[:, n],
                                 fac(m, 0) * fac(mp, 0), fac(m, 1) * fac(mp, 1),
                                 fac(m, 2) * fac(mp, 2))
                dL += term if m == mp else 2.0 * term
        d = np.zeros(self.nglobal)
        np.add.at(d, self.elem_dofs.reshape(-1), dL.reshape(-1))
        if masked:
            d = d * self.mask
        return d

    def jacobi_inverse(self, which: int, masked: bool = True):
        """1/diag on unmasked nodes, 0 on Dirichlet nodes."""
        d = self.diag(which, masked)
        out = np.zeros_like(d)
        nz = d != 0
        out[nz] = 1.0 / d[nz]
        return out
