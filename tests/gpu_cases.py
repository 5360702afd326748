"""Builders for GPU-vs-oracle comparisons: the same seeded mesh, numbering and
right-hand sides on both sides; each side places the element nodes at its
own GLL points."""
import numpy as np

import synth
from oracle.operators import Discretization
from oracle.quadrature import bp_rule as oracle_rule

TOL = 1e-12   # normwise relative FP64 parity bar


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


class Case:
    """Oracle Discretization + library Operator on one seeded mesh."""

    def __init__(self, bp, p, ex, ey, ez, seed=0, ncomp=1, fp32=False, dirichlet=None,
                 scramble=None, caller_order=False):
        import paper_2004_06722_amd.bp as B
        self.bp, self.p, self.ncomp = bp, p, ncomp
        q, quad = B.bp_quadrature(bp, p)
        self.q, self.quad = q, quad
        if dirichlet is None:
            dirichlet = bp >= 3
        # oracle side
        orule = oracle_rule(bp, p)
        om = synth.brick_mesh(ex, ey, ez, p, orule.xi, seed)
        if scramble is not None:
            # arbitrary map: random ids, element order and orientations
            om = synth.scramble_mesh(om, scramble)
        self.mesh = om
        self.dir = om.boundary if dirichlet else None
        self.disc = Discretization(orule, om.elem_dofs, om.node_xyz, om.nglobal, self.dir)
        # library side: nodes at the library's own GLL points
        xi, _ = B.rule(p + 1, B.GLL)
        lm = synth.brick_mesh(ex, ey, ez, p, xi, seed)
        if scramble is not None:
            lm = synth.scramble_mesh(lm, scramble)
        assert np.array_equal(lm.elem_dofs, om.elem_dofs)
        self.op = B.Operator(p, q, quad, lm.elem_dofs, lm.node_xyz, lm.nglobal,
                             self.dir, ncomp=ncomp, fp32=fp32, caller_order=caller_order)

    def vec(self, seed):
        v = synth.rhs_uniform(self.disc.nglobal, seed, ncomp=self.ncomp)
        return v

    def close(self):
        self.op.close()
