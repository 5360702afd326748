"""Builders shared by the oracle tests (CPU only)."""
import numpy as np

import synth
from oracle.operators import Discretization
from oracle.quadrature import Rule, bp_rule


def make_disc(bp, p, ex, ey, ez, seed=0, dirichlet=None, kappa=None, rule=None, beta=None):
    """Discretization of BPj on a (perturbed unless seed is None) brick."""
    rule = rule or bp_rule(bp, p)
    mesh = synth.brick_mesh(ex, ey, ez, p, rule.xi, seed)
    if dirichlet is None:
        dirichlet = bp >= 3
    dir_flags = mesh.boundary if dirichlet else None
    disc = Discretization(rule, mesh.elem_dofs, mesh.node_xyz, mesh.nglobal,
                          dir_flags, kappa, beta)
    return disc, mesh


def custom_disc(p, q, quad, ex, ey, ez, seed=0, dirichlet=False, beta=None):
    return make_disc(None, p, ex, ey, ez, seed, dirichlet, rule=Rule(p, q, quad), beta=beta)


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
