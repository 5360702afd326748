"""Selected outputs of the assembled operators on large meshes (oracle).

Section 4: (Q^T A_L Q u)_g sums the element contributions of the elements
that contain node g. For a few sample nodes the oracle therefore needs only
those elements: it renumbers their nodes locally, applies the plain
operators of operators.py to that patch and reads the sample values.
"""
from __future__ import annotations

import numpy as np

from .operators import Discretization


def elements_containing(elem_dofs: np.ndarray, nodes: np.ndarray) -> np.ndarray:
    """Ids of the elements that hold at least one of the given global nodes."""
    return np.nonzero(np.isin(elem_dofs, nodes).any(axis=1))[0]


def apply_at_nodes(rule, elem_dofs_sub, node_xyz_sub, u, nodes, which, masked=True,
                   dirichlet=None, kappa_sub=None):
    """(A u)_g at the sample nodes; the patch must hold every element that
    contains a sample node. u and dirichlet are global arrays."""
    uniq, inv = np.unique(elem_dofs_sub, return_inverse=True)
    local = inv.reshape(elem_dofs_sub.shape)
    dl = None if dirichlet is None else np.asarray(dirichlet)[uniq]
    disc = Discretization(rule, local, node_xyz_sub, uniq.size, dl, kappa_sub)
    w = disc.apply(which, np.asarray(u)[uniq], masked)
    return w[np.searchsorted(uniq, nodes)]
