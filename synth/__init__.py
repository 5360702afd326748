"""Seeded synthetic inputs for the bake-off problems (BP1-BP6).

This module only makes input data: element grids, perturbed brick meshes, the
global numbering of nodes, Dirichlet flags, random right-hand sides and the
smooth fields used as manufactured solutions or coefficients. It holds none of
the discretisation's arithmetic: no quadrature, no basis, no operator. Where a
mesh needs the positions of the nodes inside the reference element, the
caller passes them in (each side of a comparison uses its own rule).

Both the CPU oracle and the GPU path draw their inputs from here, so both see
bit-identical meshes and right-hand sides for a given seed.

Conventions (paper section 4, eq. (xijk)/(uijk)): a node of element e is
(i, j, k) with i the fastest index, local id l = i + p1*(j + p1*k); elements
are numbered lexicographically (x fastest); global nodes are numbered
lexicographically on the (p*Ex+1) x (p*Ey+1) x (p*Ez+1) lattice.
scramble_mesh turns such a mesh into one with an arbitrary map: random global
ids, element order and element orientations (the 24 proper cube symmetries).
"""
from .mesh import (element_grid, BrickMesh, brick_mesh, element_coordinates,
                   vertex_perturbation, trilinear_nodes, cube_rotations,
                   rotated_local_ids, scramble_mesh)
from .fields import (rhs_uniform, manufactured_u, manufactured_f, kappa_log,
                     fd_direction)

__all__ = ["element_grid", "BrickMesh", "brick_mesh", "element_coordinates",
           "vertex_perturbation",
           "trilinear_nodes", "cube_rotations", "rotated_local_ids", "scramble_mesh",
           "rhs_uniform", "manufactured_u", "manufactured_f",
           "kappa_log", "fd_direction"]
