"""Perturbed brick meshes of trilinear hexahedra (input data only).

The bake-off meshes are tensor arrays of E = 2^k elements whose per-direction
counts differ by at most a factor of two, with curvilinear (isoparametric)
elements that may not be treated as a tensor grid by the solver (paper
section 3). Here the domain is [0,1]^3, the element vertices are moved by a
seeded smooth map that vanishes on the boundary, and every element is the
trilinear image of the reference cube through its 8 moved vertices.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def element_grid(k: int) -> tuple[int, int, int]:
    """Element counts (Ex, Ey, Ez) for E = 2^k with counts within a factor 2.

    k = 3m -> (2^m)^3; k = 3m+1 -> (2^(m+1), 2^m, 2^m);
    k = 3m+2 -> (2^(m+1), 2^(m+1), 2^m).
    """
    if k < 0:
        raise ValueError("k must be >= 0")
    m, r = divmod(k, 3)
    ex = 2 ** (m + (1 if r >= 1 else 0))
    ey = 2 ** (m + (1 if r >= 2 else 0))
    ez = 2 ** m
    return ex, ey, ez


def vertex_perturbation(xyz: np.ndarray, h: float, seed: int,
                        amplitude: float = 0.1) -> np.ndarray:
    """Displacement of points xyz [..., 3] by the seeded smooth map.

    d_c(x) = amplitude * h * s(x) * sin(2 pi k_c . x + phi_c), c = 0, 1, 2,
    with s(x) = sin(pi x) sin(pi y) sin(pi z), which is zero on the boundary
    of [0,1]^3, k_c drawn from {1,2}^3 and phi_c from [0, 2 pi) by PCG64(seed).
    """
    rng = np.random.default_rng(seed)
    kvec = rng.integers(1, 3, size=(3, 3))          # row c: wave vector of d_c
    phase = rng.uniform(0.0, 2.0 * np.pi, size=3)
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    s = np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
    out = np.empty_like(xyz)
    for c in range(3):
        arg = 2.0 * np.pi * (kvec[c, 0] * x + kvec[c, 1] * y + kvec[c, 2] * z) + phase[c]
        out[..., c] = amplitude * h * s * np.sin(arg)
    return out


def trilinear_nodes(corners: np.ndarray, ref_nodes: np.ndarray) -> np.ndarray:
    """Images of the reference node lattice under trilinear maps.

    corners: [E, 2, 2, 2, 3] vertex coordinates indexed [e, c_z, c_y, c_x, :].
    ref_nodes: [p1] positions in [-1, 1] of the nodes along each direction.
    Returns [E, p1^3, 3] with local id l = i + p1*(j + p1*k).
    """
    xi = np.asarray(ref_nodes, dtype=np.float64)
    p1 = xi.size
    lin = np.stack([(1.0 - xi) * 0.5, (1.0 + xi) * 0.5], axis=1)   # [p1, 2]
    # weight of corner (cz, cy, cx) at node (k, j, i)
    w = np.einsum("kc,jb,ia->kjicba", lin, lin, lin).reshape(p1 ** 3, 8)
    flat = corners.reshape(corners.shape[0], 8, 3)
    return np.matmul(w[None, :, :], flat)


@dataclass
class BrickMesh:
    """A conforming hexahedral mesh with a global node numbering.

    elem_dofs: int64 [E, p1^3], global id of each element-local node.
    node_xyz:  float64 [E, p1^3, 3], coordinates of each element-local node.
    boundary:  uint8 [nglobal], 1 on nodes of the domain boundary.
    """
    ex: int
    ey: int
    ez: int
    p: int
    elem_dofs: np.ndarray
    node_xyz: np.ndarray
    boundary: np.ndarray
    nglobal: int

    @property
    def nelem(self) -> int:
        return self.ex * self.ey * self.ez

    @property
    def p1(self) -> int:
        return self.p + 1

    def global_coords(self) -> np.ndarray:
        """Coordinates [nglobal, 3] of the global nodes (one copy per node)."""
        out = np.empty((self.nglobal, 3))
        out[self.elem_dofs.reshape(-1)] = self.node_xyz.reshape(-1, 3)
        return out


def _grid_vertices(ex, ey, ez, seed, amplitude):
    gx = np.linspace(0.0, 1.0, ex + 1)
    gy = np.linspace(0.0, 1.0, ey + 1)
    gz = np.linspace(0.0, 1.0, ez + 1)
    Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
    verts = np.stack([X, Y, Z], axis=-1)                 # [ez+1, ey+1, ex+1, 3]
    if seed is not None:
        h = 1.0 / max(ex, ey, ez)
        verts = verts + vertex_perturbation(verts, h, seed, amplitude)
    return verts


def _element_nodes(verts, ex, ey, elems, ref_nodes):
    ix, iy, iz = elems % ex, (elems // ex) % ey, elems // (ex * ey)
    corners = np.empty((elems.size, 2, 2, 2, 3))
    for cz in range(2):
        for cy in range(2):
            for cx in range(2):
                corners[:, cz, cy, cx] = verts[iz + cz, iy + cy, ix + cx]
    return trilinear_nodes(corners, ref_nodes)


def element_coordinates(ex: int, ey: int, ez: int, p: int, ref_nodes: np.ndarray,
                        elements: np.ndarray, seed: int | None = 0,
                        amplitude: float = 0.1) -> np.ndarray:
    """node_xyz [len(elements), p1^3, 3] of the listed elements of brick_mesh."""
    ref_nodes = np.asarray(ref_nodes, dtype=np.float64)
    if ref_nodes.shape != (p + 1,):
        raise ValueError("ref_nodes must hold p+1 positions")
    verts = _grid_vertices(ex, ey, ez, seed, amplitude)
    return _element_nodes(verts, ex, ey, np.asarray(elements, dtype=np.int64), ref_nodes)


def brick_mesh(ex: int, ey: int, ez: int, p: int, ref_nodes: np.ndarray,
               seed: int | None = 0, amplitude: float = 0.1,
               chunk: int = 16384) -> BrickMesh:
    """Perturbed brick mesh on [0,1]^3 with Ex x Ey x Ez elements of order p.

    seed=None leaves the vertices unperturbed (an affine brick).
    """
    if p < 1:
        raise ValueError("p must be >= 1")
    p1 = p + 1
    ref_nodes = np.asarray(ref_nodes, dtype=np.float64)
    if ref_nodes.shape != (p1,):
        raise ValueError("ref_nodes must hold p+1 positions")
    nx, ny, nz = p * ex + 1, p * ey + 1, p * ez + 1
    nglobal = nx * ny * nz
    E = ex * ey * ez

    verts = _grid_vertices(ex, ey, ez, seed, amplitude)

    # global numbering: base of element + offset of local node
    e = np.arange(E, dtype=np.int64)
    exi, eyi, ezi = e % ex, (e // ex) % ey, e // (ex * ey)
    base = p * exi + nx * (p * eyi) + nx * ny * (p * ezi)
    l = np.arange(p1 ** 3, dtype=np.int64)
    li, lj, lk = l % p1, (l // p1) % p1, l // (p1 * p1)
    off = li + nx * lj + nx * ny * lk
    elem_dofs = base[:, None] + off[None, :]

    node_xyz = np.empty((E, p1 ** 3, 3))
    for s in range(0, E, chunk):
        node_xyz[s:s + chunk] = _element_nodes(verts, ex, ey, e[s:s + chunk], ref_nodes)

    I = np.arange(nglobal, dtype=np.int64)
    gi, gj, gk = I % nx, (I // nx) % ny, I // (nx * ny)
    boundary = ((gi == 0) | (gi == nx - 1) | (gj == 0) | (gj == ny - 1)
                | (gk == 0) | (gk == nz - 1)).astype(np.uint8)
    return BrickMesh(ex, ey, ez, p, elem_dofs, node_xyz, boundary, nglobal)


def cube_rotations() -> list[tuple[tuple[int, int, int], tuple[int, int, int]]]:
    """The 24 proper symmetries of the reference cube [-1,1]^3.

    Each is (perm, sign): new reference coordinate d is sign[d] times old
    coordinate perm[d]. The signed permutation matrix has determinant +1, so
    composing an element's map with it keeps the Jacobian positive.
    """
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        inv = sum(1 for a in range(3) for b in range(a + 1, 3) if perm[a] > perm[b])
        for sign in itertools.product((1, -1), repeat=3):
            if (-1) ** inv * sign[0] * sign[1] * sign[2] == 1:
                out.append((perm, sign))
    return out


def rotated_local_ids(p1: int, perm, sign) -> np.ndarray:
    """old[l'] = the old local id of new local node l' under a cube rotation.

    New node (i'_0, i'_1, i'_2) sits where old index i_d = i'_perm[d] if
    sign[d] > 0 and p - i'_perm[d] otherwise (the node lattice is symmetric
    about the cube's centre, so a rotation maps nodes onto nodes).
    """
    l = np.arange(p1 ** 3, dtype=np.int64)
    new = np.stack([l % p1, (l // p1) % p1, l // (p1 * p1)])     # new[d] = i'_d
    old = np.empty_like(new)
    for d in range(3):
        src = new[perm[d]]
        old[d] = src if sign[d] > 0 else (p1 - 1) - src
    return old[0] + p1 * (old[1] + p1 * old[2])


def scramble_mesh(mesh: BrickMesh, seed: int) -> BrickMesh:
    """The same mesh with an arbitrary gather map (input data only).

    Global ids are renumbered by a seeded random permutation, the elements
    are listed in a random order, and the local axes of every element are
    turned by a random proper cube symmetry (its node list re-indexed, its
    geometry unchanged). The discrete operator is then P A P^T for the
    renumbering P: nothing of the tensor-grid numbering is left for a solver
    to rely on.
    """
    rng = np.random.default_rng(seed)
    p1 = mesh.p1
    E = mesh.elem_dofs.shape[0]
    newid = rng.permutation(mesh.nglobal).astype(np.int64)      # old id -> new id
    order = rng.permutation(E)                                   # new element -> old
    rots = cube_rotations()
    tables = np.stack([rotated_local_ids(p1, *r) for r in rots])  # [24, p1^3]
    which = rng.integers(0, len(rots), size=E)
    loc = tables[which]                                          # [E, p1^3] old local id
    src = order[:, None]
    elem_dofs = newid[mesh.elem_dofs[src, loc]]
    node_xyz = mesh.node_xyz[src, loc]
    boundary = np.empty_like(mesh.boundary)
    boundary[newid] = mesh.boundary
    return BrickMesh(mesh.ex, mesh.ey, mesh.ez, mesh.p, elem_dofs, node_xyz, boundary,
                     mesh.nglobal)
