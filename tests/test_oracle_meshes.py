"""Pins for the oracle on arbitrary gather maps and for the quadrature-point
coordinates (section 3: elements may not be treated as a tensor grid;
section 4, eq. (dssum): Q is a general Boolean gather; eq. (xijk): the
isoparametric map)."""
import itertools

import numpy as np
import pytest

import synth
from oracle.assembled import assemble
from oracle.geometry import geometric_factors, quad_points
from oracle.operators import MASS, STIFF, Discretization
from oracle.quadrature import Rule, bp_rule
from synth.mesh import cube_rotations, rotated_local_ids, scramble_mesh
from tests.oracle_cases import rel_err


def _disc(rule, mesh, dirichlet):
    return Discretization(rule, mesh.elem_dofs, mesh.node_xyz, mesh.nglobal,
                          mesh.boundary if dirichlet else None)


def test_cube_rotations_are_the_24_proper_symmetries():
    mats = set()
    for perm, sign in cube_rotations():
        R = np.zeros((3, 3), int)
        for d in range(3):
            R[d, perm[d]] = sign[d]
        assert round(np.linalg.det(R)) == 1
        mats.add(R.tobytes())
    assert len(mats) == 24
    # every signed permutation with determinant +1 is among them
    count = 0
    for perm in itertools.permutations(range(3)):
        for sign in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3), int)
            for d in range(3):
                R[d, perm[d]] = sign[d]
            count += round(np.linalg.det(R)) == 1
    assert count == 24


def test_rotated_local_ids_are_permutations_and_identity_is_first_kind():
    for p1 in (2, 3, 5):
        for perm, sign in cube_rotations():
            t = rotated_local_ids(p1, perm, sign)
            assert np.array_equal(np.sort(t), np.arange(p1 ** 3))
        assert np.array_equal(rotated_local_ids(p1, (0, 1, 2), (1, 1, 1)), np.arange(p1 ** 3))


@pytest.mark.parametrize("bp,p", [(1, 2), (1, 4), (3, 1), (3, 3), (5, 2), (5, 4)])
def test_operators_commute_with_renumbering(bp, p):
    # the assembled operator depends on the mesh, not on its numbering:
    # A' = P A P^T for the renumbering P of a scrambled map (random global
    # ids, element order and element orientations)
    rule = bp_rule(bp, p)
    mesh = synth.brick_mesh(3, 2, 2, p, rule.xi, seed=p)
    sm = scramble_mesh(mesh, 100 + p)
    newid = _new_ids(mesh, sm)
    d0, d1 = _disc(rule, mesh, bp >= 3), _disc(rule, sm, bp >= 3)
    u = np.random.default_rng(p).uniform(-1, 1, (mesh.nglobal, 2))
    us = np.empty_like(u)
    us[newid] = u
    for which in (MASS, STIFF):
        for masked in (False, True):
            w0 = d0.apply(which, u, masked=masked)
            w1 = d1.apply(which, us, masked=masked)
            assert rel_err(w1[newid], w0) < 1e-13, (which, masked)
        assert rel_err(d1.diag(which)[newid], d0.diag(which)) < 1e-13


def test_scrambled_operator_equals_kronecker_assembly_on_the_scrambled_map():
    # the sum-factorised gather/scatter against the independent dense path,
    # both on the scrambled map
    for bp, p in [(3, 2), (5, 3)]:
        rule = bp_rule(bp, p)
        sm = scramble_mesh(synth.brick_mesh(2, 2, 2, p, rule.xi, seed=3), 9)
        d = _disc(rule, sm, True)
        u = np.random.default_rng(4).uniform(-1, 1, d.nglobal)
        for which in (MASS, STIFF):
            A = assemble(d, which, masked=True)
            assert rel_err(d.apply(which, u), A @ u) < 1e-13


def test_reflected_element_is_rejected():
    # a reflection (determinant -1) of an element's local axes turns its
    # Jacobian negative: the orientation handling of the scrambler matters
    rule = bp_rule(5, 3)
    mesh = synth.brick_mesh(2, 1, 1, 3, rule.xi, seed=1)
    t = rotated_local_ids(4, (0, 1, 2), (-1, 1, 1))
    xyz = mesh.node_xyz.copy()
    xyz[1] = xyz[1, t]
    with pytest.raises(ValueError, match="element 1"):
        geometric_factors(rule, xyz)


def _new_ids(mesh, sm):
    """old global id -> new global id, recovered from the node coordinates."""
    old = mesh.global_coords()
    new = sm.global_coords()
    key = lambda c: np.round(c * 2 ** 30).astype(np.int64)
    order_old = np.lexsort(key(old).T)
    order_new = np.lexsort(key(new).T)
    assert np.allclose(old[order_old], new[order_new], atol=1e-14)
    newid = np.empty(mesh.nglobal, np.int64)
    newid[order_old] = order_new
    return newid


@pytest.mark.parametrize("p", [2, 5])
def test_quad_points_equal_the_trilinear_map_at_gauss_points(p):
    # the elements are trilinear, so interpolating their GLL nodes to the
    # Gauss points must give the trilinear vertex map evaluated there
    q = p + 2
    rule = Rule(p, q, "gl")
    ex, ey, ez = 3, 2, 2
    mesh = synth.brick_mesh(ex, ey, ez, p, rule.xi, seed=5)
    xq = quad_points(rule, mesh.node_xyz)
    ref = synth.element_coordinates(ex, ey, ez, q - 1, rule.eta,
                                    np.arange(ex * ey * ez), seed=5)
    assert np.max(np.abs(xq - ref)) < 1e-14


@pytest.mark.parametrize("bp,p", [(1, 3), (3, 5)])
def test_quad_points_integrate_coordinates_exactly(bp, p):
    # sum_q rho_q Jac_q x_q = int x dx = 1/2 and int x^2 = 1/3 over [0,1]^3
    # (the perturbed map keeps the boundary fixed); the integrands are
    # polynomials of degree <= 4 per variable, exact with q = p + 2 >= 3
    rule = bp_rule(bp, p)
    mesh = synth.brick_mesh(3, 3, 2, p, rule.xi, seed=6)
    _, Bt, _ = geometric_factors(rule, mesh.node_xyz)
    xq = quad_points(rule, mesh.node_xyz)
    for l in range(3):
        assert abs(np.sum(Bt * xq[..., l]) - 0.5) < 1e-14
        assert abs(np.sum(Bt * xq[..., l] ** 2) - 1.0 / 3.0) < 1e-14
    # a mixed moment: int x y z = 1/8
    assert abs(np.sum(Bt * xq[..., 0] * xq[..., 1] * xq[..., 2]) - 0.125) < 1e-14
