"""Pins for the oracle's geometry and operators (sections 4-5, Appendix A1)."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle.assembled import assemble
from oracle.geometry import geometric_factors, quad_weights3
from oracle.operators import HELM, MASS, STIFF
from oracle.quadrature import Rule, bp_rule
from tests.oracle_cases import custom_disc, make_disc, rel_err


def test_geometric_factors_closed_form_on_affine_brick():
    # unperturbed brick, spacings hx, hy, hz: G is diagonal with
    # G11 = rho^3 hy hz / (2 hx) (and cyclic), Jac = hx hy hz / 8
    for bp, p in [(5, 3), (3, 4), (1, 2)]:
        rule = bp_rule(bp, p)
        mesh = synth.brick_mesh(2, 3, 4, p, rule.xi, seed=None)
        G, Bt, jac = geometric_factors(rule, mesh.node_xyz)
        hx, hy, hz = 1 / 2, 1 / 3, 1 / 4
        w3 = quad_weights3(rule).reshape(-1)
        assert np.allclose(jac, hx * hy * hz / 8, rtol=1e-13)
        assert np.allclose(G[:, 0], w3 * hy * hz / (2 * hx), rtol=1e-12)
        assert np.allclose(G[:, 3], w3 * hx * hz / (2 * hy), rtol=1e-12)
        assert np.allclose(G[:, 5], w3 * hx * hy / (2 * hz), rtol=1e-12)
        for c in (1, 2, 4):
            assert np.max(np.abs(G[:, c])) < 1e-13
        assert np.allclose(Bt, w3 * hx * hy * hz / 8, rtol=1e-13)


def _lattice_1d(n, h):
    """1D stiffness (1/h)(-1,2,-1) and lumped / consistent masses on n elements."""
    N = n + 1
    K = sp.diags([-np.ones(N - 1), 2 * np.ones(N), -np.ones(N - 1)], [-1, 0, 1]).tolil()
    K[0, 0] = K[-1, -1] = 1
    Ml = h * np.ones(N)
    Ml[0] = Ml[-1] = h / 2
    Mc = sp.diags([np.ones(N - 1), 4 * np.ones(N), np.ones(N - 1)], [-1, 0, 1]).tolil()
    Mc[0, 0] = Mc[-1, -1] = 2
    return (K.tocsr() / h), sp.diags(Ml), (Mc.tocsr() * h / 6)


def test_p1_gll_stiffness_is_seven_point_laplacian():
    # textbook special case: trapezoid-rule Q1 stiffness on a uniform grid is
    # K(x)M(x)M + M(x)K(x)M + M(x)M(x)K; interior rows are h*(6u - sum nbrs)
    n = 3
    disc, _ = make_disc(5, 1, n, n, n, seed=None, dirichlet=False)
    K, M, _ = _lattice_1d(n, 1.0 / n)
    ref = sp.kron(M, sp.kron(M, K)) + sp.kron(M, sp.kron(K, M)) + sp.kron(K, sp.kron(M, M))
    A = assemble(disc, STIFF, masked=False)
    assert abs(A - ref).max() < 1e-14
    u = np.random.default_rng(1).standard_normal(disc.nglobal)
    assert rel_err(disc.apply(STIFF, u, masked=False), ref @ u) < 1e-14
    # an interior row: 6h on the diagonal, -h to the six neighbours
    N = n + 1
    c = 1 + N * (1 + N * 1)
    row = ref.getrow(c).toarray().ravel()
    assert np.isclose(row[c], 6.0 / n)
    for d in (1, N, N * N):
        assert np.isclose(row[c + d], -1.0 / n) and np.isclose(row[c - d], -1.0 / n)


def test_p1_gl_mass_is_kronecker_consistent_mass():
    n = 2
    disc, _ = make_disc(1, 1, n, n, n, seed=None)
    _, _, Mc = _lattice_1d(n, 1.0 / n)
    ref = sp.kron(Mc, sp.kron(Mc, Mc))
    B = assemble(disc, MASS, masked=False)
    assert abs(B - ref).max() < 1e-15
    u = np.random.default_rng(2).standard_normal(disc.nglobal)
    assert rel_err(disc.apply(MASS, u, masked=False), ref @ u) < 1e-14


@pytest.mark.parametrize("bp,p", [(1, 1), (1, 3), (1, 6), (5, 2), (5, 5), (5, 7), (3, 4)])
def test_volume_of_perturbed_domain_is_one(bp, p):
    disc, _ = make_disc(bp, p, 3, 2, 2, seed=3, dirichlet=False)
    one = np.ones(disc.nglobal)
    assert abs(one @ disc.apply(MASS, one, masked=False) - 1.0) < 1e-13


@pytest.mark.parametrize("bp,p", [(3, 1), (3, 4), (5, 1), (5, 3), (5, 7)])
def test_constants_in_null_space(bp, p):
    disc, _ = make_disc(bp, p, 2, 2, 3, seed=4, dirichlet=False)
    one = np.ones(disc.nglobal)
    w = disc.apply(STIFF, one, masked=False)
    scale = np.abs(disc.diag(STIFF, masked=False)).max()
    assert np.abs(w).max() < 1e-13 * scale


@pytest.mark.parametrize("bp,p", [(3, 1), (3, 3), (3, 6), (5, 2), (5, 4), (5, 7)])
def test_energy_identity_coordinates(bp, p):
    # coordinates lie in the isoparametric space: X^T A X = vol * I (vol = 1)
    disc, mesh = make_disc(bp, p, 2, 3, 2, seed=5, dirichlet=False)
    X = mesh.global_coords()
    AX = disc.apply(STIFF, X, masked=False)
    assert np.allclose(X.T @ AX, np.eye(3), atol=1e-12)


@pytest.mark.parametrize("bp,p,seed", [(3, 1, 6), (3, 5, 6), (5, 2, 6), (5, 6, 6), (5, 1, None)])
def test_patch_test_linear_field(bp, p, seed):
    disc, mesh = make_disc(bp, p, 3, 3, 2, seed=seed, dirichlet=False)
    X = mesh.global_coords()
    lin = 0.3 + 1.1 * X[:, 0] - 0.7 * X[:, 1] + 0.4 * X[:, 2]
    w = disc.apply(STIFF, lin, masked=False)
    interior = mesh.boundary == 0
    scale = np.abs(disc.diag(STIFF, masked=False)).max()
    assert np.abs(w[interior]).max() < 1e-12 * scale


def test_patch_test_fails_for_gll_p1_on_perturbed_mesh():
    # sanity: the pin above is sharp. Jac * d(phi)/dx has degree p+1 per
    # variable on trilinear elements, GLL with p+1 points is exact to 2p-1,
    # so collocated quadrature passes from p=2 on and fails at p=1.
    disc, mesh = make_disc(5, 1, 3, 3, 3, seed=6, dirichlet=False)
    X = mesh.global_coords()
    w = disc.apply(STIFF, X[:, 0], masked=False)
    scale = np.abs(disc.diag(STIFF, masked=False)).max()
    assert np.abs(w[mesh.boundary == 0]).max() > 1e-9 * scale


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("quad", ["gl", "gll"])
@pytest.mark.parametrize("which", [MASS, STIFF])
def test_matrix_free_equals_brute_force(p, quad, which):
    q = p + 2 if quad == "gl" else p + 1
    disc, _ = custom_disc(p, q, quad, 2, 2, 1 + (p < 4), seed=7, dirichlet=True)
    rng = np.random.default_rng(p)
    for masked in (False, True):
        A = assemble(disc, which, masked=masked)
        u = rng.standard_normal(disc.nglobal)
        assert rel_err(disc.apply(which, u, masked=masked), A @ u) < 1e-13
        assert np.allclose(disc.diag(which, masked=masked), A.diagonal(),
                           rtol=1e-13, atol=1e-15 * abs(A.diagonal()).max())


def test_over_integration_variant_and_vector_components():
    # q = p + 3 GL (a rule outside the table) and 3 interleaved components
    disc, _ = custom_disc(3, 6, "gl", 2, 1, 2, seed=8, dirichlet=True)
    A = assemble(disc, STIFF)
    U = np.random.default_rng(9).standard_normal((disc.nglobal, 3))
    W = disc.apply(STIFF, U)
    for c in range(3):
        assert rel_err(W[:, c], A @ U[:, c]) < 1e-13


@pytest.mark.parametrize("bp,p", [(3, 3), (5, 4)])
def test_masked_operator_is_symmetric_positive_definite(bp, p):
    disc, mesh = make_disc(bp, p, 2, 2, 2, seed=10)
    A = assemble(disc, STIFF, masked=True).toarray()
    assert np.allclose(A, A.T, atol=1e-13 * abs(A).max())
    inner = mesh.boundary == 0
    ev = np.linalg.eigvalsh(A[np.ix_(inner, inner)])
    assert ev.min() > 0
    # Dirichlet rows and columns are zero
    assert np.abs(A[~inner]).max() == 0 and np.abs(A[:, ~inner]).max() == 0


def test_kappa_scales_operator_and_is_linear():
    disc, _ = make_disc(5, 3, 2, 2, 2, seed=11)
    kap = np.random.default_rng(12).uniform(0.5, 2.0, size=(disc.E, disc.rule.q ** 3))
    disc_k, _ = make_disc(5, 3, 2, 2, 2, seed=11, kappa=kap)
    disc_2, _ = make_disc(5, 3, 2, 2, 2, seed=11, kappa=2.0 * np.ones_like(kap))
    u = np.random.default_rng(13).standard_normal(disc.nglobal)
    assert rel_err(disc_2.apply(STIFF, u), 2 * disc.apply(STIFF, u)) < 1e-14
    A = assemble(disc_k, STIFF)
    assert rel_err(disc_k.apply(STIFF, u), A @ u) < 1e-13


def test_inverted_element_is_rejected():
    rule = bp_rule(5, 2)
    mesh = synth.brick_mesh(2, 1, 1, 2, rule.xi, seed=None)
    xyz = mesh.node_xyz.copy()
    xyz[1, :, 0] = 1.5 - xyz[1, :, 0]      # mirror element 1 in x
    with pytest.raises(ValueError, match="element 1"):
        geometric_factors(rule, xyz)


def test_sampled_apply_equals_full_apply():
    from oracle.sampled import apply_at_nodes, elements_containing
    disc, mesh = make_disc(5, 3, 4, 3, 3, seed=12)
    u = np.random.default_rng(14).standard_normal((disc.nglobal, 2))
    full = disc.apply(STIFF, u)
    nodes = np.array([0, 5, 77, 300, disc.nglobal // 2, disc.nglobal - 1])
    els = elements_containing(mesh.elem_dofs, nodes)
    xyz = synth.element_coordinates(4, 3, 3, 3, disc.rule.xi, els, seed=12)
    assert np.array_equal(xyz, mesh.node_xyz[els])
    w = apply_at_nodes(disc.rule, mesh.elem_dofs[els], xyz, u, nodes, STIFF, True,
                       mesh.boundary)
    assert rel_err(w, full[nodes]) < 1e-14


# -- Helmholtz operator, eq. (hm2): H = A + B_beta -------------------------------

@pytest.mark.parametrize("p,quad", [(1, "gll"), (3, "gl"), (4, "gll"), (2, "gl")])
def test_helmholtz_equals_brute_force(p, quad):
    q = p + 2 if quad == "gl" else p + 1
    rng = np.random.default_rng(20 + p)
    beta_q = rng.uniform(0.5, 3.0, size=(2 * 2 * 2, q ** 3))
    for beta in (0.7, beta_q):
        disc, _ = custom_disc(p, q, quad, 2, 2, 2, seed=21, dirichlet=True, beta=beta)
        for masked in (False, True):
            H = assemble(disc, HELM, masked=masked)
            u = rng.standard_normal(disc.nglobal)
            assert rel_err(disc.apply(HELM, u, masked=masked), H @ u) < 1e-13
            assert np.allclose(disc.diag(HELM, masked=masked), H.diagonal(),
                               rtol=1e-13, atol=1e-15 * abs(H.diagonal()).max())


@pytest.mark.parametrize("bp,p", [(5, 3), (3, 4), (5, 6)])
def test_helmholtz_constant_integrates_beta(bp, p):
    # A 1 = 0, so 1^T H 1 = int beta dx: beta times the volume (1) for a
    # constant beta, and the quadrature sum of beta_q J_q w_q for a field
    disc, mesh = make_disc(bp, p, 2, 3, 2, seed=22, dirichlet=False, beta=2.5)
    one = np.ones(disc.nglobal)
    assert abs(one @ disc.apply(HELM, one, masked=False) - 2.5) < 1e-12
    q = disc.rule.q
    xq = np.random.default_rng(23).uniform(0.2, 1.8, size=(disc.E, q ** 3))
    disc_v, _ = make_disc(bp, p, 2, 3, 2, seed=22, dirichlet=False, beta=xq)
    rho = disc.rule.rho
    w3 = np.einsum("a,b,c->cba", rho, rho, rho).reshape(-1)
    integral = np.sum(xq * disc.jac * w3[None, :])
    assert abs(one @ disc_v.apply(HELM, one, masked=False) - integral) < 1e-12 * integral


def test_helmholtz_with_zero_beta_is_stiffness_and_is_spd_without_dirichlet():
    disc, _ = make_disc(5, 3, 2, 2, 2, seed=24, dirichlet=False)
    u = np.random.default_rng(25).standard_normal(disc.nglobal)
    assert rel_err(disc.apply(HELM, u), disc.apply(STIFF, u)) == 0.0
    disc_b, _ = make_disc(5, 3, 2, 2, 2, seed=24, dirichlet=False, beta=1.0)
    H = assemble(disc_b, HELM, masked=False).toarray()
    assert np.allclose(H, H.T, atol=1e-13 * abs(H).max())
    assert np.linalg.eigvalsh(H).min() > 0


@pytest.mark.parametrize("p", [11, 15])
def test_high_order_gll_pins(p):
    # the oracle at the top of the order range: volume, constants in the null
    # space and the coordinate energy identity (trilinear geometry, exact with
    # GLL from p = 2 on)
    disc, mesh = make_disc(5, p, 2, 1, 1, seed=3, dirichlet=False)
    one = np.ones(disc.nglobal)
    assert abs(one @ disc.apply(MASS, one, masked=False) - 1.0) < 1e-13
    w = disc.apply(STIFF, one, masked=False)
    assert np.abs(w).max() < 1e-12 * np.abs(disc.diag(STIFF, masked=False)).max()
    X = mesh.global_coords()
    assert np.allclose(X.T @ disc.apply(STIFF, X, masked=False), np.eye(3), atol=1e-11)
