"""Pins for the oracle's 1D rules and matrices (section 3 Table "bps", section 5)."""
import os

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle.quadrature import (Rule, gauss_legendre, gauss_lobatto_legendre,
                               lagrange_deriv_matrix, lagrange_matrix)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("q", range(1, 18))
def test_gl_matches_library_rule(q):
    x, w = gauss_legendre(q)
    xr, wr = npleg.leggauss(q)
    assert np.allclose(x, xr, rtol=0, atol=2e-15)
    assert np.allclose(w, wr, rtol=0, atol=2e-15)


@pytest.mark.parametrize("q", range(1, 12))
def test_gl_exact_to_degree_2q_minus_1(q):
    x, w = gauss_legendre(q)
    for k in range(2 * q):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14
    k = 2 * q  # first degree not integrated exactly
    assert abs(np.dot(w, x ** k) - 2.0 / (k + 1)) > 1e-8


@pytest.mark.parametrize("p1", range(2, 17))
def test_gll_nodes_are_endpoints_and_roots_of_dP(p1):
    x, w = gauss_lobatto_legendre(p1)
    p = p1 - 1
    assert x[0] == -1.0 and x[-1] == 1.0
    assert np.all(np.diff(x) > 0)
    if p1 > 2:
        roots = np.sort(npleg.Legendre.basis(p).deriv().roots().real)
        assert np.allclose(x[1:-1], roots, rtol=0, atol=1e-13)
    assert abs(w.sum() - 2.0) < 1e-14
    assert np.allclose(x, -x[::-1], atol=1e-15)
    assert np.allclose(w, w[::-1], atol=1e-15)


@pytest.mark.parametrize("p1", range(2, 12))
def test_gll_exact_to_degree_2q_minus_3(p1):
    x, w = gauss_lobatto_legendre(p1)
    for k in range(2 * p1 - 2):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14
    k = 2 * p1 - 2
    assert abs(np.dot(w, x ** k) - 2.0 / (k + 1)) > 1e-8


@pytest.mark.parametrize("p,q,quad", [(p, p + 2, "gl") for p in range(1, 10)]
                         + [(p, p + 1, "gll") for p in range(1, 16)])
def test_interpolation_and_derivative_exact_on_polynomials(p, q, quad):
    r = Rule(p, q, quad)
    for k in range(p + 1):
        f = r.xi ** k
        assert np.allclose(r.J @ f, r.eta ** k, atol=1e-13)
        df = k * r.eta ** (k - 1) if k else np.zeros(q)
        assert np.allclose(r.D @ f, df, atol=1e-11 * max(1, k * k))
    assert np.allclose(r.D @ np.ones(p + 1), 0.0, atol=1e-12)
    assert np.allclose(r.J.sum(axis=1), 1.0, atol=1e-14)


@pytest.mark.parametrize("p,q,quad", [(3, 5, "gl"), (7, 9, "gl"), (7, 8, "gll"), (4, 5, "gll")])
def test_center_symmetry(p, q, quad):
    # Appendix A3: phi_i(xi_j) = phi_{p+2-i}(xi_{q+1-j}) and
    # phi_i'(xi_j) = -phi'_{p+2-i}(xi_{q+1-j}) (1-based)
    r = Rule(p, q, quad)
    assert np.allclose(r.J, r.J[::-1, ::-1], atol=1e-14)
    assert np.allclose(r.D, -r.D[::-1, ::-1], atol=1e-12)


def test_gll_collocation_is_identity():
    # section 5: for GLL quadrature on the nodal points J^ is the identity
    for p in range(1, 12):
        r = Rule(p, p + 1, "gll")
        assert np.array_equal(r.J, np.eye(p + 1))
        assert np.array_equal(lagrange_matrix(r.xi, r.xi), np.eye(p + 1))


def test_shape_symmetric_worked_pattern():
    pat = np.loadtxt(os.path.join(GOLDEN, "shape_symmetric_p3_q5.txt"), dtype=int)
    S = Rule(3, 5, "gl").J
    assert S.shape == pat.shape
    for lab in np.unique(pat):
        vals = S[pat == lab]
        assert np.ptp(vals) < 1e-14
    # distinct labels really are distinct values
    reps = np.array([S[pat == lab][0] for lab in np.unique(pat)])
    assert len(np.unique(np.round(reps, 12))) == len(reps)


def test_derivative_matrix_matches_numpy_polynomial_fit():
    # independent construction: differentiate the interpolating polynomial
    r = Rule(6, 8, "gl")
    for j in range(7):
        e = np.zeros(7)
        e[j] = 1.0
        c = npleg.legfit(r.xi, e, 6)
        assert np.allclose(r.D[:, j], npleg.legval(r.eta, npleg.legder(c)), atol=1e-11)
    assert np.allclose(lagrange_deriv_matrix(r.xi, r.xi).sum(axis=1), 0, atol=1e-12)
