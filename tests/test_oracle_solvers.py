"""Pins for the oracle's PCG, defect correction and adjoint gradient."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import adjoint, mixed
from oracle.assembled import assemble, d_stiffness_d_kappa
from oracle.operators import MASS, STIFF
from oracle.pcg import pcg, pcg_single_reduction
from tests.oracle_cases import make_disc, rel_err


def manufactured_rhs(disc, mesh):
    """rhs = M f (GLL mass of the problem's own rule), masked."""
    f = synth.manufactured_f(mesh.global_coords())
    return disc.apply(MASS, f, masked=False) * disc.mask


def config1():
    return make_disc(5, 3, 4, 4, 4, seed=0)


def test_config1_sizes():
    disc, mesh = config1()
    assert disc.nglobal == 13 ** 3 == 2197
    assert int((mesh.boundary == 0).sum()) == 11 ** 3
    assert disc.E * 3 ** 3 == 1728


def test_pcg_matches_direct_solve_config1():
    disc, mesh = config1()
    b = manufactured_rhs(disc, mesh)
    dinv = disc.jacobi_inverse(STIFF)
    x, info = pcg(lambda v: disc.apply(STIFF, v), b, dinv, rtol=1e-13, maxit=2000)
    assert info["rel_res"][-1] <= 1e-13
    inner = mesh.boundary == 0
    A = assemble(disc, STIFF).tocsr()[inner][:, inner]
    xd = np.zeros_like(b)
    xd[inner] = spla.spsolve(A.tocsc(), b[inner])
    assert rel_err(x, xd) < 1e-11
    # tolerance mode at 1e-8 stops at the first iterate below tolerance
    x8, info8 = pcg(lambda v: disc.apply(STIFF, v), b, dinv, rtol=1e-8, maxit=2000)
    assert info8["rel_res"][-1] <= 1e-8 < info8["rel_res"][-2]


def test_pcg_fixed_iterations_and_zero_rhs():
    disc, mesh = make_disc(5, 2, 2, 2, 2, seed=1)
    dinv = disc.jacobi_inverse(STIFF)
    b = synth.rhs_uniform(disc.nglobal, 0, dirichlet=mesh.boundary)
    x, info = pcg(lambda v: disc.apply(STIFF, v), b, dinv, maxit=100, fixed_iters=True)
    assert info["iters"] == 100 and np.all(np.isfinite(x))
    # the system is tiny: CG has converged long before 100 iterations and the
    # zero-denominator reading keeps it finite and converged
    assert info["rel_res"][-1] < 1e-12
    x0, info0 = pcg(lambda v: disc.apply(STIFF, v), 0 * b, dinv, maxit=5, fixed_iters=True)
    assert np.all(x0 == 0) and info0["iters"] == 5


def test_pcg_first_iterates_match_textbook_cg_on_assembled_matrix():
    # independent statement: plain CG on D^-1/2 A D^-1/2 (scipy-free loop on
    # the assembled matrix) gives the same iterates as Jacobi-PCG
    disc, mesh = make_disc(3, 2, 2, 2, 2, seed=2)
    b = synth.rhs_uniform(disc.nglobal, 0, dirichlet=mesh.boundary)
    inner = mesh.boundary == 0
    A = assemble(disc, STIFF).toarray()[np.ix_(inner, inner)]
    s = 1 / np.sqrt(np.diag(A))
    As = s[:, None] * A * s[None, :]
    bs = s * b[inner]
    y = np.zeros_like(bs)
    r = bs.copy()
    p = r.copy()
    ref = []
    for _ in range(6):
        Ap = As @ p
        a = (r @ r) / (p @ Ap)
        y = y + a * p
        rn = r - a * Ap
        p = rn + (rn @ rn) / (r @ r) * p
        r = rn
        ref.append(s * y)
    rec = []
    pcg(lambda v: disc.apply(STIFF, v), b, disc.jacobi_inverse(STIFF), maxit=6,
        fixed_iters=True, record=rec)
    for k in range(6):
        assert rel_err(rec[k][inner], ref[k]) < 1e-12


def test_vector_components_are_independent_systems():
    disc, mesh = make_disc(5, 2, 2, 2, 1, seed=3)
    B = synth.rhs_uniform(disc.nglobal, 0, ncomp=3, dirichlet=mesh.boundary)
    dinv = disc.jacobi_inverse(STIFF)
    X, _ = pcg(lambda v: disc.apply(STIFF, v), B, dinv, maxit=7, fixed_iters=True)
    for c in range(3):
        xc, _ = pcg(lambda v: disc.apply(STIFF, v), B[:, c], dinv, maxit=7, fixed_iters=True)
        assert rel_err(X[:, c], xc) < 1e-14


@pytest.mark.slow
def test_manufactured_solution_converges_spectrally():
    errs = []
    for N in range(2, 9):
        disc, mesh = make_disc(5, N, 4, 4, 4, seed=0)
        b = manufactured_rhs(disc, mesh)
        x, _ = pcg(lambda v: disc.apply(STIFF, v), b, disc.jacobi_inverse(STIFF),
                   rtol=1e-13, maxit=5000)
        ue = synth.manufactured_u(mesh.global_coords())
        errs.append(np.abs(x - ue).max())
    for a, b_ in zip(errs, errs[2:]):
        if a > 1e-9:
            assert b_ < a / 10, errs
    assert errs[-1] < 1e-7, errs


def test_defect_correction_reaches_fp64_tolerance():
    disc, mesh = make_disc(5, 4, 3, 3, 3, seed=4)
    b = manufactured_rhs(disc, mesh)
    x, info = mixed.defect_correction(disc, b, outer_rtol=1e-10, inner_rtol=1e-5)
    assert info["rel_res"][-1] <= 1e-10
    assert info["outer"] >= 2       # FP32 alone could not reach 1e-10
    r = b - assemble(disc, STIFF) @ x
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.5e-10
    x64, _ = mixed.solve_fp64(disc, b, 1e-10)
    assert rel_err(x, x64) < 1e-7


def test_reliable_update_cg_keeps_the_krylov_space():
    # FP32 CG with FP64 residual replacement: reaches the FP64 tolerance in
    # about the FP64 iteration count, where restarted defect correction
    # needs its inner solves' sum of iterations (a variant that resets p at
    # each substitution needs more than twice the FP64 count here)
    disc, mesh = make_disc(5, 5, 4, 4, 4, seed=4)
    b = manufactured_rhs(disc, mesh)
    x, info = mixed.reliable_cg(disc, b, rtol=1e-10, delta=1e-2)
    assert info["rel_res"][-1] <= 1e-10 and info["updates"] >= 2
    r = b - assemble(disc, STIFF) @ x
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.5e-10
    x64, i64 = mixed.solve_fp64(disc, b, 1e-10)
    assert rel_err(x, x64) < 1e-7
    assert info["iters"] <= 1.25 * i64["iters"], (info["iters"], i64["iters"])
    _, dc = mixed.defect_correction(disc, b, outer_rtol=1e-10, inner_rtol=1e-5)
    assert sum(dc["inner_iters"]) > info["iters"]


def _kappa(disc, mesh, seed=21):
    from oracle.geometry import quad_points
    return synth.kappa_log(quad_points(disc.rule, mesh.node_xyz), seed)


def test_adjoint_gradient_matches_dense_derivative():
    disc0, mesh = make_disc(5, 2, 2, 2, 2, seed=5)
    kap = _kappa(disc0, mesh)
    disc, _ = make_disc(5, 2, 2, 2, 2, seed=5, kappa=kap)
    b = synth.rhs_uniform(disc.nglobal, 100, ncomp=2, dirichlet=mesh.boundary)
    ut = adjoint.solve(disc0, b)[0]
    L, g, lam, u = adjoint.loss_and_grad(disc, b, ut)
    n = disc.rule.p1 ** 3
    for e, qp in [(0, 0), (3, 13), (7, 26), (5, 4)]:
        dA = d_stiffness_d_kappa(disc, e, qp)
        idx = disc.elem_dofs[e]
        m = disc.mask[idx][:, None]
        ref = -np.sum((lam[idx] * m) * (dA @ (u[idx] * m)))
        assert abs(g[e, qp] - ref) <= 1e-10 * max(abs(ref), 1e-30) + 1e-18
    assert g.shape == (disc.E, disc.rule.q ** 3) and n == 27


def test_adjoint_gradient_scaling_closed_form():
    # kappa = c * kappa0 => u(c) = u0 / c, so dL/dc = (u0/c - ut)^T M (-u0/c^2)
    # must equal <dL/dkappa, kappa0>
    disc0, mesh = make_disc(5, 3, 2, 2, 2, seed=6)
    kap0 = _kappa(disc0, mesh)
    b = synth.rhs_uniform(disc0.nglobal, 100, dirichlet=mesh.boundary)
    ut = 0.5 * adjoint.solve(disc0, b)[0]
    c = 1.3
    disc, _ = make_disc(5, 3, 2, 2, 2, seed=6, kappa=c * kap0)
    discB, _ = make_disc(5, 3, 2, 2, 2, seed=6, kappa=kap0)
    u0 = adjoint.solve(discB, b)[0]
    L, g, lam, u = adjoint.loss_and_grad(disc, b, ut)
    d = u0 / c - ut
    dLdc = float(np.sum(d * disc.apply(MASS, -u0 / c ** 2, masked=False)))
    assert abs(np.sum(g * kap0) - dLdc) <= 1e-9 * abs(dLdc)


def test_adjoint_gradient_finite_differences():
    disc0, mesh = make_disc(5, 2, 2, 2, 2, seed=7)
    kap = _kappa(disc0, mesh)
    b = synth.rhs_uniform(disc0.nglobal, 100, ncomp=2, dirichlet=mesh.boundary)
    ut = 0.5 * adjoint.solve(disc0, b)[0]
    disc, _ = make_disc(5, 2, 2, 2, 2, seed=7, kappa=kap)
    L, g, _, u = adjoint.loss_and_grad(disc, b, ut)
    eps = 1e-5
    for j in range(4):
        dlt = synth.fd_direction(kap.shape, 1000 + j)
        Ls = []
        for sgn in (1, -1):
            dk, _ = make_disc(5, 2, 2, 2, 2, seed=7, kappa=kap + sgn * eps * dlt)
            us = adjoint.solve(dk, b, x0=u)[0]
            Ls.append(adjoint.loss(dk, us, ut))
        fd = (Ls[0] - Ls[1]) / (2 * eps)
        an = float(np.sum(g * dlt))
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


def test_single_reduction_pcg_has_the_same_iterates():
    # the Chronopoulos-Gear recurrences reproduce standard PCG's iterates (to
    # rounding), reach the direct solution, and handle several components
    disc, mesh = config1()
    b = manufactured_rhs(disc, mesh)
    dinv = disc.jacobi_inverse(STIFF)
    A = lambda v: disc.apply(STIFF, v)
    ref, sr = [], []
    pcg(A, b, dinv, maxit=12, fixed_iters=True, record=ref)
    pcg_single_reduction(A, b, dinv, maxit=12, fixed_iters=True, record=sr)
    for k in range(12):
        assert rel_err(sr[k], ref[k]) < 1e-12, k
    x, info = pcg_single_reduction(A, b, dinv, rtol=1e-13, maxit=2000)
    inner = mesh.boundary == 0
    Ad = assemble(disc, STIFF).tocsr()[inner][:, inner]
    xd = np.zeros_like(b)
    xd[inner] = spla.spsolve(Ad.tocsc(), b[inner])
    assert rel_err(x, xd) < 1e-11
    _, info_std = pcg(A, b, dinv, rtol=1e-13, maxit=2000)
    assert abs(info["iters"] - info_std["iters"]) <= 1
    B = np.stack([b, 2 * b + 0.1 * disc.mask], axis=1)
    r2, s2 = [], []
    pcg(A, B, dinv, maxit=6, fixed_iters=True, record=r2)
    pcg_single_reduction(A, B, dinv, maxit=6, fixed_iters=True, record=s2)
    assert rel_err(s2[-1], r2[-1]) < 1e-12
