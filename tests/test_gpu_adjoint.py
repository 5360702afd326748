"""GPU checks of the differentiable variable-coefficient solve: loss,
adjoint gradients against the oracle, and against central finite
differences of the GPU loss."""
import numpy as np
import pytest

import synth
from oracle import adjoint
from oracle.operators import Discretization
from tests.gpu_cases import Case, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# Quantities that depend on a CG solution carry its error: with the relative
# residual at 1e-14 and Jacobi-preconditioned condition numbers of a few
# hundred on these meshes, solutions agree to about 1e-11; 1e-9 leaves margin.
SOLVE_TOL = 1e-9


def setup_case(p=3, grid=(3, 3, 3), ncomp=2):
    c = Case(5, p, *grid, seed=7, ncomp=ncomp)
    kap = synth.kappa_log(c.mesh.node_xyz, 31)          # GLL: points = nodes
    b = synth.rhs_uniform(c.disc.nglobal, 100, ncomp=ncomp, dirichlet=c.mesh.boundary)
    ut = 0.5 * adjoint.solve(c.disc, b, rtol=1e-14)[0]  # kappa = 1 solution, halved
    disc_k = Discretization(c.disc.rule, c.mesh.elem_dofs, c.mesh.node_xyz, c.disc.nglobal,
                            c.mesh.boundary, kappa=kap)
    return c, kap, b, ut, disc_k


@pytest.mark.parametrize("bp,p,ncomp,order", [(5, 3, 1, "internal"), (5, 7, 2, "caller"),
                                               (6, 4, 3, "internal"), (1, 3, 1, "internal"),
                                               (3, 5, 3, "internal"), (3, 2, 1, "scrambled")])
def test_mass_misfit_matches_oracle(bp, p, ncomp, order):
    # L = 1/2 sum_c d_c^T M d_c and M d (d = u - u_t, unmasked mass of the
    # operator's own quadrature: GLL collocated for BP5/6, Gauss for BP1/3)
    # against the oracle's loss and gradient; the fixed-order energy sum
    # gives the same bits on a second call
    grid = (3, 3, 3) if p <= 4 else (3, 2, 2)
    c = Case(bp, p, *grid, seed=40 + p, ncomp=ncomp, caller_order=order == "caller",
             scramble=7 if order == "scrambled" else None)
    try:
        u = synth.rhs_uniform(c.disc.nglobal, 41, ncomp=ncomp)
        ut = synth.rhs_uniform(c.disc.nglobal, 51, ncomp=ncomp)
        ud = torch.tensor(u.T.copy() if ncomp > 1 else u, device="cuda")
        utd = torch.tensor(ut.T.copy() if ncomp > 1 else ut, device="cuda")
        L, g = c.op.mass_misfit(ud, utd)
        Lo = adjoint.loss(c.disc, u, ut)
        go = adjoint.loss_grad_u(c.disc, u, ut)
        assert abs(L - Lo) <= 1e-12 * abs(Lo), (L, Lo)
        gh = g.cpu().numpy()
        assert rel(gh.T if ncomp > 1 else gh, go) <= 1e-12
        L2, g2 = c.op.mass_misfit(ud, utd, grad=False)
        assert L2 == L and g2 is None
        L0, g0 = c.op.mass_misfit(ud, ud)
        assert L0 == 0.0 and float(torch.abs(g0).max()) == 0.0
    finally:
        c.close()


def test_loss_and_gradients_match_oracle():
    from paper_2004_06722_amd.autograd import mass_norm_loss, poisson_solve
    c, kap, b, ut, disc_k = setup_case()
    try:
        # device vectors are component-major [ncomp, n]; the oracle's are [n, ncomp]
        k_t = torch.tensor(kap, device="cuda", requires_grad=True)
        b_t = torch.tensor(b.T.copy(), device="cuda", requires_grad=True)
        u = poisson_solve(c.op, k_t, b_t, rtol=1e-14)
        L = mass_norm_loss(c.op, u, torch.tensor(ut.T.copy(), device="cuda"))
        L.backward()
        Lo, go, lam_o, uo = adjoint.loss_and_grad(disc_k, b, ut, rtol=1e-14)
        assert abs(L.item() - Lo) <= SOLVE_TOL * abs(Lo)
        assert rel(u.detach().cpu().numpy().T, uo) <= SOLVE_TOL
        assert rel(k_t.grad.cpu().numpy(), go) <= SOLVE_TOL
        assert rel(b_t.grad.cpu().numpy().T, lam_o) <= SOLVE_TOL
    finally:
        c.close()


def test_gradient_matches_finite_differences():
    from paper_2004_06722_amd.autograd import mass_norm_loss, poisson_solve
    c, kap, b, ut, _ = setup_case(p=4, grid=(2, 2, 3))
    try:
        b_t = torch.tensor(b.T.copy(), device="cuda")
        ut_t = torch.tensor(ut.T.copy(), device="cuda")
        k_t = torch.tensor(kap, device="cuda", requires_grad=True)
        L = mass_norm_loss(c.op, poisson_solve(c.op, k_t, b_t, rtol=1e-14), ut_t)
        L.backward()
        g = k_t.grad.cpu().numpy()
        eps = 1e-5
        for j in range(4):
            dlt = synth.fd_direction(kap.shape, 1000 + j)
            Ls = []
            for sgn in (1.0, -1.0):
                kk = torch.tensor(kap + sgn * eps * dlt, device="cuda")
                with torch.no_grad():
                    Ls.append(mass_norm_loss(c.op, poisson_solve(c.op, kk, b_t, rtol=1e-14),
                                             ut_t).item())
            fd = (Ls[0] - Ls[1]) / (2 * eps)
            an = float(np.sum(g * dlt))
            assert abs(fd - an) <= 1e-6 * abs(an), (j, fd, an)
    finally:
        c.close()
