"""GPU parity on arbitrary gather maps and with a coefficient on Gauss-Legendre
operators.

Section 3 forbids treating the elements as a tensor grid and section 4,
eq. (dssum), makes Q a general Boolean gather: these meshes renumber the
global nodes at random, list the elements in random order and turn each
element's local axes by a random proper cube symmetry (synth.scramble_mesh),
so the atomic scatter sees non-monotone ids, the Gauss-Legendre transposed
map is built from a random numbering, and the geometric factors come from
rotated local frames. Bar: normwise relative 1e-12 against the oracle on the
same map (FP32: 2e-6, as in the other FP32 tests).
"""
import numpy as np
import pytest

import synth
from oracle.operators import HELM, MASS, STIFF, Discretization
from oracle.pcg import pcg
from oracle.geometry import quad_points
from tests.gpu_cases import TOL, Case, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    a = np.asarray(a)
    return torch.from_numpy(np.ascontiguousarray(a.T if a.ndim == 2 else a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    a = t.cpu().numpy()
    return a.T if a.ndim == 2 else a


def grid_for(p):
    return (3, 3, 3) if p <= 4 else (3, 2, 2)


def check_iterates(c, which, masked, b, ks=(1, 4, 8), disc=None):
    disc = disc or c.disc
    rec = []
    pcg(lambda v: disc.apply(which, v, masked=masked), b,
        disc.jacobi_inverse(which, masked=masked), maxit=max(ks), fixed_iters=True, record=rec)
    for k in ks:
        x, st = c.op.pcg_solve(dev(b), which=which, maxit=k, fixed_iters=True)
        assert st["iters"] == k
        assert rel(host(x), rec[k - 1]) <= TOL, (k, rel(host(x), rec[k - 1]))


@pytest.mark.parametrize("bp,p", [(1, 2), (1, 5), (1, 7), (3, 3), (3, 7), (5, 1), (5, 4),
                                  (5, 7), (5, 8)])
def test_arbitrary_map_apply_diag_iterates(bp, p):
    c = Case(bp, p, *grid_for(p), seed=p, scramble=500 + p)
    try:
        u = c.vec(40 + p)
        for which in (MASS, STIFF):
            for masked in (False, True):
                w = host(c.op.apply(which, dev(u), masked=masked))
                ref = c.disc.apply(which, u, masked=masked)
                assert rel(w, ref) <= TOL, (which, masked, rel(w, ref))
                d = host(c.op.diag(which, masked=masked))
                assert rel(d, c.disc.diag(which, masked=masked)) <= TOL, (which, masked)
        which = MASS if bp == 1 else STIFF
        masked = bp >= 3
        mask = (1 - c.mesh.boundary) if masked else np.ones(c.disc.nglobal)
        check_iterates(c, which, masked, c.vec(41 + p) * mask)
    finally:
        c.close()


@pytest.mark.parametrize("bp,p", [(2, 4), (4, 3), (6, 7)])
def test_arbitrary_map_vector_components(bp, p):
    # ncomp = 3 on one scrambled mesh: per-component apply and independent CG
    c = Case(bp, p, *grid_for(p), seed=7, ncomp=3, scramble=600 + bp)
    try:
        which = MASS if bp == 2 else STIFF
        masked = bp >= 3
        mask = (1 - c.mesh.boundary) if masked else np.ones(c.disc.nglobal)
        u = c.vec(50)
        w = host(c.op.apply(which, dev(u), masked=masked))
        ref = c.disc.apply(which, u, masked=masked)
        for k in range(3):
            assert rel(w[:, k], ref[:, k]) <= TOL, k
        check_iterates(c, which, masked, c.vec(51) * mask[:, None])
    finally:
        c.close()


@pytest.mark.parametrize("bp,p", [(1, 3), (5, 5)])
def test_arbitrary_map_single_reduction_iterates(bp, p):
    c = Case(bp, p, *grid_for(p), seed=8, scramble=700 + p)
    try:
        c.op.set_cg_variant(True)
        which = MASS if bp == 1 else STIFF
        masked = bp >= 3
        mask = (1 - c.mesh.boundary) if masked else np.ones(c.disc.nglobal)
        check_iterates(c, which, masked, c.vec(60) * mask, ks=(1, 2, 8))
    finally:
        c.close()


@pytest.mark.parametrize("bp,p", [(3, 4), (5, 6)])
def test_arbitrary_map_helmholtz_and_local(bp, p):
    # H = A + B_beta with variable beta at the quadrature points, and the
    # unassembled element operators, on rotated element frames
    c = Case(bp, p, *grid_for(p), seed=9, scramble=800 + p)
    try:
        beta = synth.kappa_log(quad_points(c.disc.rule, c.mesh.node_xyz), 61)
        c.op.set_helmholtz(0.0, torch.from_numpy(np.ascontiguousarray(beta)).cuda())
        hd = Discretization(c.disc.rule, c.mesh.elem_dofs, c.mesh.node_xyz, c.disc.nglobal,
                            c.dir, beta=beta)
        u = c.vec(62)
        assert rel(host(c.op.apply(HELM, dev(u))), hd.apply(HELM, u)) <= TOL
        assert rel(host(c.op.diag(HELM)), hd.diag(HELM)) <= TOL
        check_iterates(c, HELM, True, u * (1 - c.mesh.boundary), ks=(1, 5), disc=hd)
        uL = np.random.default_rng(63).uniform(-1, 1, c.mesh.elem_dofs.shape)
        p1 = p + 1
        wL = c.op.apply_local(STIFF, torch.from_numpy(uL).cuda()).cpu().numpy()
        ref = c.disc.stiff_local(uL.reshape(-1, p1, p1, p1)).reshape(uL.shape)
        assert rel(wL, ref) <= TOL
    finally:
        c.close()


def test_arbitrary_map_fp32_apply():
    c = Case(5, 7, 3, 2, 2, seed=10, fp32=True, scramble=901)
    try:
        u = (c.vec(64) * (1 - c.mesh.boundary)).astype(np.float32)
        w = host(c.op.apply(STIFF, dev(u)))
        assert rel(w, c.disc.apply(STIFF, u.astype(np.float64))) < 2e-6
    finally:
        c.close()


def test_arbitrary_map_many_work_groups():
    # 512 elements of order 7: hundreds of work-groups whose atomic scatters
    # meet at randomly numbered nodes
    c = Case(5, 7, 8, 8, 8, seed=11, scramble=902)
    try:
        u = c.vec(65)
        assert rel(host(c.op.apply(STIFF, dev(u))), c.disc.apply(STIFF, u)) <= TOL
        check_iterates(c, STIFF, True, u * (1 - c.mesh.boundary), ks=(3,))
    finally:
        c.close()


@pytest.mark.parametrize("p,scramble", [(3, None), (7, None), (4, 903)])
def test_kappa_on_gauss_legendre_operators(p, scramble):
    # BP3 with a coefficient at the Gauss points, given in the caller's point
    # order [c][b][a]: the library stores Gauss-Legendre quadrature data with
    # the point index reversed, so the coefficient is mapped onto that order
    c = Case(3, p, *grid_for(p), seed=12, scramble=scramble)
    try:
        kap = synth.kappa_log(quad_points(c.disc.rule, c.mesh.node_xyz), 70 + p)
        c.op.set_coeff(torch.from_numpy(np.ascontiguousarray(kap)).cuda())
        kd = Discretization(c.disc.rule, c.mesh.elem_dofs, c.mesh.node_xyz, c.disc.nglobal,
                            c.dir, kappa=kap)
        u = c.vec(71)
        for masked in (False, True):
            assert rel(host(c.op.apply(STIFF, dev(u), masked=masked)),
                       kd.apply(STIFF, u, masked=masked)) <= TOL, masked
            assert rel(host(c.op.diag(STIFF, masked=masked)), kd.diag(STIFF, masked=masked)) \
                <= TOL, masked
        check_iterates(c, STIFF, True, u * (1 - c.mesh.boundary), disc=kd)
        # a non-symmetric coefficient pattern within each element would expose
        # a wrong point order: check it differs from the unscaled operator
        assert rel(kd.apply(STIFF, u), c.disc.apply(STIFF, u)) > 1e-3
        c.op.set_coeff(None)
        assert rel(host(c.op.apply(STIFF, dev(u))), c.disc.apply(STIFF, u)) <= TOL
    finally:
        c.close()
