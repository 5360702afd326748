"""GPU parity of the Helmholtz operator H = A + B_beta (eq. (hm2)): apply,
element-local apply, diagonal and Jacobi-PCG iterates against the oracle,
for a constant beta and for beta given at the quadrature points, on GLL
meshes (term fused into the stiffness kernel) and GL meshes (a second
kernel adding into w). Meshes span several work-groups with a ragged last
one; the bar is the FP64 normwise 1e-12."""
import numpy as np
import pytest

from oracle.operators import HELM, STIFF, Discretization
from oracle.pcg import pcg
from tests.gpu_cases import TOL, Case, rel
from tests.test_gpu_local import local_input, oracle_local, run_local
from tests.test_gpu_parity import dev, host, host_array

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def helm_disc(c, beta):
    return Discretization(c.disc.rule, c.mesh.elem_dofs, c.mesh.node_xyz, c.disc.nglobal,
                          c.dir, beta=beta)


def beta_field(c, seed):
    return np.random.default_rng(seed).uniform(0.5, 3.0, size=(c.disc.E, c.q ** 3))


def set_beta(c, beta):
    if np.ndim(beta) == 0:
        c.op.set_helmholtz(float(beta))
    else:
        c.op.set_helmholtz(0.0, torch.tensor(beta, device="cuda"))


@pytest.mark.parametrize("bp,p", [(5, 1), (5, 3), (5, 6), (5, 7), (5, 8),
                                  (3, 1), (3, 3), (3, 5), (3, 7), (3, 8)])
def test_helmholtz_apply_matches_oracle(bp, p):
    c = Case(bp, p, *((3, 3, 3) if p <= 4 else (3, 2, 2)), seed=60 + p)
    try:
        u = c.vec(61 + p)
        for beta in (1.7, beta_field(c, 62 + p)):
            set_beta(c, beta)
            hd = helm_disc(c, beta)
            for masked in (False, True):
                w = host(c.op.apply(HELM, dev(u), masked=masked))
                ref = hd.apply(HELM, u, masked=masked)
                assert rel(w, ref) <= TOL, (masked, rel(w, ref))
            d = host_array(c.op.diag(HELM))
            assert rel(d, hd.diag(HELM)) <= TOL
            uL = local_input(c, 63 + p)
            assert rel(run_local(c.op, HELM, uL), oracle_local_helm(hd, uL)) <= TOL
    finally:
        c.close()


def oracle_local_helm(disc, uL):
    p1 = disc.rule.p1
    x = np.moveaxis(uL, 0, -1).reshape((disc.E, p1, p1, p1, uL.shape[0]))
    w = disc.helm_local(x)
    return np.moveaxis(w.reshape(disc.E, p1 ** 3, uL.shape[0]), -1, 0)


def test_zero_beta_is_stiffness_and_beta_can_be_reset():
    # same kernel both times; only the order of the atomic adds may differ
    c = Case(5, 4, 3, 3, 3, seed=70)
    try:
        u = dev(c.vec(71))
        a = host(c.op.apply(STIFF, u))
        assert rel(host(c.op.apply(HELM, u)), a) <= 1e-15
        c.op.set_helmholtz(2.0)
        assert rel(host(c.op.apply(HELM, u)), a) > 1e-3
        c.op.set_helmholtz(0.0)
        assert rel(host(c.op.apply(HELM, u)), a) <= 1e-15
        # solves: without a beta term H uses the stiffness's inverse diagonal;
        # with one, its own (allocated when beta is set, computed at the first solve)
        b = u * torch.from_numpy(1.0 - c.mesh.boundary).cuda()
        xa, _ = c.op.pcg_solve(b, which=STIFF, maxit=4, fixed_iters=True)
        xh, _ = c.op.pcg_solve(b, which=HELM, maxit=4, fixed_iters=True)
        assert rel(host(xh), host(xa)) <= 1e-13
        c.op.set_helmholtz(2.0)
        xb, _ = c.op.pcg_solve(b, which=HELM, maxit=4, fixed_iters=True)
        assert rel(host(xb), host(xa)) > 1e-3
        c.op.set_helmholtz(0.0)
        xh, _ = c.op.pcg_solve(b, which=HELM, maxit=4, fixed_iters=True)
        assert rel(host(xh), host(xa)) <= 1e-13
    finally:
        c.close()


@pytest.mark.parametrize("bp,p,ncomp", [(5, 7, 1), (5, 3, 3), (3, 4, 1), (3, 7, 2), (3, 5, 3)])
def test_helmholtz_pcg_iterates_match_oracle(bp, p, ncomp):
    c = Case(bp, p, *((3, 3, 3) if p <= 4 else (3, 2, 2)), seed=72, ncomp=ncomp)
    try:
        beta = beta_field(c, 73)
        set_beta(c, beta)
        hd = helm_disc(c, beta)
        mask = 1 - c.mesh.boundary
        b = c.vec(74) * (mask[:, None] if ncomp > 1 else mask)
        rec = []
        pcg(lambda v: hd.apply(HELM, v), b, hd.jacobi_inverse(HELM), maxit=8,
            fixed_iters=True, record=rec)
        for k in (1, 4, 8):
            x, st = c.op.pcg_solve(dev(b), which=HELM, maxit=k, fixed_iters=True)
            assert rel(host(x), rec[k - 1]) <= TOL, (k, rel(host(x), rec[k - 1]))
    finally:
        c.close()


def test_helmholtz_without_dirichlet_converges():
    # beta > 0 makes H definite without boundary conditions (BP1-type mesh)
    c = Case(1, 5, 3, 2, 2, seed=75, dirichlet=False)
    try:
        c.op.set_helmholtz(4.0)
        hd = helm_disc(c, 4.0)
        b = c.vec(76)
        x, st = c.op.pcg_solve(dev(b), which=HELM, rtol=1e-13, maxit=2000)
        assert st["converged"]
        ref, info = pcg(lambda v: hd.apply(HELM, v, masked=False), b,
                        hd.jacobi_inverse(HELM, masked=False), rtol=1e-13, maxit=2000)
        assert rel(host(x), ref) <= 1e-11
    finally:
        c.close()


@pytest.mark.parametrize("sr,fuse", [(False, True), (False, False), (True, True)])
def test_indefinite_operator_reports_breakdown(sr, fuse):
    # H = A + beta B with beta = -300 is indefinite on this mesh (the smooth
    # modes have generalised eigenvalues near 3 pi^2 < 300) while diag(H)
    # stays positive, and for the smooth rhs M f the first step has r.z > 0
    # and p.Hp < 0 (checked on the oracle below). A tolerance solve stops
    # there, not at maxit, with BP_ERR_BREAKDOWN and x = x0 = 0; the
    # fixed-count mode runs every iteration and reports the breakdown at the
    # end.
    import ctypes

    import synth
    from oracle.operators import MASS
    from paper_2004_06722_amd import _lib
    c = Case(5, 3, 3, 3, 3, seed=66)
    try:
        beta = -300.0
        hd = helm_disc(c, beta)
        f = synth.manufactured_f(c.mesh.global_coords())
        bh = c.disc.apply(MASS, f, masked=False) * c.disc.mask
        z = hd.jacobi_inverse(HELM) * bh
        assert hd.diag(HELM)[c.mesh.boundary == 0].min() > 0
        assert bh @ z > 0 and z @ hd.apply(HELM, z) < 0
        c.op.set_cg_variant(sr)
        c.op.set_option(_lib.BP_OPT_CG_FUSE, 1 if fuse else 0)
        c.op.set_helmholtz(beta)
        b = dev(bh)
        x = torch.zeros_like(b)
        lib = _lib.load()
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        for fixed, maxit in ((0, 50), (1, 6)):
            x.zero_()
            st = _lib.PcgStats()
            rc = lib.bp_pcg_solve(c.op._h, HELM, ctypes.c_void_p(b.data_ptr()),
                                  ctypes.c_void_p(x.data_ptr()), 1e-8, maxit, fixed,
                                  ctypes.byref(st), stream)
            torch.cuda.synchronize()
            assert rc == _lib.BP_ERR_BREAKDOWN, (fixed, rc)
            if not fixed:
                assert st.iters == 0, st.iters
                assert float(torch.abs(x).max()) == 0.0
            else:
                assert st.iters == maxit
        # the operator stays usable: with beta > 0 the solve converges
        c.op.set_helmholtz(2.0)
        xs, st = c.op.pcg_solve(b, which=HELM, rtol=1e-10, maxit=500)
        assert st["converged"]
    finally:
        c.close()
