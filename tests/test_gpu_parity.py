"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Sizes span several work-groups with a ragged last one; the bar is the
normwise relative FP64 tolerance 1e-12 (apply, diagonal, CG iterates,
gradient) unless a test states otherwise with its reason.
"""
import numpy as np
import pytest

import synth
from oracle import adjoint, mixed
from oracle.assembled import assemble
from oracle.operators import MASS, STIFF, Discretization
from oracle.pcg import pcg
from tests.gpu_cases import TOL, Case, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    """Vector to the device: the oracle's [n, ncomp] becomes [ncomp, n]."""
    a = np.asarray(a)
    return torch.from_numpy(np.ascontiguousarray(a.T if a.ndim == 2 else a)).to("cuda")


def host(t):
    """Vector back to the oracle's layout [n, ncomp]."""
    torch.cuda.synchronize()
    a = t.cpu().numpy()
    return a.T if a.ndim == 2 else a


def host_array(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def grid_for(p):
    # E = 27 (ragged against 16, 7 and 4 elements per work-group) or 12
    return (3, 3, 3) if p <= 4 else (3, 2, 2)


@pytest.mark.parametrize("p", range(1, 9))
@pytest.mark.parametrize("bp", [1, 3, 5])
def test_apply_matches_oracle(bp, p):
    c = Case(bp, p, *grid_for(p), seed=p)
    try:
        u = c.vec(10 + p)
        for which in (MASS, STIFF):
            for masked in (False, True):
                w = host(c.op.apply(which, dev(u), masked=masked))
                ref = c.disc.apply(which, u, masked=masked)
                assert rel(w, ref) <= TOL, (which, masked, rel(w, ref))
    finally:
        c.close()


@pytest.mark.parametrize("bp,p,ncomp", [(2, 3, 3), (4, 4, 3), (6, 7, 3), (6, 5, 8), (5, 2, 2)])
def test_vector_components_match_oracle(bp, p, ncomp):
    c = Case(bp, p, *grid_for(p), seed=3, ncomp=ncomp)
    try:
        u = c.vec(20)
        which = MASS if bp <= 2 else STIFF
        w = host(c.op.apply(which, dev(u), masked=True))
        ref = c.disc.apply(which, u, masked=True)
        for k in range(ncomp):
            assert rel(w[:, k], ref[:, k]) <= TOL
    finally:
        c.close()


@pytest.mark.parametrize("p", range(1, 9))
def test_gauss_legendre_vector_components_every_order(p):
    # ncomp = 3 with Gauss-Legendre quadrature (BP2 and BP4 on one mesh): the
    # multi-component launch at every order, in both of its stage-3 forms
    # (point values staged in LDS for even p1, registers for odd p1) and the
    # per-component launches it falls back to at p = 8; the energies p.Ap of
    # all components come from the same launch
    c = Case(4, p, *grid_for(p), seed=30 + p, ncomp=3)
    try:
        u = c.vec(31)
        for which in (MASS, STIFF):
            for masked in (False, True):
                w = host(c.op.apply(which, dev(u), masked=masked))
                ref = c.disc.apply(which, u, masked=masked)
                for k in range(3):
                    assert rel(w[:, k], ref[:, k]) <= TOL, (which, masked, k)
        mask = 1 - c.mesh.boundary
        b = c.vec(32) * mask[:, None]
        rec = []
        pcg(lambda v: c.disc.apply(STIFF, v, masked=True), b,
            c.disc.jacobi_inverse(STIFF, masked=True), maxit=6, fixed_iters=True, record=rec)
        for k in (1, 6):
            x, _ = c.op.pcg_solve(dev(b), which=STIFF, maxit=k, fixed_iters=True)
            assert rel(host(x), rec[k - 1]) <= TOL, k
    finally:
        c.close()


@pytest.mark.parametrize("bp,p", [(1, 2), (1, 7), (3, 1), (3, 5), (3, 8), (5, 1), (5, 4), (5, 7), (5, 8)])
def test_diagonal_matches_oracle(bp, p):
    c = Case(bp, p, *grid_for(p), seed=4)
    try:
        for which in (MASS, STIFF):
            for masked in (False, True):
                d = host(c.op.diag(which, masked=masked))
                assert rel(d, c.disc.diag(which, masked=masked)) <= TOL
    finally:
        c.close()


def test_diagonal_equals_assembled_diagonal():
    c = Case(3, 3, 2, 2, 2, seed=5)
    try:
        A = assemble(c.disc, STIFF, masked=True)
        assert rel(host(c.op.diag(STIFF)), A.diagonal()) <= TOL
    finally:
        c.close()


def test_fp32_apply_matches_single_precision_oracle():
    c = Case(5, 7, 3, 2, 2, seed=6, fp32=True)
    try:
        u = c.vec(7) * (1 - c.mesh.boundary)
        w32 = host(c.op.apply(STIFF, dev(u.astype(np.float32))))
        ref32 = mixed.apply_stiff_f32(c.disc, u.astype(np.float32))
        ref64 = c.disc.apply(STIFF, u)
        # float32 rounding of G, D and the sums: a few ulp times the
        # contraction length, relative to the result's norm
        assert rel(w32, ref64) < 2e-6
        assert rel(w32, ref32) < 2e-6
    finally:
        c.close()


@pytest.mark.parametrize("p,ncomp", [(7, 1), (5, 2), (3, 3)])
def test_fp32_stiffness_apply_components(p, ncomp):
    # float32 rounding of G, D and the sums, relative to the result's norm
    c = Case(6 if ncomp > 1 else 5, p, 3, 2, 2, seed=80 + p, ncomp=ncomp, fp32=True)
    try:
        u = c.vec(81).astype(np.float32)
        w = host(c.op.apply(STIFF, dev(u)))
        ref = c.disc.apply(STIFF, u.astype(np.float64))
        if ncomp == 1:
            assert rel(w, ref) < 2e-6
        else:
            for k in range(ncomp):
                assert rel(w[:, k], ref[:, k]) < 2e-6
    finally:
        c.close()


def test_fp32_stiffness_apply_with_kappa():
    c = Case(5, 4, 3, 3, 2, seed=90, fp32=True)
    try:
        kap = synth.kappa_log(c.mesh.node_xyz, 91)
        c.op.set_coeff(torch.tensor(kap, device="cuda"))
        kd = Discretization(c.disc.rule, c.mesh.elem_dofs, c.mesh.node_xyz, c.disc.nglobal,
                            c.dir, kappa=kap)
        u = (c.vec(92) * (1 - c.mesh.boundary)).astype(np.float32)
        w = host(c.op.apply(STIFF, dev(u)))
        assert rel(w, kd.apply(STIFF, u.astype(np.float64))) < 2e-6
    finally:
        c.close()


def manufactured_rhs(c):
    f = synth.manufactured_f(c.mesh.global_coords())
    return c.disc.apply(MASS, f, masked=False) * c.disc.mask


@pytest.mark.parametrize("fuse", [3, 2, 1, 0])
@pytest.mark.parametrize("bp,p,ncomp", [(5, 1, 1), (5, 2, 1), (5, 4, 1), (5, 5, 1), (5, 6, 2),
                                         (5, 7, 1), (5, 7, 3), (5, 8, 2), (5, 5, 8), (3, 4, 1),
                                         (3, 6, 1), (1, 5, 1)])
def test_pcg_iterates_match_oracle_orders(bp, p, ncomp, fuse):
    # every order's thread plane (including planes that leave idle lanes in a
    # wave) and several components: the fused energy p.Ap drives alpha; with
    # fuse 1 the vector updates compute alpha and beta themselves (small
    # meshes), with fuse 2 the collocated stiffness operator of one component
    # also forms the direction p = z + beta p while it gathers (two launches
    # per iteration; several components keep the three-launch form), with
    # fuse 3 it takes beta from the finisher (four launches)
    from paper_2004_06722_amd._lib import BP_OPT_CG_FUSE
    c = Case(bp, p, *grid_for(p), seed=21, ncomp=ncomp)
    try:
        c.op.set_option(BP_OPT_CG_FUSE, fuse)
        which = MASS if bp == 1 else STIFF
        mask = (1 - c.mesh.boundary) if bp >= 3 else np.ones(c.disc.nglobal)
        b = c.vec(3) * (mask[:, None] if ncomp > 1 else mask)
        rec = []
        A = lambda v: c.disc.apply(which, v, masked=bp >= 3)
        pcg(A, b, c.disc.jacobi_inverse(which, masked=bp >= 3), maxit=8, fixed_iters=True,
            record=rec)
        for k in (1, 4, 8):
            x, st = c.op.pcg_solve(dev(b), which=which, maxit=k, fixed_iters=True)
            assert rel(host(x), rec[k - 1]) <= TOL, (k, rel(host(x), rec[k - 1]))
    finally:
        c.close()



@pytest.mark.parametrize("bp,p,sr", [(1, 4, False), (3, 3, False), (5, 5, False), (5, 3, True),
                                      (1, 3, True)])
def test_pcg_from_nonzero_initial_guess(bp, p, sr):
    # x holds x0 on entry: the first residual is b - A x0 (the operator on x0
    # before the loop; for BP1 the mass kernel and the stand-alone gather)
    c = Case(bp, p, *grid_for(p), seed=31)
    try:
        c.op.set_cg_variant(sr)
        which = MASS if bp == 1 else STIFF
        masked = bp >= 3
        mask = (1 - c.mesh.boundary) if masked else np.ones(c.disc.nglobal)
        b = c.vec(32) * mask
        x0 = c.vec(33) * mask
        rec = []
        pcg(lambda v: c.disc.apply(which, v, masked=masked), b,
            c.disc.jacobi_inverse(which, masked=masked), x0=x0, maxit=5, fixed_iters=True,
            record=rec)
        for k in (1, 5):
            x, st = c.op.pcg_solve(dev(b), x=dev(x0), which=which, maxit=k, fixed_iters=True)
            assert st["iters"] == k
            assert rel(host(x), rec[k - 1]) <= TOL, (k, rel(host(x), rec[k - 1]))
    finally:
        c.close()

@pytest.mark.parametrize("bp,p,ncomp", [(5, 3, 1), (5, 7, 1), (5, 4, 3), (3, 5, 1), (1, 4, 1),
                                         (5, 1, 2)])
def test_single_reduction_pcg_iterates_match_oracle(bp, p, ncomp):
    # the Chronopoulos-Gear recurrences against the oracle's standard PCG:
    # the same iterates up to rounding
    c = Case(bp, p, *grid_for(p), seed=23, ncomp=ncomp)
    try:
        c.op.set_cg_variant(True)
        which = MASS if bp == 1 else STIFF
        mask = (1 - c.mesh.boundary) if bp >= 3 else np.ones(c.disc.nglobal)
        b = c.vec(5) * (mask[:, None] if ncomp > 1 else mask)
        rec = []
        A = lambda v: c.disc.apply(which, v, masked=bp >= 3)
        pcg(A, b, c.disc.jacobi_inverse(which, masked=bp >= 3), maxit=8, fixed_iters=True,
            record=rec)
        for k in (1, 2, 5, 8):
            x, st = c.op.pcg_solve(dev(b), which=which, maxit=k, fixed_iters=True)
            assert st["iters"] == k
            assert rel(host(x), rec[k - 1]) <= TOL, (k, rel(host(x), rec[k - 1]))
        # tolerance mode: the same stopping iteration (+-1) and solution as standard
        xs, sts = c.op.pcg_solve(dev(b), which=which, rtol=1e-10, maxit=5000)
        c.op.set_cg_variant(False)
        x0, st0 = c.op.pcg_solve(dev(b), which=which, rtol=1e-10, maxit=5000)
        assert sts["converged"] and abs(sts["iters"] - st0["iters"]) <= 1
        assert rel(host(xs), host(x0)) <= 1e-9
    finally:
        c.close()


def test_pcg_iterates_match_oracle_config1():
    c = Case(5, 3, 4, 4, 4, seed=0)
    try:
        b = manufactured_rhs(c)
        rec = []
        pcg(lambda v: c.disc.apply(STIFF, v), b, c.disc.jacobi_inverse(STIFF), maxit=10,
            fixed_iters=True, record=rec)
        bd = dev(b)
        for k in (1, 2, 3, 5, 10):
            x, st = c.op.pcg_solve(bd, maxit=k, fixed_iters=True)
            assert st["iters"] == k
            assert rel(host(x), rec[k - 1]) <= TOL, (k, rel(host(x), rec[k - 1]))
    finally:
        c.close()


def test_two_launch_iteration_on_a_mid_size_mesh():
    # E = 12^3 at p = 7 (n = 593k): the operator's launch reduces a vector
    # table of 580 rows (more than the 8 rows per thread it requests first)
    # and the vector kernel an operator table of 1728 rows (several unrolled
    # batches); iterates against the oracle and against the five-launch form
    from paper_2004_06722_amd._lib import BP_OPT_CG_FUSE
    c = Case(5, 7, 12, 12, 12, seed=31)
    try:
        mask = 1 - c.mesh.boundary
        b = c.vec(33) * mask
        rec = []
        pcg(lambda v: c.disc.apply(STIFF, v, masked=True), b,
            c.disc.jacobi_inverse(STIFF, masked=True), maxit=3, fixed_iters=True, record=rec)
        xs = {}
        for fuse in (2, 3, 0):
            c.op.set_option(BP_OPT_CG_FUSE, fuse)
            x, st = c.op.pcg_solve(dev(b), maxit=3, fixed_iters=True)
            assert st["iters"] == 3
            xs[fuse] = host(x)
            assert rel(xs[fuse], rec[2]) <= TOL, (fuse, rel(xs[fuse], rec[2]))
        assert rel(xs[2], xs[0]) <= 1e-13 and rel(xs[3], xs[0]) <= 1e-13
    finally:
        c.close()


@pytest.mark.parametrize("fuse", [3, 2, 1, 0])
def test_indefinite_coefficient_reports_breakdown(fuse):
    # kappa = -2 at the quadrature points within 0.15 of the centre and 1
    # elsewhere makes the BP5 stiffness indefinite while its diagonal stays
    # positive on the free nodes, and for the smooth rhs M f the first step
    # has r.z > 0 and p.Ap < 0 (checked on the oracle below). Every CG form,
    # the two-launch one included, stops there with BP_ERR_BREAKDOWN and
    # x = 0; the fixed-count mode runs every iteration and reports it at the
    # end.
    import ctypes

    from oracle.geometry import quad_points
    from paper_2004_06722_amd import _lib
    c = Case(5, 3, 3, 3, 3, seed=66)
    try:
        xyz = quad_points(c.disc.rule, c.mesh.node_xyz)
        kap = np.where(((xyz - 0.5) ** 2).sum(-1) < 0.15 ** 2, -2.0, 1.0)
        kd = Discretization(c.disc.rule, c.mesh.elem_dofs, c.mesh.node_xyz, c.disc.nglobal,
                            c.dir, kappa=kap)
        f = synth.manufactured_f(c.mesh.global_coords())
        bh = c.disc.apply(MASS, f, masked=False) * c.disc.mask
        z = kd.jacobi_inverse(STIFF) * bh
        assert kd.diag(STIFF)[c.mesh.boundary == 0].min() > 0
        assert bh @ z > 0 and z @ kd.apply(STIFF, z) < 0
        c.op.set_option(_lib.BP_OPT_CG_FUSE, fuse)
        c.op.set_coeff(torch.from_numpy(np.ascontiguousarray(kap)).cuda())
        b = dev(bh)
        x = torch.zeros_like(b)
        lib = _lib.load()
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        for fixed, maxit in ((0, 50), (1, 6)):
            x.zero_()
            st = _lib.PcgStats()
            rc = lib.bp_pcg_solve(c.op._h, STIFF, ctypes.c_void_p(b.data_ptr()),
                                  ctypes.c_void_p(x.data_ptr()), 1e-8, maxit, fixed,
                                  ctypes.byref(st), stream)
            torch.cuda.synchronize()
            assert rc == _lib.BP_ERR_BREAKDOWN, (fixed, rc)
            if not fixed:
                assert st.iters == 0, st.iters
                assert float(torch.abs(x).max()) == 0.0
            else:
                assert st.iters == maxit
        # with the coefficient removed the solve converges
        c.op.set_coeff(None)
        _, st = c.op.pcg_solve(b, rtol=1e-10, maxit=500)
        assert st["converged"]
    finally:
        c.close()


@pytest.mark.parametrize("fuse", [3, 2, 1, 0])
def test_pcg_converged_solution_config1(fuse):
    import scipy.sparse.linalg as spla
    from paper_2004_06722_amd._lib import BP_OPT_CG_FUSE
    c = Case(5, 3, 4, 4, 4, seed=0)
    try:
        c.op.set_option(BP_OPT_CG_FUSE, fuse)
        b = manufactured_rhs(c)
        x, st = c.op.pcg_solve(dev(b), rtol=1e-14, maxit=5000)
        assert st["converged"] and st["rel_res"][0] <= 1e-14
        xo, info = pcg(lambda v: c.disc.apply(STIFF, v), b, c.disc.jacobi_inverse(STIFF),
                       rtol=1e-14, maxit=5000)
        inner = c.mesh.boundary == 0
        A = assemble(c.disc, STIFF).tocsr()[inner][:, inner]
        xd = np.zeros_like(b)
        xd[inner] = spla.spsolve(A.tocsc(), b[inner])
        xg = host(x)
        assert rel(xg, xd) <= TOL
        assert rel(xg, xo) <= TOL
        # tolerance mode: same stopping iteration as the oracle, +-1
        x8, st8 = c.op.pcg_solve(dev(b), rtol=1e-8, maxit=5000)
        _, info8 = pcg(lambda v: c.disc.apply(STIFF, v), b, c.disc.jacobi_inverse(STIFF),
                       rtol=1e-8, maxit=5000)
        assert abs(st8["iters"] - info8["iters"]) <= 1
        assert st8["rel_res"][0] <= 1e-8
    finally:
        c.close()


def test_mass_solve_bp1_matches_oracle():
    c = Case(1, 3, 3, 3, 2, seed=8)
    try:
        b = c.vec(0)
        x, st = c.op.pcg_solve(dev(b), which=MASS, rtol=1e-14, maxit=2000)
        xo, _ = pcg(lambda v: c.disc.apply(MASS, v, masked=False), b,
                    c.disc.jacobi_inverse(MASS, masked=False), rtol=1e-14, maxit=2000)
        assert rel(host(x), xo) <= TOL
    finally:
        c.close()


def test_vector_pcg_components_independent():
    c = Case(6, 3, 3, 3, 2, seed=9, ncomp=3)
    try:
        B = c.vec(0) * (1 - c.mesh.boundary)[:, None]
        x, st = c.op.pcg_solve(dev(B), maxit=6, fixed_iters=True)
        X, _ = pcg(lambda v: c.disc.apply(STIFF, v), B, c.disc.jacobi_inverse(STIFF),
                   maxit=6, fixed_iters=True)
        assert rel(host(x), X) <= TOL
    finally:
        c.close()


def test_mixed_precision_defect_correction():
    c = Case(5, 4, 4, 4, 4, seed=10, fp32=True)
    try:
        b = manufactured_rhs(c)
        x, st = c.op.pcg_solve_mixed(dev(b), outer_rtol=1e-10, inner_rtol=1e-5)
        xg = host(x)
        r = b - c.disc.apply(STIFF, xg)
        assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.2e-10
        assert st["outer"] >= 2 and st["converged"]
        x64, _ = mixed.solve_fp64(c.disc, b, 1e-12)
        assert rel(xg, x64) < 1e-8
    finally:
        c.close()


@pytest.mark.parametrize("ncomp", [1, 3])
def test_mixed_precision_reliable_updates(ncomp):
    # FP32 CG with FP64 residual replacement: FP64 accuracy in about the FP64
    # iteration count (the oracle's same algorithm and the FP64 solve decide)
    c = Case(5, 5, 4, 4, 4, seed=4, fp32=True, ncomp=ncomp)
    try:
        b1 = manufactured_rhs(c)
        b = np.stack([b1 * (1 + 0.5 * k) for k in range(ncomp)], axis=1) if ncomp > 1 else b1
        x, st = c.op.pcg_solve_mixed(dev(b), outer_rtol=1e-10, inner_rtol=1e-2,
                                     max_outer=100, max_inner=5000, reliable=True)
        xg = host(x)
        assert st["converged"] and st["outer"] >= 2
        x64, i64 = mixed.solve_fp64(c.disc, b1, 1e-10)
        xo, io = mixed.reliable_cg(c.disc, b1, rtol=1e-10, delta=1e-2)
        for k in range(ncomp):
            xk = xg[:, k] / (1 + 0.5 * k) if ncomp > 1 else xg
            r = b1 - c.disc.apply(STIFF, xk)
            assert np.linalg.norm(r) / np.linalg.norm(b1) <= 1.2e-10
            assert rel(xk, x64) < 1e-8
        # same algorithm as the oracle: FP32 rounding moves the count a little
        assert abs(st["iters"] - io["iters"]) <= 0.1 * io["iters"] + 3, (st["iters"], io["iters"])
        assert st["iters"] <= 1.25 * i64["iters"]
    finally:
        c.close()


def test_grad_kappa_matches_oracle():
    from oracle.geometry import quad_points
    c = Case(5, 5, 3, 2, 2, seed=11, ncomp=2)
    try:
        kap = synth.kappa_log(quad_points(c.disc.rule, c.mesh.node_xyz), 3)
        lam = c.vec(1) * (1 - c.mesh.boundary)[:, None]
        u = c.vec(2) * (1 - c.mesh.boundary)[:, None]
        g = host_array(c.op.grad_kappa(dev(lam), dev(u)))
        ref = adjoint.grad_kappa(c.disc, lam, u)
        assert rel(g, ref) <= TOL
        # kappa-scaled operator
        c.op.set_coeff(torch.from_numpy(np.ascontiguousarray(kap)).cuda())  # [nelem, q^3]
        c.disc.kappa = kap
        w = host(c.op.apply(STIFF, dev(u)))
        assert rel(w, c.disc.apply(STIFF, u)) <= TOL
        assert rel(host(c.op.diag(STIFF)), c.disc.diag(STIFF)) <= TOL
        c.op.set_coeff(None)
        c.disc.kappa = None
        assert rel(host(c.op.apply(STIFF, dev(u))), c.disc.apply(STIFF, u)) <= TOL
    finally:
        c.close()


# ---- properties that hold at any size ------------------------------------
def test_properties_symmetry_nullspace_volume():
    c = Case(5, 6, 3, 3, 2, seed=12)
    try:
        u, v = c.vec(1), c.vec(2)
        Au = host(c.op.apply(STIFF, dev(u)))
        Av = host(c.op.apply(STIFF, dev(v)))
        assert abs(v @ Au - u @ Av) <= 1e-13 * abs(v @ Au)
        one = np.ones(c.disc.nglobal)
        A1 = host(c.op.apply(STIFF, dev(one), masked=False))
        assert np.abs(A1).max() <= 1e-13 * np.abs(host(c.op.diag(STIFF, masked=False))).max()
        M1 = host(c.op.apply(MASS, dev(one), masked=False))
        assert abs(M1.sum() - 1.0) <= 1e-13
        X = c.mesh.global_coords()
        for l in range(3):
            AX = host(c.op.apply(STIFF, dev(X[:, l]), masked=False))
            for m in range(3):
                assert abs(X[:, m] @ AX - (l == m)) <= 1e-12
    finally:
        c.close()


# ---- edge cases and errors -------------------------------------------------
def test_single_element_and_zero_rhs():
    c = Case(5, 7, 1, 1, 1, seed=13, dirichlet=False)
    try:
        u = c.vec(3)
        assert rel(host(c.op.apply(STIFF, dev(u), masked=False)),
                   c.disc.apply(STIFF, u, masked=False)) <= TOL
    finally:
        c.close()
    c = Case(5, 3, 2, 2, 2, seed=13)
    try:
        x, st = c.op.pcg_solve(dev(np.zeros(c.disc.nglobal)), rtol=1e-8)
        assert st["iters"] == 0 and np.all(host(x) == 0)
        x, st = c.op.pcg_solve(dev(c.vec(1)), maxit=0)
        assert st["iters"] == 0
    finally:
        c.close()


def test_errors_are_reported():
    import paper_2004_06722_amd.bp as B
    from paper_2004_06722_amd import BpError
    xi, _ = B.rule(4, B.GLL)
    m = synth.brick_mesh(2, 1, 1, 3, xi, seed=None)
    with pytest.raises(BpError, match="BP_ERR_ARG"):
        B.Operator(3, 5, B.GLL, m.elem_dofs, m.node_xyz, m.nglobal)
    bad = m.elem_dofs.copy()
    bad[1, 5] = m.nglobal
    with pytest.raises(BpError, match="BP_ERR_MESH"):
        B.Operator(3, 4, B.GLL, bad, m.node_xyz, m.nglobal)
    xyz = m.node_xyz.copy()
    xyz[1, :, 0] = 1.5 - xyz[1, :, 0]
    with pytest.raises(BpError, match="element 1"):
        B.Operator(3, 4, B.GLL, m.elem_dofs, xyz, m.nglobal)
    with pytest.raises(BpError, match="BP_ERR_ARG"):
        B.Operator(9, 11, B.GL, np.zeros((1, 1000), np.int64), np.zeros((1, 1000, 3)), 1000)
    # the device set-up reports the smallest bad element, also on GL points
    m4 = synth.brick_mesh(4, 2, 1, 3, xi, seed=None)
    xyz = m4.node_xyz.copy()
    for e in (6, 3):
        xyz[e, :, 1] = -xyz[e, :, 1]
    with pytest.raises(BpError, match="element 3$"):
        B.Operator(3, 5, B.GL, m4.elem_dofs, xyz, m4.nglobal)
    xyz = m4.node_xyz.copy()
    xyz[7, 0, 2] = np.inf
    with pytest.raises(BpError, match="element 7$"):
        B.Operator(3, 4, B.GLL, m4.elem_dofs, xyz, m4.nglobal)
    op = B.Operator(3, 4, B.GLL, m.elem_dofs, m.node_xyz, m.nglobal, m.boundary)
    try:
        b = np.zeros(m.nglobal)
        b[np.nonzero(m.boundary == 0)[0][0]] = np.nan
        with pytest.raises(BpError, match="NONFINITE"):
            op.pcg_solve(dev(b))
        with pytest.raises(BpError, match="FP32"):
            op.apply(STIFF, dev(np.zeros(m.nglobal, np.float32)))
    finally:
        op.close()


@pytest.mark.parametrize("sr", [False, True])
def test_operator_timing_option(sr):
    # BP_OPT_TIME_APPLY: one event pair per operator launch of the loop (the
    # operator of the initial residual is outside it), summed into apply_ms;
    # the iterates are those of the untimed solve
    from paper_2004_06722_amd._lib import BP_OPT_TIME_APPLY
    c = Case(5, 3, 3, 3, 3, seed=41)
    try:
        c.op.set_cg_variant(sr)
        b = dev(c.vec(42) * (1 - c.mesh.boundary))
        x0, st0 = c.op.pcg_solve(b, maxit=6, fixed_iters=True)
        assert st0["apply_count"] == 0 and st0["apply_ms"] == 0.0
        c.op.set_option(BP_OPT_TIME_APPLY, 1)
        x1, st1 = c.op.pcg_solve(b, maxit=6, fixed_iters=True)
        # the single-reduction form skips the operator of the last fixed iteration
        assert st1["apply_count"] == (5 if sr else 6)
        assert 0.0 < st1["apply_ms"] < st1["ms"]
        assert rel(host(x1), host(x0)) <= 1e-14
        c.op.set_option(BP_OPT_TIME_APPLY, 0)
        _, st2 = c.op.pcg_solve(b, maxit=6, fixed_iters=True)
        assert st2["apply_count"] == 0
    finally:
        c.close()
