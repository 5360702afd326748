"""GPU parity of the mass operator on Gauss-Legendre points (BP1/BP2), whose
assembly w = Q^T w_L (section 4) runs as a fixed-order gather over the
transposed map instead of an atomic scatter: the stand-alone apply (element
kernel, then the gather), the PCG iteration (the gather fused into the
residual update) with one and several components, with and without a
Dirichlet mask, in FP32, in tolerance mode, and the bitwise repeatability that
the fixed order gives. The bar is the FP64 normwise 1e-12 of the other parity
tests; FP32 results are held to 2e-6 against the FP64 oracle (float32
rounding of the factors and sums, relative to the result's norm)."""
import numpy as np
import pytest

import synth
from oracle.operators import MASS
from oracle.pcg import pcg
from tests.gpu_cases import TOL, Case, rel
from tests.test_gpu_parity import dev, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("p", [1, 4, 7, 8])
def test_mass_apply_is_bitwise_repeatable(p):
    c = Case(1, p, 3, 3, 2, seed=40 + p)
    try:
        u = dev(c.vec(41 + p))
        w1 = c.op.apply(MASS, u, masked=False)
        w2 = c.op.apply(MASS, u, masked=False)
        torch.cuda.synchronize()
        assert torch.equal(w1, w2)
        assert rel(host(w1), c.disc.apply(MASS, c.vec(41 + p), masked=False)) <= TOL
        x1, _ = c.op.pcg_solve(u, which=MASS, maxit=5, fixed_iters=True)
        x2, _ = c.op.pcg_solve(u, which=MASS, maxit=5, fixed_iters=True)
        torch.cuda.synchronize()
        assert torch.equal(x1, x2)
    finally:
        c.close()


@pytest.mark.parametrize("p,ncomp,dirichlet", [(3, 3, False), (7, 2, False), (5, 1, True),
                                               (2, 4, True)])
def test_mass_pcg_iterates_match_oracle(p, ncomp, dirichlet):
    # the fused residual update reads component c of w_L at c * nelem * p1^3
    c = Case(1, p, 3, 2, 3, seed=50 + p, ncomp=ncomp, dirichlet=dirichlet)
    try:
        mask = (1 - c.mesh.boundary) if dirichlet else np.ones(c.disc.nglobal)
        b = c.vec(51) * (mask[:, None] if ncomp > 1 else mask)
        rec = []
        pcg(lambda v: c.disc.apply(MASS, v, masked=dirichlet), b,
            c.disc.jacobi_inverse(MASS, masked=dirichlet), maxit=6, fixed_iters=True, record=rec)
        for k in (1, 3, 6):
            x, st = c.op.pcg_solve(dev(b), which=MASS, maxit=k, fixed_iters=True)
            assert st["iters"] == k
            assert rel(host(x), rec[k - 1]) <= TOL, (k, rel(host(x), rec[k - 1]))
        # the stand-alone apply with the mask, every component
        u = c.vec(52)
        w = host(c.op.apply(MASS, dev(u), masked=dirichlet))
        assert rel(w, c.disc.apply(MASS, u, masked=dirichlet)) <= TOL
    finally:
        c.close()


def test_mass_pcg_tolerance_mode_two_components():
    # stops inside a chunk of queued iterations: the element kernel and the
    # fused update skip on the done flag together
    c = Case(2, 4, 3, 3, 3, seed=60, ncomp=2)
    try:
        b = c.vec(61)
        x, st = c.op.pcg_solve(dev(b), which=MASS, rtol=1e-9, maxit=500)
        _, info = pcg(lambda v: c.disc.apply(MASS, v, masked=False), b,
                       c.disc.jacobi_inverse(MASS, masked=False), rtol=1e-9, maxit=500)
        assert st["converged"] and abs(st["iters"] - info["iters"]) <= 1
        assert max(st["rel_res"][:2]) <= 1e-9
        # the iterate it stopped at is the oracle's iterate of that count
        xk, _ = pcg(lambda v: c.disc.apply(MASS, v, masked=False), b,
                    c.disc.jacobi_inverse(MASS, masked=False), maxit=st["iters"],
                    fixed_iters=True)
        assert rel(host(x), xk) <= TOL
    finally:
        c.close()


def test_fp32_mass_apply_matches_oracle():
    c = Case(1, 6, 3, 2, 2, seed=70, ncomp=2, fp32=True)
    try:
        u = c.vec(71).astype(np.float32)
        w32 = host(c.op.apply(MASS, dev(u), masked=False))
        ref = c.disc.apply(MASS, u.astype(np.float64), masked=False)
        # float32 rounding of B~, J^ and the sums, relative to the result's norm
        assert rel(w32, ref) < 2e-6
    finally:
        c.close()



def test_mass_gather_with_unreferenced_nodes():
    # nglobal may exceed the ids the elements use: the trailing nodes have an
    # empty slot range (off[v] = off[v + 1] = nelem p1^3), read nothing that
    # counts and get w = 0; the other nodes are unchanged
    import paper_2004_06722_amd.bp as B
    c = Case(1, 3, 2, 2, 2, seed=95)
    try:
        xi, _ = B.rule(4, B.GLL)
        lm = synth.brick_mesh(2, 2, 2, 3, xi, 95)
        n = c.disc.nglobal
        with B.Operator(3, 5, B.GL, lm.elem_dofs, lm.node_xyz, n + 3) as op:
            u = np.concatenate([c.vec(96), [1.0, -2.0, 3.0]])
            w = host(op.apply(MASS, dev(u), masked=False))
            assert np.all(w[n:] == 0.0)
            assert rel(w[:n], c.disc.apply(MASS, u[:n], masked=False)) <= TOL
            d = host(op.diag(MASS, masked=False))
            assert np.all(d[n:] == 0.0)
            x, st = op.pcg_solve(dev(u * np.r_[np.ones(n), np.zeros(3)]), which=MASS, maxit=4,
                                 fixed_iters=True)
            rec = []
            pcg(lambda v: c.disc.apply(MASS, v, masked=False), u[:n],
                c.disc.jacobi_inverse(MASS, masked=False), maxit=4, fixed_iters=True, record=rec)
            xh = host(x)
            assert np.all(xh[n:] == 0.0)
            assert rel(xh[:n], rec[-1]) <= TOL
    finally:
        c.close()
