"""GPU parity of the collocated GLL operators at p = 9..15 (the top of the
order range of section 3, and of the single-GPU BK5 study of section 8):
assembled mass and stiffness apply, the element operators alone, the
diagonal, Jacobi-PCG iterates, components, FP32, Helmholtz and kappa, on
meshes of 2-4 elements (one element per work-group at these orders). The bar
is the FP64 normwise 1e-12 of the other parity tests."""
import numpy as np
import pytest

import synth
from oracle.operators import HELM, MASS, STIFF, Discretization
from oracle.pcg import pcg
from tests.gpu_cases import TOL, Case, rel
from tests.test_gpu_local import local_input, oracle_local, run_local
from tests.test_gpu_parity import dev, host, host_array

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("p", range(9, 16))
def test_high_order_apply_and_local_match_oracle(p):
    c = Case(5, p, 2, 1, 1, seed=80 + p)
    try:
        u = c.vec(81 + p)
        for which in (MASS, STIFF):
            for masked in (False, True):
                w = host(c.op.apply(which, dev(u), masked=masked))
                ref = c.disc.apply(which, u, masked=masked)
                assert rel(w, ref) <= TOL, (which, masked, rel(w, ref))
        uL = local_input(c, 82 + p)
        for which in (MASS, STIFF):
            assert rel(run_local(c.op, which, uL), oracle_local(c.disc, which, uL)) <= TOL
    finally:
        c.close()


@pytest.mark.parametrize("p", [9, 12, 15])
def test_high_order_diagonal_and_pcg_iterates(p):
    c = Case(5, p, 2, 2, 1, seed=90 + p)
    try:
        d = host_array(c.op.diag(STIFF))
        assert rel(d, c.disc.diag(STIFF)) <= TOL
        mask = 1 - c.mesh.boundary
        b = c.vec(91 + p) * mask
        rec = []
        pcg(lambda v: c.disc.apply(STIFF, v), b, c.disc.jacobi_inverse(STIFF), maxit=6,
            fixed_iters=True, record=rec)
        for k in (1, 6):
            x, _ = c.op.pcg_solve(dev(b), maxit=k, fixed_iters=True)
            assert rel(host(x), rec[k - 1]) <= TOL, (k, rel(host(x), rec[k - 1]))
    finally:
        c.close()


def test_high_order_vector_fp32_helmholtz_and_coefficient():
    # BP6 at p = 11 with three components
    c = Case(6, 11, 2, 1, 1, seed=95, ncomp=3)
    try:
        u = c.vec(96)
        w = host(c.op.apply(STIFF, dev(u)))
        ref = c.disc.apply(STIFF, u)
        for k in range(3):
            assert rel(w[:, k], ref[:, k]) <= TOL
    finally:
        c.close()
    # FP32 operator at p = 13 against the FP64 oracle (same bar as at low order)
    c = Case(5, 13, 2, 1, 1, seed=97, fp32=True)
    try:
        u = c.vec(98)
        w32 = c.op.apply(STIFF, torch.tensor(u, dtype=torch.float32, device="cuda"))
        torch.cuda.synchronize()
        assert rel(w32.cpu().numpy().astype(np.float64), c.disc.apply(STIFF, u)) <= 2e-6
    finally:
        c.close()
    # Helmholtz with beta at the points, and kappa, at p = 14
    c = Case(5, 14, 2, 1, 1, seed=99)
    try:
        u = c.vec(100)
        beta = np.random.default_rng(101).uniform(0.5, 3.0, size=(c.disc.E, c.q ** 3))
        c.op.set_helmholtz(0.0, torch.tensor(beta, device="cuda"))
        hd = Discretization(c.disc.rule, c.mesh.elem_dofs, c.mesh.node_xyz, c.disc.nglobal,
                            c.dir, beta=beta)
        assert rel(host(c.op.apply(HELM, dev(u))), hd.apply(HELM, u)) <= TOL
        kap = synth.kappa_log(c.mesh.node_xyz, 102)
        c.op.set_coeff(torch.tensor(kap, device="cuda"))
        kd = Discretization(c.disc.rule, c.mesh.elem_dofs, c.mesh.node_xyz, c.disc.nglobal,
                            c.dir, kappa=kap)
        assert rel(host(c.op.apply(STIFF, dev(u))), kd.apply(STIFF, u)) <= TOL
    finally:
        c.close()


def test_orders_outside_the_compiled_range_are_rejected():
    import paper_2004_06722_amd.bp as B
    from paper_2004_06722_amd import BpError
    xi, _ = B.rule(10, B.GLL)
    m = synth.brick_mesh(1, 1, 1, 9, xi, seed=None)
    with pytest.raises(BpError, match="BP_ERR_ARG"):   # GL q = p + 2 stops at p = 8
        B.Operator(9, 11, B.GL, m.elem_dofs, m.node_xyz, m.nglobal)
    c = Case(5, 9, 1, 1, 1, seed=1)
    try:                                                 # the gradient stops at p = 8
        z = torch.zeros(c.disc.nglobal, dtype=torch.float64, device="cuda")
        with pytest.raises(BpError, match="p <= 8"):
            c.op.grad_kappa(z, z)
    finally:
        c.close()
