"""GPU parity of the bake-off kernels on their own (bp_apply_local): the
unassembled element operators w_L = A_L u_L and w_L = B_L u_L against the
oracle's element-by-element sum factorisation, with no gather, scatter or
mask. Meshes span several work-groups with a ragged last one."""
import numpy as np
import pytest

import synth
from oracle.operators import MASS, STIFF, Discretization
from tests.gpu_cases import TOL, Case, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def local_input(c, seed, ncomp=1):
    """Seeded uniform[-1,1] element-local vectors [ncomp][E][p1^3]."""
    rng = np.random.default_rng(seed)
    p1 = c.p + 1
    return rng.uniform(-1.0, 1.0, size=(ncomp, c.disc.E, p1 ** 3))


def oracle_local(disc, which, uL):
    """[ncomp][E][p1^3] through the oracle's [E][k][j][i](...) layout."""
    p1 = disc.rule.p1
    ncomp = uL.shape[0]
    x = np.moveaxis(uL, 0, -1).reshape((disc.E, p1, p1, p1, ncomp))
    w = disc.stiff_local(x) if which == STIFF else disc.mass_local(x)
    return np.moveaxis(w.reshape(disc.E, p1 ** 3, ncomp), -1, 0)


def run_local(op, which, uL, dtype=torch.float64):
    w = op.apply_local(which, torch.from_numpy(np.ascontiguousarray(uL)).to("cuda", dtype))
    torch.cuda.synchronize()
    return w.cpu().numpy().astype(np.float64)


def grid_for(p):
    return (4, 4, 4) if p <= 2 else ((3, 3, 3) if p <= 4 else (3, 2, 2))


@pytest.mark.parametrize("p", range(1, 9))
@pytest.mark.parametrize("bp", [1, 3, 5])
def test_apply_local_matches_oracle(bp, p):
    c = Case(bp, p, *grid_for(p), seed=p + 40)
    try:
        uL = local_input(c, 500 + p)
        for which in (MASS, STIFF):
            w = run_local(c.op, which, uL)
            ref = oracle_local(c.disc, which, uL)
            assert rel(w, ref) <= TOL, (which, rel(w, ref))
    finally:
        c.close()


@pytest.mark.parametrize("bp,p,ncomp", [(6, 7, 3), (4, 3, 3), (4, 7, 3), (4, 6, 2), (2, 5, 2)])
def test_apply_local_vector_components(bp, p, ncomp):
    c = Case(bp, p, 3, 2, 2, seed=7, ncomp=ncomp)
    try:
        uL = local_input(c, 77, ncomp)
        for which in (MASS, STIFF):
            w = run_local(c.op, which, uL)
            assert rel(w, oracle_local(c.disc, which, uL)) <= TOL
    finally:
        c.close()


def test_apply_local_fp32_and_coefficient():
    c = Case(5, 6, 2, 2, 3, seed=3, fp32=True)
    try:
        uL = local_input(c, 31)
        ref = oracle_local(c.disc, STIFF, uL)
        # FP32: same 2e-6 bar as the assembled FP32 apply
        w32 = run_local(c.op, STIFF, uL.astype(np.float32), torch.float32)
        assert rel(w32, ref) <= 2e-6
        # kappa at the quadrature points scales G as in bp_apply
        kap = synth.kappa_log(c.mesh.node_xyz, 5)
        c.op.set_coeff(torch.tensor(kap, device="cuda"))
        disc_k = Discretization(c.disc.rule, c.mesh.elem_dofs, c.mesh.node_xyz,
                                c.disc.nglobal, c.dir, kappa=kap)
        w = run_local(c.op, STIFF, uL)
        assert rel(w, oracle_local(disc_k, STIFF, uL)) <= TOL
    finally:
        c.close()


def test_apply_local_single_element_and_errors():
    import paper_2004_06722_amd.bp as B
    c = Case(3, 4, 1, 1, 1, seed=2)
    try:
        uL = local_input(c, 9)
        for which in (MASS, STIFF):
            assert rel(run_local(c.op, which, uL), oracle_local(c.disc, which, uL)) <= TOL
        # aliased input and output: rejected by the library, not computed
        t = torch.zeros(c.disc.E * 125, dtype=torch.float64, device="cuda")
        rc = c.op._lib.bp_apply_local(c.op._h, STIFF, 0, B._ptr(t), B._ptr(t), B._stream())
        assert rc < 0 and b"alias" in c.op._lib.bp_last_error()
        with pytest.raises(ValueError):
            c.op.apply_local(STIFF, torch.zeros(7, dtype=torch.float64, device="cuda"))
    finally:
        c.close()
