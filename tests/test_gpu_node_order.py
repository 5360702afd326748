"""GPU parity of the library's internal node order (element-interior nodes in
per-element blocks, written with plain stores) against the oracle and against
the caller's order (BP_SETUP_CALLER_ORDER), and its fallback when the map
shares an element-interior slot. Bar: normwise relative 1e-12."""
import numpy as np
import pytest

import synth
import paper_2004_06722_amd.bp as B
from oracle.operators import MASS, STIFF, Discretization
from oracle.pcg import pcg
from oracle.quadrature import bp_rule
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


@pytest.mark.parametrize("caller_order", [False, True])
@pytest.mark.parametrize("bp,p,ncomp,scramble", [(5, 7, 1, None), (5, 2, 2, 31), (3, 4, 1, None),
                                                 (1, 5, 3, 32), (5, 8, 1, 33), (1, 7, 1, None),
                                                 (1, 7, 3, None)])
def test_both_node_orders_match_the_oracle(bp, p, ncomp, scramble, caller_order):
    c = Case(bp, p, *((3, 3, 3) if p <= 4 else (3, 2, 2)), seed=p, ncomp=ncomp,
             scramble=scramble, caller_order=caller_order)
    try:
        which = MASS if bp == 1 else STIFF
        masked = bp >= 3
        u = c.vec(70)
        for wh in (MASS, STIFF):
            assert rel(host(c.op.apply(wh, dev(u), masked=masked)),
                       c.disc.apply(wh, u, masked=masked)) <= TOL, wh
        assert rel(host(c.op.diag(which, masked=masked)), c.disc.diag(which, masked=masked)) <= TOL
        mask = (1 - c.mesh.boundary) if masked else np.ones(c.disc.nglobal)
        b = u * (mask[:, None] if ncomp > 1 else mask)
        x0 = c.vec(71) * (mask[:, None] if ncomp > 1 else mask)
        rec = []
        pcg(lambda v: c.disc.apply(which, v, masked=masked), b,
            c.disc.jacobi_inverse(which, masked=masked), x0=x0, maxit=6, fixed_iters=True,
            record=rec)
        bd = dev(b)
        x, st = c.op.pcg_solve(bd, x=dev(x0), which=which, maxit=6, fixed_iters=True)
        assert rel(host(x), rec[-1]) <= TOL
        # the right-hand side is left as it was
        assert np.array_equal(host(bd), b)
    finally:
        c.close()


def test_shared_interior_slot_falls_back_to_atomic_assembly():
    # a map whose element-interior slot names a node of another element's
    # interior: the interior nodes are not owned by one element, so the
    # library must keep adding them atomically (a plain store would lose one
    # of the two contributions)
    p = 4
    rule = bp_rule(5, p)
    xi, _ = B.rule(p + 1, B.GLL)
    om = synth.brick_mesh(2, 2, 1, p, rule.xi, seed=2)
    lm = synth.brick_mesh(2, 2, 1, p, xi, seed=2)
    ed = om.elem_dofs.copy()
    l = 1 + (p + 1) * (1 + (p + 1) * 1)          # local (1, 1, 1): an interior slot
    ed[3, l] = ed[0, l]
    disc = Discretization(rule, ed, om.node_xyz, om.nglobal, None)
    op = B.Operator(p, p + 1, B.GLL, ed, lm.node_xyz, lm.nglobal, None)
    try:
        u = synth.rhs_uniform(om.nglobal, 5)
        for wh in (MASS, STIFF):
            assert rel(host(op.apply(wh, dev(u), masked=False)),
                       disc.apply(wh, u, masked=False)) <= TOL, wh
        assert rel(host(op.diag(STIFF, masked=False)), disc.diag(STIFF, masked=False)) <= TOL
    finally:
        op.close()


def test_fp32_and_mixed_solve_in_internal_order():
    c = Case(5, 5, 3, 3, 2, seed=72, fp32=True)
    try:
        u = (c.vec(73) * (1 - c.mesh.boundary)).astype(np.float32)
        assert rel(host(c.op.apply(STIFF, dev(u))), c.disc.apply(STIFF, u.astype(np.float64))) \
            < 2e-6
        f = synth.manufactured_f(c.mesh.global_coords())
        b = c.disc.apply(MASS, f, masked=False) * c.disc.mask
        for reliable in (False, True):
            x, st = c.op.pcg_solve_mixed(dev(b), outer_rtol=1e-10, inner_rtol=1e-3,
                                         max_outer=50, max_inner=5000, reliable=reliable)
            r = b - c.disc.apply(STIFF, host(x))
            assert st["converged"] and np.linalg.norm(r) / np.linalg.norm(b) <= 1.2e-10
    finally:
        c.close()
