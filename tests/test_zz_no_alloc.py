"""bp_pcg_solve_static, the solve for callers that cannot allocate, against
bp_pcg_solve: the same iterates and solution from a workspace held in one
static device array, over two calls in a row (the second on a smaller
operator, so stale contents of the array must not leak into it), and a clear
error for an operator beyond the array's size."""
import ctypes

import numpy as np
import pytest

from oracle.operators import MASS, STIFF
from oracle.pcg import pcg
from tests.gpu_cases import TOL, Case, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    a = np.asarray(a)
    return torch.from_numpy(np.ascontiguousarray(a.T if a.ndim == 2 else a)).to("cuda")


def _solve(c, name, which, b, maxit, fixed, rtol=1e-10):
    from paper_2004_06722_amd import _lib
    lib = _lib.load()
    x = torch.zeros_like(b)
    st = _lib.PcgStats()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(lib, name)(c.op._h, which, ctypes.c_void_p(b.data_ptr()),
                            ctypes.c_void_p(x.data_ptr()), rtol, maxit, 1 if fixed else 0,
                            ctypes.byref(st), stream)
    torch.cuda.synchronize()
    a = x.cpu().numpy()
    return rc, (a.T if a.ndim == 2 else a), st


def _compare(c, which, masked, b_host):
    b = _dev(b_host)
    rec = []
    pcg(lambda v: c.disc.apply(which, v, masked=masked), b_host,
        c.disc.jacobi_inverse(which, masked=masked), maxit=6, fixed_iters=True, record=rec)
    for fixed, maxit in ((True, 6), (False, 2000)):
        rc0, x0, st0 = _solve(c, "bp_pcg_solve", which, b, maxit, fixed)
        rc1, x1, st1 = _solve(c, "bp_pcg_solve_static", which, b, maxit, fixed)
        assert rc0 == 0 and rc1 == 0, (rc0, rc1)
        assert st1.iters == st0.iters, (st1.iters, st0.iters)
        assert rel(x1, x0) <= TOL, rel(x1, x0)
        if fixed:
            assert rel(x1, rec[-1]) <= TOL
        else:
            assert st1.converged == 1 and st1.rel_res[0] <= 1e-10


def test_static_solve_matches_the_allocating_solve_twice():
    # first call: 3 components of BP5 at p = 5; second: a smaller scalar BP5
    # and a Gauss-Legendre mass solve (its own element-local buffer)
    for bp, p, grid, ncomp in ((5, 5, (3, 2, 2), 3), (5, 3, (2, 2, 2), 1), (1, 3, (2, 2, 1), 1)):
        c = Case(bp, p, *grid, seed=90 + p, ncomp=ncomp)
        try:
            which = MASS if bp == 1 else STIFF
            masked = bp >= 3
            mask = (1 - c.mesh.boundary) if masked else np.ones(c.disc.nglobal)
            b = c.vec(91) * (mask[:, None] if ncomp > 1 else mask)
            _compare(c, which, masked, b)
        finally:
            c.close()


def test_static_solve_rejects_an_operator_beyond_its_workspace():
    from paper_2004_06722_amd import _lib
    # p = 7 on 16 x 16 x 8 elements with 4 components: 727,833 nodes x 4,
    # three vectors of 23 MB each exceed the 64 MiB array
    c = Case(5, 7, 16, 16, 8, seed=1, ncomp=4)
    try:
        b = torch.zeros((4, c.disc.nglobal), dtype=torch.float64, device="cuda")
        rc, _, _ = _solve(c, "bp_pcg_solve_static", STIFF, b, 3, True)
        assert rc == _lib.BP_ERR_ARG
        msg = _lib.load().bp_last_error().decode()
        assert "bytes of workspace" in msg and "bp_pcg_solve" in msg
        # the allocating entry point still serves it
        rc, _, st = _solve(c, "bp_pcg_solve", STIFF, b, 3, True)
        assert rc == 0 and st.iters == 3
    finally:
        c.close()
