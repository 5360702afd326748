"""CPU checks of the C ABI: libbp.so loads without a GPU, exports every entry
point include/bp.h declares, and its host-only 1D rules are right."""
import os
import re
import subprocess

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bp.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bp_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2004_06722_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2004_06722_amd.build import build
        build()
    return _lib.load()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("bp_setup", "bp_apply", "bp_diag", "bp_pcg_solve", "bp_pcg_solve_mixed",
              "bp_set_coeff", "bp_grad_kappa", "bp_destroy", "bp_last_error", "bp_rule"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2004_06722_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(bp_\w+)", out))
    for n in declared_functions():
        assert n in exported, n
        assert hasattr(lib, n)
    # and nothing else: the C++ internals stay local
    functions = set(re.findall(r"\s[TW]\s(\S+)", out))
    assert functions == set(declared_functions()), sorted(functions - set(declared_functions()))[:5]
    # the binding declares exactly the header's functions
    assert sorted(_lib.SIGNATURES) == declared_functions()


def test_version_and_error_string(lib):
    assert lib.bp_version() >= 100
    assert isinstance(lib.bp_last_error(), bytes)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 9, 10, 16])
def test_library_gl_rule(lib, n):
    from paper_2004_06722_amd._lib import BP_QUAD_GL
    x, w = np.zeros(n), np.zeros(n)
    assert lib.bp_rule(n, BP_QUAD_GL, x.ctypes.data, w.ctypes.data) == 0
    xr, wr = npleg.leggauss(n)
    assert np.allclose(x, xr, atol=2e-15) and np.allclose(w, wr, atol=2e-15)


@pytest.mark.parametrize("n", [2, 3, 4, 8, 9, 16])
def test_library_gll_rule(lib, n):
    from paper_2004_06722_amd._lib import BP_QUAD_GLL
    x, w = np.zeros(n), np.zeros(n)
    assert lib.bp_rule(n, BP_QUAD_GLL, x.ctypes.data, w.ctypes.data) == 0
    assert x[0] == -1 and x[-1] == 1 and abs(w.sum() - 2) < 1e-14
    if n > 2:
        roots = np.sort(npleg.Legendre.basis(n - 1).deriv().roots().real)
        assert np.allclose(x[1:-1], roots, atol=1e-14)
    for k in range(2 * n - 2):   # exact to degree 2n-3
        assert abs(w @ x ** k - (0 if k % 2 else 2 / (k + 1))) < 1e-14


def test_rule_rejects_bad_arguments(lib):
    from paper_2004_06722_amd._lib import BP_ERR_ARG, BP_QUAD_GLL
    x = np.zeros(4)
    assert lib.bp_rule(1, BP_QUAD_GLL, x.ctypes.data, None) == BP_ERR_ARG
    assert b"GLL" in lib.bp_last_error()
    assert lib.bp_rule(4, 7, x.ctypes.data, None) == BP_ERR_ARG
