"""CPU tests of the C-ABI library: it loads, exports every declared symbol,
and its host numerics (FD operator, Pade exponential, argument checks) agree
with the oracle.  No device work is started here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import cgl_inputs as ci
from oracle import operators as ops

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2403_02816_amd import _lib as L
    return L


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "cgl.h")).read()
    return sorted(set(re.findall(r"\b(cgl_[a-z0-9_]+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    L = _lib()
    lib = L.lib()
    syms = _declared_symbols()
    assert "cgl_plan" in syms and "cgl_run" in syms and len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s
        assert s in L.SIGNATURES, f"binding lacks {s}"


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("n,d", [(7, 1), (64, 2), (33, 3)])
def test_fd_operator_matches_oracle(bc, n, d):
    from paper_2403_02816_amd import cgl
    c = ci.CQ.as_tuple()
    A = cgl.fd_operator(n, -15.0, 15.0, bc, c, d)
    ref = ops.operator_A(n, -15.0, 15.0, bc, c, d)
    assert np.abs(A - ref).max() <= 1e-15 * np.abs(ref).max()


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("n,t", [(16, 1e-2), (128, 5e-3), (64, 0.5), (200, 2e-3)])
def test_pade_expm_matches_closed_form(bc, n, t):
    from paper_2403_02816_amd import cgl
    c = ci.CQ.as_tuple()
    A = ops.operator_A(n, -15.0, 15.0, bc, c, 3)
    E = cgl.expm(A, t)
    ref = ops.exp_closed_form(n, -15.0, 15.0, bc, c, 3, t)
    assert np.linalg.norm(E - ref) / np.linalg.norm(ref) < 1e-14


def test_pade_expm_general_complex_matrix_vs_scipy():
    from paper_2403_02816_amd import cgl
    A = ci.random_complex((23, 23), 77) * 2.0
    E = cgl.expm(A, 1.3)
    ref = ops.exp_scipy(A, 1.3)
    assert np.linalg.norm(E - ref) / np.linalg.norm(ref) < 1e-13


def test_plan_argument_errors_are_reported_before_device_work():
    L = _lib()
    lib = L.lib()
    h = C.c_void_p()
    c = L.Coeffs(1.0, 0.5, 0.1, -1.0, 1.0, 0.0, 0.0)
    n3 = (C.c_int64 * 3)(8, 8, 8)
    assert lib.cgl_plan(None, 3, n3, C.byref(c), 0.01, 0, 0, None) == L.EINVAL
    assert lib.cgl_plan(C.byref(h), 0, n3, C.byref(c), 0.01, 0, 0, None) == L.EINVAL
    assert lib.cgl_plan(C.byref(h), 4, n3, C.byref(c), 0.01, 0, 0, None) == L.EINVAL
    assert lib.cgl_plan(C.byref(h), 3, n3, C.byref(c), 0.0, 0, 0, None) == L.EINVAL
    assert lib.cgl_plan(C.byref(h), 3, n3, C.byref(c), -1.0, 0, 0, None) == L.EINVAL
    assert lib.cgl_plan(C.byref(h), 3, n3, C.byref(c), 0.01, 7, 0, None) == L.EINVAL
    assert lib.cgl_plan(C.byref(h), 3, n3, C.byref(c), 0.01, 0, 1, None) == L.EINVAL  # master needs split
    small = (C.c_int64 * 3)(8, 2, 8)
    assert lib.cgl_plan(C.byref(h), 3, small, C.byref(c), 0.01, 0, 0, None) == L.EINVAL
    bad = L.Coeffs(0.0, 0.5, 0.1, -1.0, 1.0, 0.0, 0.0)  # a1 must be positive
    assert lib.cgl_plan(C.byref(h), 3, n3, C.byref(bad), 0.01, 0, 0, None) == L.EINVAL
    assert h.value is None
    for fn, args in (("cgl_step_strang", (None, None, 1)), ("cgl_step_lawson4", (None, None, 1)),
                     ("cgl_run", (None, 0, None, 1, 1)), ("cgl_tucker", (None, 0, None, None)),
                     ("cgl_status", (None,)), ("cgl_get_operator", (None, 0, 0, None))):
        assert getattr(lib, fn)(*args) == L.EINVAL, fn
    lib.cgl_destroy(None)
    assert lib.cgl_strerror(L.EBLOWUP).decode().startswith("exact cubic or quintic flow")
    # the RK4 sub-flow and the three-term splitting exclude each other
    assert lib.cgl_plan(C.byref(h), 3, n3, C.byref(c), 0.01, 0, 2 | 4, None) == L.EINVAL
    assert lib.cgl_plan(C.byref(h), 3, n3, C.byref(c), 0.01, 0, 8, None) == L.EINVAL
    assert lib.cgl_step(None, 2, None, 1) == L.EINVAL


def test_fd_operator_argument_errors():
    L = _lib()
    lib = L.lib()
    c = L.Coeffs(1.0, 0.5, 0.1, -1.0, 1.0, 0.0, 0.0)
    out = (C.c_double * 2)()
    assert lib.cgl_fd_operator(2, 0.0, 1.0, 0, C.byref(c), 2, out) == L.EINVAL
    assert lib.cgl_fd_operator(5, 1.0, 0.0, 0, C.byref(c), 2, out) == L.EINVAL
    assert lib.cgl_fd_operator(5, 0.0, 1.0, 3, C.byref(c), 2, out) == L.EINVAL


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("lo,hi", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("n,d", [(9, 1), (64, 2), (33, 3)])
def test_fd_operator_ex_matches_oracle(order, lo, hi, n, d):
    """cgl_fd_operator_ex against the oracle's matrices written from the
    displays of Sections 4.1.1 and 4.2 (orders 2 and 4, every pair of ends)."""
    from paper_2403_02816_amd import cgl
    c = ci.PAPER_CUBIC.as_tuple()
    A = cgl.fd_operator_ex(n, 0.0, 100.0, lo, hi, order, c, d)
    ref = ops.operator_A_fd(n, 0.0, 100.0, lo, hi, order, c, d)
    assert np.abs(A - ref).max() <= 4e-15 * np.abs(ref).max()
    if order == 2 and lo == hi:  # the plain builder's operators are the same
        assert np.array_equal(A, cgl.fd_operator(n, 0.0, 100.0, lo, c, d))


def test_fd_operator_ex_argument_errors():
    L = _lib()
    lib = L.lib()
    c = L.Coeffs(1.0, 0.5, 0.1, -1.0, 1.0, 0.0, 0.0)
    out = (C.c_double * 200)()
    assert lib.cgl_fd_operator_ex(5, 0.0, 1.0, 0, 0, 4, C.byref(c), 2, out) == L.EINVAL  # n < 6
    assert lib.cgl_fd_operator_ex(8, 0.0, 1.0, 0, 0, 3, C.byref(c), 2, out) == L.EINVAL
    assert lib.cgl_fd_operator_ex(8, 0.0, 1.0, 2, 0, 2, C.byref(c), 2, out) == L.EINVAL
    assert lib.cgl_fd_operator_ex(8, 1.0, 0.0, 0, 1, 2, C.byref(c), 2, out) == L.EINVAL
    assert lib.cgl_fd_operator_ex(8, 0.0, 1.0, 0, 1, 2, None, 2, out) == L.EINVAL
    assert lib.cgl_fd_operator_ex(8, 0.0, 1.0, 0, 1, 2, C.byref(c), 2, None) == L.EINVAL
