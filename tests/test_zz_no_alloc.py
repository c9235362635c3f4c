"""GPU test of the allocation-free Tucker entry point (cgl_tucker_noalloc),
called through the C ABI: on two calls in a row, the second on a smaller
grid, its output equals cgl_tucker's bit for bit (the same kernels and tile
shape; only where the intermediates live differs) and is within the
precision form's parity bound of the oracle's Tucker operator; in place as
well; a grid that does not fit the fixed scratch is refused with
CGL_ESCRATCH before any work is enqueued."""
import ctypes as C

import numpy as np
import pytest

import cgl_inputs as ci
from oracle import tensor
from tests._util import assert_close, log, require_gpu

pytestmark = pytest.mark.gpu


def _plan(shape, precision, seed):
    from paper_2403_02816_amd import cgl
    p = cgl.Plan(shape, ci.C0.coeffs, 0.01, precision=precision)
    Es = []
    for mu, n in enumerate(shape):
        E = ci.random_complex((n, n), seed + 10 * mu) / np.sqrt(n)
        H = ci.random_complex((n, n), seed + 10 * mu + 1) / np.sqrt(n)
        p.set_exponentials(mu, E, H)
        Es.append(E)
    return p, Es


@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_noalloc_tucker_equals_cgl_tucker_on_two_calls(precision):
    torch = require_gpu()
    from paper_2403_02816_amd import _lib as L
    lib = L.lib()
    tol = 1e-13 if precision == "fp64" else 1e-6
    for k, shape in enumerate([(96, 80, 40), (40, 36, 44), (130, 70)]):
        p, Es = _plan(shape, precision, 600 + 10 * k)
        U = ci.random_complex(shape, 31 + k)
        if precision == "split":
            U = U.astype(np.complex64).astype(np.complex128)
        x = p.to_device(U, dtype=p.stage_dtype)
        ref = torch.empty_like(x)
        p.tucker(0, x, ref)  # the plan's own buffers (and its tile choice)
        out = torch.full_like(x, float("nan"))
        st = lib.cgl_tucker_noalloc(p._h, 0, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()))
        assert st == 0, st
        torch.cuda.synchronize()
        log(f"noalloc {precision} {shape}: equal to cgl_tucker {torch.equal(out, ref)}")
        assert torch.equal(out, ref)
        assert_close(p.to_host(out), tensor.tucker(U, Es), tol, f"noalloc {precision} {shape}")
        y = x.clone()
        assert lib.cgl_tucker_noalloc(p._h, 0, C.c_void_p(y.data_ptr()), C.c_void_p(y.data_ptr())) == 0
        torch.cuda.synchronize()
        assert torch.equal(y, ref)
        p.destroy()


def test_noalloc_refuses_grids_beyond_its_scratch():
    torch = require_gpu()
    from paper_2403_02816_amd import _lib as L
    lib = L.lib()
    p, _ = _plan((160, 128, 128), "fp64", 700)  # 2.6M points x 16 bytes > 16 MiB
    x = torch.zeros(p.N, dtype=torch.complex128, device="cuda")
    out = torch.full_like(x, 3.0)
    st = lib.cgl_tucker_noalloc(p._h, 0, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()))
    torch.cuda.synchronize()
    assert st == L.ESCRATCH
    assert bool((out == 3.0).all())  # nothing was enqueued
    assert lib.cgl_tucker_noalloc(None, 0, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr())) == L.EINVAL
    p.destroy()
