"""Edge cases on the GPU: the largest direction a plan accepts (n = 4096)
beside the smallest (n = 3), zero-step calls, and the linear equation
(g = 0), where every step of either method is exactly the exponential
action e^{tau K} (eq. Strang and eq. lawson4 with g = 0)."""
import numpy as np
import pytest

import cgl_inputs as ci
from oracle import tensor
from tests._util import assert_close, log, require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,nmax", [("fp64", 4096), ("split", 512), ("split", 4096)])
def test_largest_and_smallest_direction(precision, nmax):
    """A direction of nmax points beside one of 3.  The FP64 form meets 1e-13
    up to the largest direction a plan accepts (4096).  The split form's FP32
    accumulation over ~3n/4 additions per output drifts like u sqrt(3n/4):
    it meets the 1e-6 bound in both measures up to n = 512 (the limit cgl.h
    states; measured at n = 1024: 7.2e-7 in the 2-norm but 1.25e-6 in the
    max-norm); at n = 4096 (1.45e-6, 2.5e-6) it is held to 3e-6, outside the
    stated range."""
    torch = require_gpu()
    from paper_2403_02816_amd import cgl
    shape = (nmax, 3)
    p = cgl.Plan(shape, ci.C0.coeffs, 0.01, precision=precision)
    M = []
    for mu, n in enumerate(shape):
        E = ci.random_complex((n, n), 70 + mu) / np.sqrt(n)
        H = ci.random_complex((n, n), 80 + mu) / np.sqrt(n)
        p.set_exponentials(mu, E, H)
        M.append(H)
    U = ci.random_complex(shape, 90)
    if precision == "split":
        U = U.astype(np.complex64).astype(np.complex128)
    x = p.to_device(U, dtype=p.stage_dtype)
    out = torch.empty_like(x)
    tol = 1e-13 if precision == "fp64" else (1e-6 if nmax <= 512 else 3e-6)
    for mu in range(2):
        p.mode_product(mu, 1, x, out)
        torch.cuda.synchronize()
        assert_close(p.to_host(out), tensor.mode_product(U, M[mu], mu), tol,
                     f"{precision} ({nmax}, 3) mode {mu}")
    p.tucker(1, x, out)
    torch.cuda.synchronize()
    assert_close(p.to_host(out), tensor.tucker(U, M), tol, f"{precision} ({nmax}, 3) tucker")
    p.destroy()


@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_zero_steps_leave_the_state_unchanged(precision):
    torch = require_gpu()
    from tests._util import make_plan
    p = ci.scaled(ci.C0, (20, 24))
    plan = make_plan(p, precision)
    u = plan.to_device(ci.initial_state(p))
    v = u.clone()
    plan.step_strang(u, 0)
    plan.step_lawson4(u, 0)
    assert plan.run("lawson4", u, 0) == 0
    torch.cuda.synchronize()
    assert torch.equal(u, v)
    plan.destroy()


@pytest.mark.parametrize("method", ["strang", "lawson4"])
def test_linear_equation_steps_are_the_exponential_action(method):
    torch = require_gpu()
    from paper_2403_02816_amd import cgl
    c = ci.Coeffs(1.0, 0.7, 0.3, 0.0, 0.0)  # g = 0
    n = (30, 26, 22)
    plan = cgl.Plan(n, c, 0.01, precision="fp64")
    plan.set_fd_operators(-10.0, 10.0, ci.DIRICHLET, c)
    u0 = ci.random_complex(n, 5)
    u = plan.to_device(u0)
    getattr(plan, f"step_{method}")(u, 3)
    torch.cuda.synchronize()
    H = [plan.get_operator(mu, 1) for mu in range(3)]
    E = [h @ h for h in H] if method == "lawson4" else [plan.get_operator(mu, 0) for mu in range(3)]
    ref = u0
    for _ in range(3):
        ref = tensor.tucker(ref, E)
    assert_close(plan.to_host(u), ref, 1e-13, f"linear {method}")
    plan.destroy()
