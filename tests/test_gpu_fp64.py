"""GPU parity of the FP64 form against the FP64 oracle (relative 2-norm).

Kernel level: one mu-mode product and the Tucker operator for every mu, on
shapes that span several workgroup tiles with ragged tails (tolerance 1e-13;
FP64 summation-order differences are ~1e-15).  Stepper level: Strang and
Lawson4 trajectories with the oracle stepping on the library's exponentials
(tolerance 1e-12, the FP64 target).
"""
import numpy as np
import pytest

import cgl_inputs as ci
from oracle import tensor
from tests._util import assert_close, log, make_plan, oracle_run, plan_ops, require_gpu

pytestmark = pytest.mark.gpu

SHAPES = [(150,), (64, 45), (130, 70), (20, 33, 17), (64, 64, 40), (3, 5, 4)]


def _random_plan(shape, seed):
    from paper_2403_02816_amd import cgl
    p = cgl.Plan(shape, ci.C0.coeffs, 0.01, precision="fp64")
    Es, Hs = [], []
    for mu, n in enumerate(shape):
        E = ci.random_complex((n, n), seed + 10 * mu) / np.sqrt(n)
        H = ci.random_complex((n, n), seed + 10 * mu + 1) / np.sqrt(n)
        p.set_exponentials(mu, E, H)
        Es.append(E)
        Hs.append(H)
    return p, Es, Hs


@pytest.mark.parametrize("shape", SHAPES)
def test_mode_product_every_mu(shape):
    torch = require_gpu()
    p, Es, Hs = _random_plan(shape, 100)
    U = ci.random_complex(shape, 7)
    x = p.to_device(U)
    out = torch.empty_like(x)
    for mu in range(len(shape)):
        for which, Ms in ((0, Es), (1, Hs)):
            log(f"mode_product shape={shape} mu={mu} which={which}")
            p.mode_product(mu, which, x, out)
            torch.cuda.synchronize()
            ref = tensor.mode_product(U, Ms[mu], mu)
            assert_close(p.to_host(out), ref, 1e-13, f"fp64 mode {shape} mu={mu} which={which}")
    p.destroy()


@pytest.mark.parametrize("shape", SHAPES)
def test_tucker_and_inplace(shape):
    torch = require_gpu()
    p, Es, Hs = _random_plan(shape, 200)
    U = ci.random_complex(shape, 8)
    x = p.to_device(U)
    out = torch.empty_like(x)
    p.tucker(0, x, out)
    torch.cuda.synchronize()
    assert_close(p.to_host(out), tensor.tucker(U, Es), 1e-13, f"fp64 tucker {shape}")
    p.tucker(1, x, x)  # in place
    torch.cuda.synchronize()
    assert_close(p.to_host(x), tensor.tucker(U, Hs), 1e-13, f"fp64 tucker in place {shape}")
    p.destroy()


def _traj_case(p, method, m, rk4_flow=False, use_run=False, check_every=0):
    torch = require_gpu()
    log(f"trajectory {p.name} {method} m={m} rk4={rk4_flow} run={use_run}")
    plan = make_plan(p, "fp64", rk4_flow=rk4_flow)
    u0 = ci.initial_state(p)
    u = plan.to_device(u0)
    if use_run:
        st = plan.run(method, u, m, check_every)
        assert st == 0
    elif method == "strang":
        plan.step_strang(u, m)
    else:
        plan.step_lawson4(u, m)
    torch.cuda.synchronize()
    assert plan.status() == 0
    E, H = plan_ops(plan)
    ref = oracle_run(p, u0, method, m, E, H, rk4_flow=rk4_flow)
    got = plan.to_host(u)
    plan.destroy()
    assert_close(got, ref, 1e-12, f"fp64 {p.name} {method} m={m}")


def test_c0_strang_full_trajectory():
    _traj_case(ci.C0, "strang", ci.C0.steps)


def test_c0_lawson4_trajectory():
    _traj_case(ci.C0, "lawson4", 50)


@pytest.mark.parametrize("shape", [(24, 24, 24), (19, 26, 21)])
def test_c1_shape_lawson4_trajectory(shape):
    p = ci.scaled(ci.C1, shape)
    _traj_case(p, "lawson4", 40, use_run=True, check_every=10)


def test_c2_shape_strang_rk4_trajectory():
    p = ci.scaled(ci.C2, (20, 22, 18))
    _traj_case(p, "strang", 30, use_run=True, check_every=7)


def test_d1_and_rk4_flow_for_cubic():
    p = ci.Problem("d1", (97,), ci.DIRICHLET, -10.0, 10.0, ci.C0.coeffs, 1e-2, 20, "strang", 9)
    _traj_case(p, "strang", 20)
    _traj_case(p, "strang", 20, rk4_flow=True)
    _traj_case(p, "lawson4", 20)


def test_graph_replay_equals_eager_bitwise():
    torch = require_gpu()
    p = ci.scaled(ci.C1, (20, 18, 22))
    plan = make_plan(p, "fp64")
    u0 = ci.initial_state(p)
    a = plan.to_device(u0)
    b = plan.to_device(u0)
    plan.step_lawson4(a, 12)
    assert plan.run("lawson4", b, 12, 5) == 0
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan.destroy()


def test_c1_full_size_one_step():
    torch = require_gpu()
    p = ci.C1
    plan = make_plan(p, "fp64")
    u0 = ci.initial_state(p)
    u = plan.to_device(u0)
    plan.step_lawson4(u, 2)
    torch.cuda.synchronize()
    E, H = plan_ops(plan)
    ref = oracle_run(p, u0, "lawson4", 2, E, H)
    assert_close(plan.to_host(u), ref, 1e-12, "C1 128^3 FP64 Lawson4 2 steps")
    plan.destroy()


def test_nonfinite_state_is_reported():
    torch = require_gpu()
    p = ci.scaled(ci.C0, (32, 32))
    plan = make_plan(p, "fp64")
    u0 = ci.initial_state(p)
    u0[5, 7] = np.nan
    u = plan.to_device(u0)
    assert plan.run("lawson4", u, 3, 1) == -5  # CGL_ENONFINITE
    plan.destroy()


def test_blowup_of_exact_cubic_flow_is_reported():
    torch = require_gpu()
    c = ci.Coeffs(1.0, 0.5, 0.0, 1.0, 0.3)  # a3 > 0: the cubic flow blows up for large |u|^2 tau
    p = ci.Problem("blow", (16, 16), ci.DIRICHLET, -5.0, 5.0, c, 0.5, 2, "strang", 3)
    plan = make_plan(p, "fp64")
    u0 = 3.0 * np.ones(p.n, dtype=np.complex128)
    u = plan.to_device(u0)
    assert plan.run("strang", u, 1, 1) == -6  # CGL_EBLOWUP
    plan.destroy()
