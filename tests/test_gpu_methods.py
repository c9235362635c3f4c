"""GPU parity of the further steppers and operators against the FP64 oracle:

* split4 (eq. Richardson) and Lawson2b (eq. lawson2b): FP64 trajectories
  within 1e-12 (relative 2-norm and max-norm) of the oracle stepping on the
  plan's exported exponentials, exact-cubic and RK4 sub-flows, d = 1..3;
  split-form one-step gates within 1e-6 at the C0/C1/C2 shapes and on the
  full 256^3 grid, with and without the FP64 master state; the paired and
  two-action Lawson2b schedules bit for bit; graph replay = eager;
* strang_3t / split4_3t (Section 4.3, exact cubic and quintic flows);
* batched plans: split4 / Lawson2b one-step gates per instance and FP64
  batched trajectories;
* the paper's fourth-order operators: FP64 trajectories on the Table 1 shape
  (256^2 Dirichlet) and the Table 3 shape (128^3, Dirichlet on the faces
  through 0 and Neumann on the others) within 1e-12 of the oracle, and the
  observed order of split4 on the Table 1 workload.
"""
import numpy as np
import pytest

import cgl_inputs as ci
from oracle import metrics, steppers
from tests._util import assert_close, errors, log, plan_ops, require_gpu

pytestmark = pytest.mark.gpu


def _c64(u):
    return u.astype(np.complex64).astype(np.complex128)


def _plan(p, precision, **kw):
    from paper_2403_02816_amd import cgl
    plan = cgl.Plan(p.n, p.coeffs, p.tau, precision=precision, **kw)
    plan.set_problem_operators(p)
    return plan


def _oracle(p, u0, method, m, E, H, rk4_flow=False):
    nl = steppers.CGLNonlinearity(p.coeffs.as_tuple(), force_rk4=rk4_flow)
    u, bad = steppers.run(u0, steppers.make_step(method, E, H, p.tau, nl), m)
    assert not bad
    return u


def _fp64_traj(p, method, m, lib_method=None, use_run=True, **kw):
    torch = require_gpu()
    plan = _plan(p, "fp64", **{k: v for k, v in kw.items() if k in ("rk4_flow", "three_term")})
    u0 = ci.initial_state(p)
    u = plan.to_device(u0)
    lm = lib_method or method
    if use_run:
        assert plan.run(lm, u, m, max(1, m // 3)) == 0
    else:
        plan.step(lm, u, m)
    torch.cuda.synchronize()
    assert plan.status() == 0
    E, H = plan_ops(plan)
    ref = _oracle(p, u0, method, m, E, H, rk4_flow=kw.get("rk4_flow", False))
    got = plan.to_host(u)
    plan.destroy()
    return assert_close(got, ref, 1e-12, f"fp64 {p.name} {method} m={m}")


CASES_2D = ci.scaled(ci.C0, (40, 36))
CASES_3D = ci.scaled(ci.C1, (20, 18, 22))
CASES_1D = ci.Problem("d1", (97,), ci.DIRICHLET, -10.0, 10.0, ci.C0.coeffs, 1e-2, 20, "split4", 9)


@pytest.mark.parametrize("method", ["split4", "lawson2"])
def test_fp64_trajectories(method):
    _fp64_traj(CASES_2D, method, 30)
    _fp64_traj(CASES_3D, method, 12)  # cubic-quintic: RK4 sub-flow
    _fp64_traj(CASES_1D, method, 10, use_run=False)
    _fp64_traj(ci.scaled(ci.C2, (18, 20, 16)), method, 8)


def test_fp64_split4_with_rk4_flow_for_the_cubic_equation():
    _fp64_traj(CASES_2D, "split4", 20, rk4_flow=True)


@pytest.mark.parametrize("method,lib", [("strang_3t", "strang"), ("split4_3t", "split4")])
def test_fp64_three_term_schemes(method, lib):
    _fp64_traj(CASES_3D, method, 12, lib_method=lib, three_term=True)
    _fp64_traj(ci.Problem("cq2d", (33, 29), ci.DIRICHLET, -8.0, 8.0, ci.CQ, 5e-3, 0, method, 6),
               method, 15, lib_method=lib, three_term=True)


def _split_gate(p, method, master=False, three_term=False, lib=None):
    torch = require_gpu()
    kw = {"master": master}
    if three_term:
        kw["three_term"] = True
    plan = _plan(p, "split", **kw)
    u0 = ci.initial_state(p)
    if not master:
        u0 = _c64(u0)
    u = plan.to_device(u0)
    plan.step(lib or method, u, 1)
    torch.cuda.synchronize()
    assert plan.status() == 0
    E, H = plan_ops(plan)
    ref = _oracle(p, u0, method, 1, E, H)
    got = plan.to_host(u)
    plan.destroy()
    return assert_close(got, ref, 1e-6, f"split {p.name} {method} master={master}")


@pytest.mark.parametrize("method", ["split4", "lawson2"])
def test_split_one_step_gates(method):
    _split_gate(ci.C0, method)
    _split_gate(ci.scaled(ci.C1, (40, 36, 44)), method)
    _split_gate(ci.scaled(ci.C1, (40, 36, 44)), method, master=True)
    _split_gate(ci.scaled(ci.C2, (48, 40, 52)), method)
    _split_gate(CASES_1D, method)
    _split_gate(ci.scaled(ci.C0, (256, 256)), method)


@pytest.mark.parametrize("method", ["split4", "lawson2"])
def test_split_one_step_gate_full_256(method):
    """The full 256^3 Dirichlet cubic-quintic grid (the oracle takes a few s)."""
    _split_gate(ci.C2, method)


@pytest.mark.parametrize("method,lib", [("strang_3t", "strang"), ("split4_3t", "split4")])
def test_split_three_term_gates(method, lib):
    _split_gate(ci.scaled(ci.C1, (40, 36, 44)), method, three_term=True, lib=lib)
    _split_gate(ci.scaled(ci.C1, (40, 36, 44)), method, master=True, three_term=True, lib=lib)


@pytest.mark.parametrize("shape,master", [((96, 80, 40), False), ((130, 70, 9), True),
                                          ((256, 256), False), ((77,), False)])
def test_paired_lawson2_equals_two_actions_bitwise(shape, master, monkeypatch):
    torch = require_gpu()
    p = ci.scaled(ci.C1, shape) if len(shape) == 3 else (
        ci.scaled(ci.C0, shape) if len(shape) == 2 else CASES_1D)
    u0 = ci.initial_state(p)
    out = {}
    for paired in ("0", "1"):
        monkeypatch.setenv("CGL_LAWSON_PAIRED", paired)
        plan = _plan(p, "split", master=master)
        u = plan.to_device(u0)
        assert plan.run("lawson2", u, 3, 3) == 0
        plan.step("lawson2", u, 1)
        torch.cuda.synchronize()
        out[paired] = plan.to_host(u)
        plan.destroy()
    assert np.array_equal(out["0"], out["1"])


@pytest.mark.parametrize("method", ["split4", "lawson2"])
def test_graph_replay_equals_eager_bitwise(method):
    torch = require_gpu()
    for prec in ("fp64", "split"):
        plan = _plan(CASES_3D, prec)
        u0 = ci.initial_state(CASES_3D)
        a = plan.to_device(u0)
        b = plan.to_device(u0)
        plan.step(method, a, 7)
        assert plan.run(method, b, 7, 3) == 0
        torch.cuda.synchronize()
        assert torch.equal(a, b), (method, prec)
        plan.destroy()


def _batched(problems, precision):
    from paper_2403_02816_amd import cgl
    bp = cgl.BatchedPlan([p.n for p in problems], [p.coeffs for p in problems], problems[0].tau,
                         precision=precision)
    bp.set_fd_operators_batched(problems)
    return bp


@pytest.mark.parametrize("method", ["split4", "lawson2"])
def test_batched_split_gate_and_fp64_trajectory(method):
    torch = require_gpu()
    probs = ci.batched_sweep(count=24, seed=12)
    bp = _batched(probs, "split")
    u0 = [_c64(ci.initial_state(p)) for p in probs]
    u = bp.to_device_batched(u0)
    bp.step(method, u, 1)
    torch.cuda.synchronize()
    assert bp.status() == 0
    outs = bp.to_host_batched(u)
    worst = (0.0, 0.0)
    for j, p in enumerate(probs):
        E = [bp.get_instance_operator(j, mu, 0) for mu in range(2)]
        H = [bp.get_instance_operator(j, mu, 1) for mu in range(2)]
        l2, linf = errors(outs[j], _oracle(p, u0[j], method, 1, E, H))
        worst = (max(worst[0], l2), max(worst[1], linf))
        assert l2 < 1e-6 and linf < 1e-6, (j, p.n, l2, linf)
    log(f"batched split {method}: worst one-step rel-L2 {worst[0]:.2e}, rel-Linf {worst[1]:.2e}")
    bp.destroy()
    probs = ci.batched_sweep(count=5, seed=13, sizes=(64, 96))
    bp = _batched(probs, "fp64")
    u0 = [ci.initial_state(p) for p in probs]
    u = bp.to_device_batched(u0)
    assert bp.run(method, u, 8, 4) == 0
    torch.cuda.synchronize()
    outs = bp.to_host_batched(u)
    for j, p in enumerate(probs):
        E = [bp.get_instance_operator(j, mu, 0) for mu in range(2)]
        H = [bp.get_instance_operator(j, mu, 1) for mu in range(2)]
        assert_close(outs[j], _oracle(p, u0[j], method, 8, E, H), 1e-12,
                     f"batched fp64 {method} instance {j}")
    bp.destroy()


@pytest.mark.parametrize("method", ["strang", "split4", "lawson4", "lawson2"])
def test_fp64_table1_shape_fourth_order_dirichlet(method):
    """256^2, (0,100)^2, homogeneous Dirichlet, 4th-order FD (Section 4.1.1)."""
    _fp64_traj(ci.T1, method, 12)


@pytest.mark.parametrize("method", ["strang", "split4", "lawson4"])
def test_fp64_table3_shape_fourth_order_dirichlet_neumann(method):
    """128^3, (0,100)^3, Dirichlet at x_mu = 0 and Neumann at x_mu = 100 in
    every direction, 4th-order FD on the semi-internal grid (Section 4.2)."""
    _fp64_traj(ci.T3, method, 3)


def _paper_column(table, method):
    """{steps: error} and {steps: order} of a column the paper prints."""
    import os
    errs, orders = {}, {}
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_table_orders.txt")
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            t, m, m0, e0, m1, e1, order = line.split()
            if t == table and m == method:
                errs[int(m0)] = float(e0)
                errs[int(m1)] = float(e1)
                orders[int(m1)] = float(order)
    return errs, orders


def test_split4_errors_and_orders_on_the_table1_workload():
    """The Table 1 experiment (split4, FP64 form, 256^2 Dirichlet 4th-order FD,
    T = 6, m = 100 ... 300 steps) on a seeded random datum of the paper's
    distribution (normal / 5000), errors in the relative max-norm against
    split4 with 1200 steps (the paper does not say how its reference was
    made).  The paper's printed errors (5.9e-10 ... 2.4e-11) and orders
    (2.2 ... 3.9, pre-asymptotic) are for its own random datum; ours must
    fall within a factor 2 and 0.6 of them (the oracle gives 6.5e-10 ...
    3.2e-11, orders 2.19, 2.68, 3.08, 3.66)."""
    torch = require_gpu()
    p = ci.T1
    T = 6.0
    u0 = ci.initial_state(p)

    def run(m):
        q = ci.Problem(p.name, p.n, p.bc, p.a, p.b, p.coeffs, T / m, m, "split4", p.seed,
                       bc_hi=p.bc_hi, order=p.order, init=p.init)
        plan = _plan(q, "fp64")
        u = plan.to_device(u0)
        assert plan.run("split4", u, m, m) == 0
        torch.cuda.synchronize()
        out = plan.to_host(u)
        plan.destroy()
        return out

    ref = run(1200)
    ms = (100, 150, 200, 250, 300)
    errs = [metrics.rel_linf(run(m), ref) for m in ms]
    orders = [metrics.observed_order(ms[i], errs[i], ms[i + 1], errs[i + 1]) for i in range(4)]
    log(f"split4 Table 1 workload: errors {['%.3e' % e for e in errs]}, orders "
        f"{['%.3f' % o for o in orders]}")
    perr, pord = _paper_column("table1", "split4")
    for i, m in enumerate(ms):
        assert 0.5 < errs[i] / perr[m] < 2.0, (m, errs[i], perr[m])
        if i:
            assert abs(orders[i - 1] - pord[m]) < 0.6, (m, orders[i - 1], pord[m])
