"""Shared helpers of the GPU tests: run the oracle and the library on the same
seeded inputs and compare."""
from __future__ import annotations

import numpy as np

import cgl_inputs as ci
from oracle import metrics, steppers, tensor


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def make_plan(p: ci.Problem, precision="fp64", master=False, rk4_flow=False, tau=None):
    from paper_2403_02816_amd import cgl
    plan = cgl.Plan(p.n, p.coeffs, p.tau if tau is None else tau, precision=precision,
                    master=master, rk4_flow=rk4_flow)
    plan.set_fd_operators(p.a, p.b, p.bc, p.coeffs)
    return plan


def plan_ops(plan):
    """FP64 exponentials the plan holds (data, shared with the oracle)."""
    E = [plan.get_operator(mu, 0) for mu in range(plan.d)]
    H = [plan.get_operator(mu, 1) for mu in range(plan.d)]
    return E, H


def oracle_run(p: ci.Problem, u0: np.ndarray, method: str, m: int, E, H, rk4_flow=False):
    """The oracle stepping with the given exponentials.  For Lawson4 the
    library applies e^{tau K} as e^{tau K/2} e^{tau K/2}; the oracle is given
    E = H H so both use the same data."""
    nl = steppers.CGLNonlinearity(p.coeffs.as_tuple(), force_rk4=rk4_flow)
    if method == "lawson4" or E is None:
        E = [h @ h for h in H]
    u, bad = steppers.run(u0, steppers.make_step(method, E, H, p.tau, nl), m)
    return u


def rel_l2(a, b) -> float:
    return metrics.rel_l2(a, b)


def log(msg: str):
    print(msg, flush=True)
