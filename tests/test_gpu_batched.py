"""GPU tests of batched plans (many independent 2-D instances with their own
grids and coefficients, stepped together by persistent launches).

* one-step gate of the split form for every instance vs the FP64 oracle
  stepping on that instance's exponentials (relative 2-norm <= 1e-6);
* the batched split plan equals one plain plan per instance bitwise (same
  kernels and tile shape on the same data);
* the FP64 batched form matches the oracle over 10 Lawson4 steps (<= 1e-12);
* graph replay equals eager steps bitwise.
"""
import numpy as np
import pytest

import cgl_inputs as ci
from tests._util import log, oracle_run, rel_l2, require_gpu

pytestmark = pytest.mark.gpu


def _sweep(count, seed, sizes=ci.C3_SIZES):
    return ci.batched_sweep(count=count, seed=seed, sizes=sizes)


def _batched(problems, precision):
    from paper_2403_02816_amd import cgl
    bp = cgl.BatchedPlan([p.n for p in problems], [p.coeffs for p in problems], problems[0].tau,
                         precision=precision)
    bp.set_fd_operators_batched(problems)
    return bp


def _c64(u):
    return u.astype(np.complex64).astype(np.complex128)


def test_batched_split_one_step_gate_every_instance():
    torch = require_gpu()
    probs = _sweep(12, 7)
    bp = _batched(probs, "split")
    u0 = [_c64(ci.initial_state(p)) for p in probs]
    u = bp.to_device_batched(u0)
    bp.step_lawson4(u, 1)
    torch.cuda.synchronize()
    assert bp.status() == 0
    outs = bp.to_host_batched(u)
    worst = 0.0
    for j, p in enumerate(probs):
        H = [bp.get_instance_operator(j, mu, 1) for mu in range(2)]
        ref = oracle_run(p, u0[j], "lawson4", 1, None, H)
        err = rel_l2(outs[j], ref)
        worst = max(worst, err)
        assert err < 1e-6, (j, p.n, err)
    log(f"batched split 12 instances: worst one-step rel-L2 {worst:.2e}")
    bp.destroy()


@pytest.mark.parametrize("tile", ["0", "1", "2", "3"])
def test_batched_equals_plain_plans_bitwise(tile, monkeypatch):
    monkeypatch.setenv("CGL_SPLIT_TILE", tile)
    torch = require_gpu()
    from paper_2403_02816_amd import cgl
    probs = _sweep(6, 8)
    bp = _batched(probs, "split")
    u0 = [ci.initial_state(p) for p in probs]
    u = bp.to_device_batched(u0)
    assert bp.run("lawson4", u, 3, 3) == 0
    torch.cuda.synchronize()
    outs = bp.to_host_batched(u)
    for j, p in enumerate(probs):
        sp = cgl.Plan(p.n, p.coeffs, p.tau, precision="split")
        for mu in range(2):
            sp.set_exponentials(mu, bp.get_instance_operator(j, mu, 0), bp.get_instance_operator(j, mu, 1))
        v = sp.to_device(u0[j])
        assert sp.run("lawson4", v, 3, 3) == 0
        torch.cuda.synchronize()
        assert np.array_equal(sp.to_host(v), outs[j]), (j, p.n)
        sp.destroy()
    bp.destroy()


def test_batched_fp64_trajectory_matches_oracle():
    torch = require_gpu()
    probs = _sweep(5, 9, sizes=(64, 96))
    bp = _batched(probs, "fp64")
    u0 = [ci.initial_state(p) for p in probs]
    u = bp.to_device_batched(u0)
    bp.step_lawson4(u, 10)
    torch.cuda.synchronize()
    outs = bp.to_host_batched(u)
    for j, p in enumerate(probs):
        H = [bp.get_instance_operator(j, mu, 1) for mu in range(2)]
        ref = oracle_run(p, u0[j], "lawson4", 10, None, H)
        assert rel_l2(outs[j], ref) < 1e-12, j
    bp.destroy()


def test_batched_graph_equals_eager():
    torch = require_gpu()
    probs = _sweep(9, 10)
    bp = _batched(probs, "split")
    u0 = [ci.initial_state(p) for p in probs]
    a = bp.to_device_batched(u0)
    b = bp.to_device_batched(u0)
    bp.step_lawson4(a, 4)
    assert bp.run("lawson4", b, 4, 2) == 0
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    bp.destroy()
