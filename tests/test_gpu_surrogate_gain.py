"""What the trained surrogate gains over the plain stepper.

The network is trained on the GPU from scratch (pairs from the batched
split-precision Lawson4 stepper: 512 trajectories of the sweep at 128^2,
100-step burn-in, 40 pairs of 50 steps each), then run gated on held-out
instances for 20 jumps of 50 steps, checked every 10th jump at rel-L2 1e-3.
Measured: single-jump error of the trained network, its speed against 50
plain steps, acceptance, wall time to T and the final state against the
plain run.  Asserted: training lowers the held-out jump error, every
rejected span is redone exactly by the plain stepper, the cost of gating is
bounded, and a jump is far cheaper than the steps it replaces.
"""
import time

import numpy as np
import pytest

import cgl_inputs as ci
from tests._util import log, require_gpu

pytestmark = pytest.mark.gpu

JUMPS, CHECK, TOL, EPOCHS = 20, 10, 1e-3, 10


def test_trained_surrogate_gain():
    torch = require_gpu()
    from paper_2403_02816_amd import cgl
    from paper_2403_02816_amd import surrogate as S
    M = ci.C4_JUMP
    data = S.generate_pairs(512, ci.C4_TRAIN_SEED)
    tr, va = S.split_trajectories(data.B)
    sur = cgl.Surrogate(128, 128, 64)
    sur.set_params(S.init_params(0))
    ids_va = data.pair_ids(va)[::4]
    e_init = S.validation_error(sur, data, ids_va)
    t0 = time.perf_counter()
    losses = S.train(sur, data, data.pair_ids(tr), EPOCHS, batch=64)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    e_trained = S.validation_error(sur, data, ids_va)
    log(f"data {data.seconds:.1f} s; training {EPOCHS} epochs {t_train:.1f} s; loss "
        f"{losses[0]:.2e} -> {losses[-1]:.2e}; held-out jump rel-L2 mean/max "
        f"{e_init[0]:.3g}/{e_init[1]:.3g} -> {e_trained[0]:.3g}/{e_trained[1]:.3g}")
    assert e_trained[0] < e_init[0]

    net = cgl.Surrogate(128, 128, 1)
    net.set_params(sur.get_params())
    sur.destroy()
    rows = []
    for p in ci.batched_sweep(4, ci.C4_EVAL_SEED, fixed_n=128):
        plan = cgl.Plan(p.n, p.coeffs, p.tau, precision="split")
        plan.set_fd_operators(p.a, p.b, p.bc, p.coeffs)
        cs = S.standardise(p.coeffs)
        u = plan.to_device(ci.initial_state(p))
        assert plan.run("lawson4", u, 100) == 0
        ua, ub, uj = u.clone(), u.clone(), u.clone()
        # untimed first runs on the same tensors: graphs captured, tiles tuned
        cgl.run_surrogate(plan, net, ua, cs, JUMPS, M, CHECK, TOL)
        plan.run("lawson4", ub, JUMPS * M)
        ua.copy_(u)
        ub.copy_(u)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, stats = cgl.run_surrogate(plan, net, ua, cs, JUMPS, M, CHECK, TOL)
        torch.cuda.synchronize()
        t_gated = time.perf_counter() - t
        assert st == 0
        t = time.perf_counter()
        assert plan.run("lawson4", ub, JUMPS * M) == 0
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t
        # the ungated network: jump cost and error of one jump from the same state
        cst = torch.from_numpy(cs.astype(np.float32)[None]).to("cuda")
        ref1 = u.clone()
        plan.run("lawson4", ref1, M)
        net.forward(1, uj, cst, uj)
        torch.cuda.synchronize()
        e_jump = (torch.linalg.vector_norm(uj - ref1) / torch.linalg.vector_norm(ref1)).item()
        t = time.perf_counter()
        for _ in range(JUMPS):
            net.forward(1, uj, cst, uj)
        torch.cuda.synchronize()
        t_jump = (time.perf_counter() - t) / JUMPS
        err = (torch.linalg.vector_norm(ua - ub) / torch.linalg.vector_norm(ub)).item()
        rows.append((p.name, stats, t_gated, t_plain, e_jump, t_jump, err))
        log(f"{p.name}: gated {1e3 * t_gated:.1f} ms vs plain {1e3 * t_plain:.1f} ms "
            f"(gain {t_plain / t_gated:.2f}x) {stats}; final rel-L2 vs plain {err:.2e}; "
            f"one jump {1e3 * t_jump:.3f} ms vs {M} steps {1e3 * t_plain / JUMPS:.2f} ms "
            f"({t_plain / JUMPS / t_jump:.0f}x) at jump rel-L2 {e_jump:.3g}")
        if stats["accepted"] == 0:
            assert torch.equal(ua, ub)  # every span redone by the plain stepper
        else:
            assert err < 10 * TOL * stats["checks"]
        # a check costs one span of plain steps per check_every jumps
        assert t_gated < 1.6 * t_plain
        assert t_jump < 0.1 * t_plain / JUMPS
        plan.destroy()
    acc = sum(r[1]["accepted"] for r in rows) / (JUMPS * len(rows))
    gain = sum(r[3] for r in rows) / sum(r[2] for r in rows)
    log(f"accepted fraction {acc:.2f}; wall-time gain to T at rel-L2 {TOL}: {gain:.2f}x")
    net.destroy()
