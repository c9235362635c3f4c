"""What the trained surrogate gains over the plain stepper, for each reading
of the network's output: a correction about the state itself ("input"),
about the exact linear flow e^{M tau K} u ("linear": the change of variables
behind the Lawson schemes, Section 2.2, one Tucker operator of a plan with
step M tau), or about one Strang step of size M tau ("strang").

Per reading the network starts as its base (zero output layer) with its
output scale set to the root mean square of the corrections it has to learn,
and is trained on the GPU from scratch (MSE; pairs from the batched
split-precision Lawson4 stepper: 512 trajectories of the sweep at 128^2,
100-step burn-in, 40 pairs of 50 steps each, the bases from the batched
coarse plan).  Both the base alone (the untrained network) and the trained
network are then run gated on held-out instances for 20 jumps of 50 steps,
checked every 10th jump at rel-L2 1e-3.  Reported: the held-out jump errors
before and after training, acceptance and wall time to T against the plain
run.  Asserted: training lowers its loss, every rejected span is redone
exactly by the plain stepper, accepted spans stay within the checked
tolerance, the cost of gating is bounded, and a jump is far cheaper than
the steps it replaces.
"""
import time

import numpy as np
import pytest

import cgl_inputs as ci
from tests._util import log, require_gpu

pytestmark = pytest.mark.gpu

JUMPS, CHECK, TOL, EPOCHS = 20, 10, 1e-3, 10
READINGS = ("input", "linear", "strang")


def _median_jump_error(sur, data, ids, torch):
    """Median relative L2 error of single held-out jumps (the median: some
    instances decay towards zero and their relative errors mean little)."""
    P = data.n * data.n
    errs = []
    out = torch.empty((64 * P,), dtype=torch.complex64, device="cuda")
    for b0 in range(0, len(ids), 64):
        sel = ids[b0:b0 + 64]
        n = len(sel)
        src = torch.cat([data.snaps[int(i) * P:(int(i) + 1) * P] for i in sel])
        tgt = torch.cat([data.snaps[(int(i) + data.B) * P:(int(i) + data.B + 1) * P] for i in sel])
        bs = None
        if data.bases is not None:
            bs = torch.cat([data.bases[int(i) * P:(int(i) + 1) * P] for i in sel])
        cs = data.cstd[torch.from_numpy(sel.astype(np.int64)).to("cuda")]
        sur.forward(n, src, cs, out, base=bs)
        d = (out[:n * P] - tgt).view(n, P)
        errs.append((torch.linalg.vector_norm(d, dim=1) /
                     torch.linalg.vector_norm(tgt.view(n, P), dim=1)).cpu().numpy())
    return float(np.median(np.concatenate(errs)))


def _gated(cgl, S, net, base, M, torch):
    """Gated runs on four held-out instances; rows of (name, stats, t_gated,
    t_plain, final error, jump error, base error, jump time)."""
    rows = []
    for p in ci.batched_sweep(4, ci.C4_EVAL_SEED, fixed_n=128):
        plan = cgl.Plan(p.n, p.coeffs, p.tau, precision="split")
        plan.set_fd_operators(p.a, p.b, p.bc, p.coeffs)
        coarse = None if base == "input" else S.coarse_plan([p], p.tau, M, batched=False)
        cs = S.standardise(p.coeffs)
        u = plan.to_device(ci.initial_state(p))
        assert plan.run("lawson4", u, 100) == 0
        ua, ub, uj = u.clone(), u.clone(), u.clone()
        # untimed first runs on the same tensors: graphs captured, tiles tuned
        cgl.run_surrogate(plan, net, ua, cs, JUMPS, M, CHECK, TOL, coarse=coarse, base=base)
        plan.run("lawson4", ub, JUMPS * M)
        ua.copy_(u)
        ub.copy_(u)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, stats = cgl.run_surrogate(plan, net, ua, cs, JUMPS, M, CHECK, TOL, coarse=coarse,
                                      base=base)
        torch.cuda.synchronize()
        t_gated = time.perf_counter() - t
        assert st == 0
        t = time.perf_counter()
        assert plan.run("lawson4", ub, JUMPS * M) == 0
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t
        # one jump from the same state: the base alone and the network about it
        cst = torch.from_numpy(cs.astype(np.float32)[None]).to("cuda")
        ref1 = u.clone()
        plan.run("lawson4", ref1, M)
        bj = None
        e_base = float("nan")
        if coarse is not None:
            bj = torch.empty_like(u)
            S.apply_base(coarse, base, uj, bj)
            e_base = (torch.linalg.vector_norm(bj - ref1) / torch.linalg.vector_norm(ref1)).item()
        net.forward(1, uj, cst, uj, base=bj)
        torch.cuda.synchronize()
        e_jump = (torch.linalg.vector_norm(uj - ref1) / torch.linalg.vector_norm(ref1)).item()
        # the cost of a jump: the base and the network
        t = time.perf_counter()
        for _ in range(JUMPS):
            if coarse is not None:
                S.apply_base(coarse, base, uj, bj)
            net.forward(1, uj, cst, uj, base=bj)
        torch.cuda.synchronize()
        t_jump = (time.perf_counter() - t) / JUMPS
        err = (torch.linalg.vector_norm(ua - ub) / torch.linalg.vector_norm(ub)).item()
        rows.append((p.name, stats, t_gated, t_plain, err, e_jump, e_base, t_jump))
        if stats["accepted"] == 0:
            assert torch.equal(ua, ub)  # every span redone by the plain stepper
        else:
            assert err < 10 * TOL * stats["checks"]
        # a check costs one span of plain steps per check_every jumps
        assert t_gated < 1.6 * t_plain
        assert t_jump < 0.1 * t_plain / JUMPS
        plan.destroy()
        if coarse is not None:
            coarse.destroy()
    return rows


def _report(tag, rows, M):
    for name, stats, tg, tp, err, ej, eb, tj in rows:
        log(f"[{tag}] {name}: gated {1e3 * tg:.1f} ms vs plain {1e3 * tp:.1f} ms (gain "
            f"{tp / tg:.2f}x) {stats}; final rel-L2 vs plain {err:.2e}; one jump {1e3 * tj:.3f} ms "
            f"vs {M} steps {1e3 * tp / JUMPS:.2f} ms ({tp / JUMPS / tj:.0f}x) at jump rel-L2 "
            f"{ej:.3g} (base alone {eb:.3g})")
    acc = sum(r[1]["accepted"] for r in rows) / (JUMPS * len(rows))
    gain = sum(r[3] for r in rows) / sum(r[2] for r in rows)
    log(f"[{tag}] accepted fraction {acc:.2f}; wall-time gain to T at rel-L2 {TOL}: {gain:.2f}x")


@pytest.mark.parametrize("base", READINGS)
def test_trained_surrogate_gain(base):
    torch = require_gpu()
    from paper_2403_02816_amd import cgl
    from paper_2403_02816_amd import surrogate as S
    M = ci.C4_JUMP
    data = S.generate_pairs(512, ci.C4_TRAIN_SEED, base=base)
    tr, va = S.split_trajectories(data.B)
    ids_va = data.pair_ids(va)[::4]
    sur = cgl.Surrogate(128, 128, 64)
    sur.set_params(S.init_params(0, zero_output=True))
    scale = S.correction_rms(data, data.pair_ids(tr))
    sur.set_output_scale(scale)
    e_init = _median_jump_error(sur, data, ids_va, torch)
    t0 = time.perf_counter()
    losses = S.train(sur, data, data.pair_ids(tr), EPOCHS, batch=64)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    e_trained = _median_jump_error(sur, data, ids_va, torch)
    log(f"[{base}] data {data.seconds:.1f} s; output scale {scale:.3e}; training {EPOCHS} epochs "
        f"{t_train:.1f} s; loss {losses[0]:.2e} -> {losses[-1]:.2e}; held-out jump rel-L2 "
        f"(median) {e_init:.3g} (base alone) -> {e_trained:.3g} (trained)")
    assert losses[-1] < losses[0]

    net = cgl.Surrogate(128, 128, 1)
    net.set_output_scale(scale)
    net.set_params(S.init_params(0, zero_output=True))
    _report(f"{base} alone", _gated(cgl, S, net, base, M, torch), M)
    net.set_params(sur.get_params())
    sur.destroy()
    _report(f"{base} + trained network", _gated(cgl, S, net, base, M, torch), M)
    net.destroy()
