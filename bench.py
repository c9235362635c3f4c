#!/usr/bin/env python3
"""Throughput benchmark of the CGL exponential stepper on one MI355X.

Workload (default): 3-D cubic-quintic CGL on a 256^3 interior grid on
(-15,15)^3 with homogeneous Dirichlet boundaries, 2nd-order FD, Lawson4 with
tau = 2e-3, seeded Gaussian vortex ring u0 (16.8M grid points).  One step =
one Lawson4 step of the whole grid: four actions of e^{tau K/2} (three
mu-mode passes each), run as two rounds of three paired passes, with g and
the Lawson4 stage combinations fused into the first-pass prologue and the
last-pass epilogues.

The timed form is the split-precision form (complex64 stage tensors,
bf16x3 operands, FP32 accumulation); the FP64 form and the split Strang
step of the same grid are timed beside it.  Inputs are resident in HBM
before the timed region; the K steps are replayed from a captured HIP graph
(cgl_run), the state reset to u0 before each replay, and the median of the
replays is reported.  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_PEAK_BF16_TFLOPS = 2500.0  # dense MFMA
MI355X_PEAK_FP64_TFLOPS = 78.6
MI355X_PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the dominant kernel of a workload, from two
# rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled
# by the factor the same counter reads for a 256 MiB device copy in the same
# run), valid only for the kernel sources whose digest is recorded with them
# (profiles/split_pass_c1_128_lawson4.md, profiles/split_pass_c2_256_lawson4.md).
SPLIT_TRAFFIC = {
    # mean over the six paired launches of a step (128-row tiles, the shape the
    # autotuner picks): (FETCH_SIZE x 2 + WRITE_SIZE) KiB = (15888 x 2 + 30037) KiB
    "c1": {"bytes_per_launch": 63296683.0, "sources_sha256_16": "c15fdcc26ffd29a0"},
    # (144818 x 2 + 240299) KiB = 1.011 x the algorithmic 536870912 bytes
    "c2_lawson4": {"bytes_per_launch": 542652224.0, "sources_sha256_16": "c15fdcc26ffd29a0"},
}
SPLIT_SOURCES = ("kernels_split.hip", "kernels.hpp", "pointwise.hpp", "split_layout.cpp",
                 "split_layout.hpp")

# The paper's own throughput on the nearest workload (context, not the target:
# another machine, another precision, 4th-order FD, 128^3 rather than 256^3).
PAPER_TABLE3 = {
    "source": "Table 3: 3-D cubic CGL, 128^3, Dirichlet on x1x2x3 = 0 faces and Neumann "
              "elsewhere, if4 (Lawson4), T = 10",
    "hardware": "Intel Core i7-10750H (6 cores), MATLAB R2022a, FP64, level-3 BLAS",
    "if4_steps": 250, "if4_time_s": 120.6, "grid_points": 128 ** 3,
    "gp_steps_per_s": 128 ** 3 * 250 / 120.6,
}


def split_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for name in SPLIT_SOURCES:
        with open(os.path.join(ROOT, "paper_2403_02816_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--replays", type=int, default=5,
                    help="graph replays of the K timed steps (median reported)")
    ap.add_argument("--workload", default="c2_lawson4",
                    choices=["c2_lawson4", "c2_strang", "c1", "c3", "c4", "t4", "t5"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the second method timed beside the workload")
    ap.add_argument("--cpu-budget-s", type=float, default=15.0,
                    help="host time spent on the oracle baseline (whole steps, at least one)")
    ap.add_argument("--cpu-max-steps", type=int, default=200)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 256 MiB device-to-device copy (a kernel of known "
                         "traffic for scaling HBM counters)")
    return ap.parse_args()


def workload(name):
    import cgl_inputs as ci
    if name == "c1":
        return ci.C1, "lawson4"
    if name == "c2_strang":
        return ci.C2, "strang"
    return ci.C2, "lawson4"


def paired_lawson4(method, precision="split"):
    """Split-form Lawson4 runs both actions of a round in one paired pass per
    direction unless CGL_LAWSON_PAIRED=0."""
    return method == "lawson4" and precision == "split" and os.environ.get("CGL_LAWSON_PAIRED", "1") != "0"


def launches_per_step(method, d, paired=False):
    """mu-mode pass launches per step: one exponential action (d passes) for
    Strang, four actions of e^{tau K/2} for Lawson4 (two rounds of d paired
    passes when paired)."""
    if method == "strang":
        return d
    return 2 * d if paired else 4 * d


def time_form(p, method, precision, steps, warmup, u0, replays):
    """Plan, warm up, capture the graph of `steps` steps, then replay it
    `replays` times from u0 (reset outside the timed region), each replay
    bracketed by HIP events on the stream the plan joins (torch's current
    stream).  Returns (plan, final state after the last replay = `steps`
    steps from u0, list of replay times in ms)."""
    import torch
    from paper_2403_02816_amd import cgl
    plan = cgl.Plan(p.n, p.coeffs, p.tau, precision=precision)
    plan.set_fd_operators(p.a, p.b, p.bc, p.coeffs)
    u = plan.to_device(u0)
    u_init = u.clone()
    if warmup > 0:
        st = plan.run(method, u, warmup, warmup)
        assert st == 0, st
    st = plan.run(method, u, steps, steps)  # graph capture of the timed chunk size
    assert st == 0, st
    times = []
    stream = torch.cuda.current_stream()
    for _ in range(max(1, replays)):
        u.copy_(u_init)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        st = plan.run(method, u, steps, steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        assert st == 0, st
        times.append(ev0.elapsed_time(ev1))
    return plan, u, times


def one_step_gate(p, method, plan):
    """One split step vs the FP64 oracle step from the same (complex64) input:
    (relative 2-norm, relative max-norm = the paper's measure)."""
    import torch
    import cgl_inputs as ci
    from oracle import metrics, steppers
    u0 = ci.initial_state(p).astype(np.complex64).astype(np.complex128)
    u = plan.to_device(u0)
    (plan.step_strang if method == "strang" else plan.step_lawson4)(u, 1)
    torch.cuda.synchronize()
    E = [plan.get_operator(mu, 0) for mu in range(p.d)]
    H = [plan.get_operator(mu, 1) for mu in range(p.d)]
    if method == "lawson4":
        E = [h @ h for h in H]
    nl = steppers.CGLNonlinearity(p.coeffs.as_tuple())
    ref = steppers.make_step(method, E, H, p.tau, nl)(u0)
    got = plan.to_host(u)
    return metrics.rel_l2(got, ref), metrics.rel_linf(got, ref)


def _blas_threads():
    """Threads the host BLAS uses."""
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()]))
    except Exception:
        return int(os.cpu_count())


def _host_cpu_info():
    """Physical cores of the host (lscpu: distinct (core, socket) pairs) and
    the CPUs this process may run on."""
    import subprocess
    phys = None
    try:
        out = subprocess.run(["lscpu", "-p=CORE,SOCKET"], capture_output=True, text=True,
                             timeout=10).stdout
        phys = len({ln for ln in out.splitlines() if ln and not ln.startswith("#")})
    except Exception:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except Exception:
        aff = os.cpu_count()
    return phys, aff


def cpu_baseline(p, method, budget_s, max_steps):
    """The FP64 oracle as written (six exponential actions per Lawson4 step,
    numpy tensordot on the host BLAS) timed on the host cores on a bounded
    sample: whole full-grid steps until the time budget is spent (at least
    one, at most max_steps), with all BLAS threads; then one more step with
    one BLAS thread."""
    import cgl_inputs as ci
    from oracle import steppers
    E = steppers.operators_for(p, p.tau)
    H = steppers.operators_for(p, 0.5 * p.tau)
    nl = steppers.CGLNonlinearity(p.coeffs.as_tuple())
    step = steppers.make_step(method, E, H, p.tau, nl)
    u = ci.initial_state(p)
    nsteps = 0
    t0 = time.perf_counter()
    while nsteps < max_steps and (nsteps == 0 or time.perf_counter() - t0 < budget_s):
        u = step(u)
        nsteps += 1
    dt = time.perf_counter() - t0
    threads = _blas_threads()
    phys, aff = _host_cpu_info()
    one = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            u = step(u)
            s1 = time.perf_counter() - t1
        one = {"threads": 1, "value": p.N / s1, "step_s": s1,
               "sample": f"one {method} step of the full grid with one BLAS thread"}
    except Exception as e:  # threadpoolctl missing: report without the 1-thread figure
        one = {"error": repr(e)}
    return {"value": p.N * nsteps / dt, "unit": "grid-point-steps/s", "cores": threads,
            "kind": "oracle", "physical_cores_lscpu": phys, "affinity_cpus": aff,
            "sample": f"{nsteps} {method} step(s) of the full {'x'.join(map(str, p.n))} grid "
                      f"(numpy FP64, literal scheme, {threads} BLAS threads); {dt:.2f} s",
            "one_thread": one}


def bench_batched(args):
    """512 independent 2-D cubic instances (n1, n2 in {64,...,192}), Lawson4,
    tau = 1e-2, split form, one persistent launch per mu-mode pass."""
    import torch
    import cgl_inputs as ci
    from oracle import metrics
    from paper_2403_02816_amd import cgl
    probs = ci.batched_sweep()
    K, W = args.steps, args.warmup
    t_setup = time.perf_counter()
    bp = cgl.BatchedPlan([p.n for p in probs], [p.coeffs for p in probs], ci.C3_TAU,
                         precision="split")
    bp.set_fd_operators_batched(probs)
    t_setup = time.perf_counter() - t_setup
    u0 = [ci.initial_state(p) for p in probs]
    u = bp.to_device_batched(u0)
    u_init = u.clone()
    if W > 0:
        assert bp.run("lawson4", u, W, W) == 0
    assert bp.run("lawson4", u, K, K) == 0  # captures the timed chunk's graph
    times = []
    for _ in range(max(1, args.replays)):
        u.copy_(u_init)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        assert bp.run("lawson4", u, K, K) == 0
        ev1.record()
        torch.cuda.synchronize()
        times.append(ev0.elapsed_time(ev1))
    ms = float(np.median(times))
    Ntot = sum(p.N for p in probs)
    launches = launches_per_step("lawson4", 2, paired_lawson4("lawson4"))  # persistent launches
    launch_ms = ms / (K * launches)
    mfma = sum(6.0 * 8.0 * p.N * (p.n[0] + p.n[1]) for p in probs) * 4 / launches
    achieved = mfma / (launch_ms * 1e-3) / 1e12
    # one-step gate of every instance, oracle on each instance's exponentials
    from oracle import steppers
    ug = bp.to_device_batched([ci.initial_state(p).astype(np.complex64) for p in probs])
    bp.step_lawson4(ug, 1)
    torch.cuda.synchronize()
    outs = bp.to_host_batched(ug)
    gate = 0.0
    gate_inf = 0.0
    for j, p in enumerate(probs):
        H = [bp.get_instance_operator(j, mu, 1) for mu in range(2)]
        E = [h @ h for h in H]
        nl = steppers.CGLNonlinearity(p.coeffs.as_tuple())
        ref = steppers.lawson4_step(ci.initial_state(p).astype(np.complex64).astype(np.complex128),
                                    E, H, p.tau, nl)
        gate = max(gate, metrics.rel_l2(outs[j], ref))
        gate_inf = max(gate_inf, metrics.rel_linf(outs[j], ref))
    sample = probs
    split_state = u.clone()
    bp.destroy()
    fp64 = None
    traj = None
    if not args.no_fp64:
        b64 = cgl.BatchedPlan([p.n for p in probs], [p.coeffs for p in probs], ci.C3_TAU,
                              precision="fp64")
        b64.set_fd_operators_batched(probs)
        v = b64.to_device_batched(u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b64.step_lawson4(v, K)
        torch.cuda.synchronize()
        s64 = time.perf_counter() - t0
        fp64 = {"value": Ntot * K / s64, "ms_per_step": 1e3 * s64 / K,
                "note": "FP64 form, one launch per instance and pass (eager)"}
        a = split_state.to(torch.complex128)
        traj = max(float(torch.linalg.vector_norm(a[o:o + p.N] - v[o:o + p.N]).item()
                         / torch.linalg.vector_norm(v[o:o + p.N]).item())
                   for p, o in zip(probs, b64.offsets))
        b64.destroy()
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_batched(probs[::8], 150, budget_s=12.0)
    rec = {
        "metric": "grid-point-steps/s at rel-L2 <=1e-6 vs FP64 oracle; MFMA util % of peak",
        "value": Ntot * K / (ms * 1e-3), "unit": "grid-point-steps/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": ms / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3->f32 (split), state c64",
        "data": "synthetic",
        "config": {"workload": f"batched sweep: {len(probs)} 2-D cubic CGL instances, n1,n2 in "
                               f"{list(ci.C3_SIZES)}, Lawson4, tau={ci.C3_TAU}, split form, "
                               f"{Ntot} grid points", "instances": len(probs),
                   "grid_points": Ntot, "method": "lawson4", "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": MI355X_PEAK_BF16_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / MI355X_PEAK_BF16_TFLOPS,
                     "traffic": None, "kernel": ("k_pass_split_batched_pair (persistent, both actions of a Lawson4 round)" if paired_lawson4("lawson4") else "k_pass_split_batched (persistent)"),
                     "launch_ms": launch_ms},
        "replays_ms": times,
        "accuracy": {"one_step_rel_l2_vs_fp64_oracle_max": gate,
                     "one_step_rel_linf_vs_fp64_oracle_max": gate_inf, "gate": 1e-6,
                     "gated_instances": len(sample),
                     "trajectory_rel_l2_vs_fp64_form_max": traj, "trajectory_steps": K},
        "fp64_form": fp64, "cpu_baseline": cpu, "setup_s": t_setup,
    }
    print(json.dumps(rec))


def cpu_baseline_batched(problems, nsteps, budget_s):
    """The oracle on a sample of the sweep: nsteps Lawson4 steps of each
    instance in turn until the time budget is spent (whole instances only)."""
    import cgl_inputs as ci
    from oracle import steppers
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    pts = 0
    done = 0
    dt = 0.0
    for p in problems:
        E = steppers.operators_for(p, p.tau)
        H = steppers.operators_for(p, 0.5 * p.tau)
        nl = steppers.CGLNonlinearity(p.coeffs.as_tuple())
        step = steppers.make_step("lawson4", E, H, p.tau, nl)
        u = ci.initial_state(p)
        t0 = time.perf_counter()
        for _ in range(nsteps):
            u = step(u)
        dt += time.perf_counter() - t0
        pts += u.size * nsteps
        done += 1
        if dt > budget_s:
            break
    return {"value": pts / dt, "unit": "grid-point-steps/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{nsteps} Lawson4 steps of each of {done} instances (every 8th of the "
                      f"sweep, {pts // nsteps} grid points; numpy FP64, literal scheme); "
                      f"{dt:.2f} s"}


def bench_surrogate(args):
    """The learned surrogate on 128^2 2-D cubic instances: K timed training
    steps (batch 64, Adam), the batched forward pass, and gated runs of 20
    jumps of 50 Lawson4 steps (checked every 10th jump at rel-L2 1e-3) against
    the plain stepper to the same time on held-out instances."""
    import torch
    import cgl_inputs as ci
    from paper_2403_02816_amd import cgl
    from paper_2403_02816_amd import surrogate as S
    K, W = args.steps, args.warmup
    M, JUMPS, CHECK, TOL, B = ci.C4_JUMP, 20, 10, 1e-3, 64
    n = ci.C4_N
    P = n * n
    data = S.generate_pairs(512, ci.C4_TRAIN_SEED)
    tr, _ = S.split_trajectories(data.B)
    sur = cgl.Surrogate(n, n, B)
    sur.set_params(S.init_params(0))
    order = np.random.default_rng(0).permutation(
        np.resize(data.pair_ids(tr), (W + K) * B)).astype(np.int32)
    idx = torch.from_numpy(order).to("cuda")
    for b in range(W):
        sur.train_step(B, data.snaps, data.cstd, idx[b * B:(b + 1) * B], data.B, 1e-3)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for b in range(W, W + K):
        sur.train_step(B, data.snaps, data.cstd, idx[b * B:(b + 1) * B], data.B, 1e-3)
    ev1.record()
    torch.cuda.synchronize()
    train_ms = ev0.elapsed_time(ev1) / K
    loss = sur.take_loss()
    # batched forward pass (inference: 6 conv launches + packing)
    out = torch.empty((B * P,), dtype=torch.complex64, device="cuda")
    src = data.snaps[:B * P]
    cs = data.cstd[:B].contiguous()
    for _ in range(3):
        sur.forward(B, src, cs, out)
    reps = 20
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        sur.forward(B, src, cs, out)
    ev1.record()
    torch.cuda.synchronize()
    fwd_ms = ev0.elapsed_time(ev1) / reps
    layers = [(48, 7)] + [(48, 48)] * 4 + [(2, 48)]
    flops_px = sum(2.0 * 9 * co * cin for co, cin in layers)
    # per point and sample, each stage reads its input and writes its output
    # once in FP32 (pack 8 + 28, conv_in 28 + 192, residual convs 192 + 192,
    # conv_out 192 + 8 + 8, unpack 8 + 8)
    bytes_px = 36 + 220 + 4 * 384 + 208 + 16
    fwd_gbs = bytes_px * B * P / (fwd_ms * 1e-3) / 1e9
    fwd_tf = flops_px * B * P / (fwd_ms * 1e-3) / 1e12
    net = cgl.Surrogate(n, n, 1)
    net.set_params(sur.get_params())
    sur.destroy()
    rows = []
    for p in ci.batched_sweep(4, ci.C4_EVAL_SEED, fixed_n=n):
        plan = cgl.Plan(p.n, p.coeffs, p.tau, precision="split")
        plan.set_fd_operators(p.a, p.b, p.bc, p.coeffs)
        c5 = S.standardise(p.coeffs)
        u = plan.to_device(ci.initial_state(p))
        assert plan.run("lawson4", u, 100) == 0
        ua, ub = u.clone(), u.clone()
        cgl.run_surrogate(plan, net, ua, c5, JUMPS, M, CHECK, TOL)
        plan.run("lawson4", ub, JUMPS * M)
        ua.copy_(u)
        ub.copy_(u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, stats = cgl.run_surrogate(plan, net, ua, c5, JUMPS, M, CHECK, TOL)
        torch.cuda.synchronize()
        tg = time.perf_counter() - t0
        t0 = time.perf_counter()
        plan.run("lawson4", ub, JUMPS * M)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        err = float(torch.linalg.vector_norm(ua - ub).item() / torch.linalg.vector_norm(ub).item())
        # the plain FP64 form to the same time, from the same state
        p64 = cgl.Plan(p.n, p.coeffs, p.tau, precision="fp64")
        p64.set_fd_operators(p.a, p.b, p.bc, p.coeffs)
        uf = u.to(torch.complex128)
        p64.run("lawson4", uf.clone(), M)  # graph and launch setup
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        assert p64.run("lawson4", uf, JUMPS * M) == 0
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        e64 = float(torch.linalg.vector_norm(ua.to(torch.complex128) - uf).item()
                    / torch.linalg.vector_norm(uf).item())
        p64.destroy()
        rows.append((stats, tg, tp, err, tf, e64))
        plan.destroy()
    net.destroy()
    tg = sum(r[1] for r in rows)
    tp = sum(r[2] for r in rows)
    acc = sum(r[0]["accepted"] for r in rows) / (JUMPS * len(rows))
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_surrogate(data, S)
    rec = {
        "metric": "grid-point-steps/s to T, surrogate jumps gated at rel-L2 <=1e-3 vs plain "
                  "Lawson4 (fallback: the plain stepper)",
        "value": len(rows) * P * JUMPS * M / tg, "unit": "grid-point-steps/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": train_ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16->f32 (conv MFMA), state c64",
        "data": "synthetic",
        "config": {"workload": f"surrogate: 6-layer residual CNN (48 ch, 3x3), 128^2 2-D cubic "
                               f"CGL, jump = {M} Lawson4 steps; trained on 512 x 40 pairs of the "
                               f"sweep; {len(rows)} held-out instances x {JUMPS} jumps, check "
                               f"every {CHECK}th", "batch": B, "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": fwd_gbs, "peak": MI355X_PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": fwd_gbs / MI355X_PEAK_HBM_GBS, "traffic": None,
                     "kernel": "k_conv (forward pass of 64 samples: 6 conv launches + packing)",
                     "forward_ms": fwd_ms, "mfma_tflops": fwd_tf},
        "surrogate": {"train_ms_per_step": train_ms, "train_samples_per_s": B / (train_ms * 1e-3),
                      "train_loss_mean": loss, "forward_ms_batch64": fwd_ms,
                      "gated_ms": 1e3 * tg / len(rows), "plain_ms": 1e3 * tp / len(rows),
                      "gain_vs_plain": tp / tg, "accepted_fraction": acc,
                      "final_rel_l2_vs_plain_max": max(r[3] for r in rows),
                      "fp64_plain_ms": 1e3 * sum(r[4] for r in rows) / len(rows),
                      "final_rel_l2_vs_fp64_plain_max": max(r[5] for r in rows),
                      "stats": [r[0] for r in rows]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


def cpu_baseline_surrogate(data, S):
    """The oracle network forward pass (numpy FP64) on single 128^2 samples."""
    from oracle import surrogate as osur
    params = osur.init_params(0)
    P = data.n * data.n
    u = data.snaps[:P].cpu().numpy().astype(np.complex128).reshape(data.n, data.n, order="F")
    x = osur.make_input(u, data.cstd[0].cpu().numpy().astype(np.float64))[None]
    done, t0 = 0, time.perf_counter()
    while done < 1 or (time.perf_counter() - t0 < 10.0 and done < 8):
        osur.forward(params, x)
        done += 1
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "jumps/s (forward passes of one 128^2 sample)",
            "cores": _blas_threads(), "kind": "oracle",
            "sample": f"{done} forward passes of the FP64 numpy network; {dt:.2f} s"}


def split_roofline(p, method, times_ms, steps):
    """Roofline of the dominant kernel of a split-form step, from the median
    replay: every launch of the step is the same pass kernel (the paired pass
    for Lawson4, the autotuned single-action pass for Strang), so its average
    launch duration is the timed region divided by the launches."""
    ms = float(np.median(times_ms))
    paired = paired_lawson4(method)
    nl = launches_per_step(method, p.d, paired)
    launch_ms = ms / (steps * nl)
    # algorithmic work of one launch: every grid point gets one complex
    # mu-mode product of length n (8 n real flops) per product (two in a
    # paired pass); the split form issues 6 bf16 term products for each, so
    # its MFMA work is 6x that
    prod = 2 if paired else 1
    n_mu = p.n[0]
    alg_flops = 8.0 * p.N * n_mu * prod
    mfma_flops = 6.0 * alg_flops
    alg_bytes = p.N * (8 + 8) * prod
    achieved_tf = mfma_flops / (launch_ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": achieved_tf, "peak": MI355X_PEAK_BF16_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved_tf / MI355X_PEAK_BF16_TFLOPS,
            "kernel": ("k_pass_split_pair (both actions of a Lawson4 round per launch)" if paired
                       else "k_pass_split_dma / k_pass_split (the autotuned split pass)"),
            "launch_ms": launch_ms, "launches_per_step": nl,
            "mfma_flops_per_launch": mfma_flops, "alg_flops_per_launch": alg_flops,
            "alg_bytes_per_launch": alg_bytes,
            "hbm_gbs_algorithmic": alg_bytes / (launch_ms * 1e-3) / 1e9}


# The paper's Table 4 (3-D cubic-quintic CGL, periodic, 128^3 Fourier, if4,
# T = 5): context for the Fourier path, not the target (MATLAB + FFTW on a
# laptop, FP64).
PAPER_TABLE4 = {
    "source": "Table 4: 3-D cubic-quintic CGL, periodic, 128^3 Fourier pseudospectral, if4 "
              "(Lawson4), 300 steps, T = 5",
    "hardware": "Intel Core i7-10750H (6 cores), MATLAB R2022a with FFTW, FP64",
    "if4_steps": 300, "if4_time_s": 141.7, "grid_points": 128 ** 3,
    "gp_steps_per_s": 128 ** 3 * 300 / 141.7,
}


def bench_fourier(args):
    """The Table 4 workload on the Fourier path: every direction periodic, each
    pass a length-128 transform, the factors and the inverse transform in one
    read and one write of the tensor (HBM-bound).  Lawson4, tau = 5/300,
    complex64 state (FP32 transforms), the FP64 form beside it."""
    import torch
    import cgl_inputs as ci
    from oracle import fourier as fo, metrics, steppers
    p = ci.T4
    u0 = ci.initial_state(p)
    K, W, R = args.steps, args.warmup, args.replays

    def timed(precision):
        from paper_2403_02816_amd import cgl
        plan = cgl.Plan(p.n, p.coeffs, p.tau, precision=precision)
        plan.set_problem_operators(p)
        u = plan.to_device(u0)
        u_init = u.clone()
        if W > 0:
            assert plan.run("lawson4", u, W, W) == 0
        assert plan.run("lawson4", u, K, K) == 0
        times = []
        for _ in range(max(1, R)):
            u.copy_(u_init)
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record()
            assert plan.run("lawson4", u, K, K) == 0
            ev1.record()
            torch.cuda.synchronize()
            times.append(ev0.elapsed_time(ev1))
        return plan, u, times

    plan, u, times = timed("split")
    ms = float(np.median(times))
    # algorithmic HBM bytes per Lawson4 step (complex64, per point): round 1:
    # P = H u (3 passes x 16) + Q = H g(u) (2 x 16, last pass reads its input
    # and P, writes X and Y: 32); round 2: H X (48) + H Y (32 + 24) = 216
    alg_bytes = 216.0 * p.N
    achieved = alg_bytes / (ms / K * 1e-3) / 1e9
    # one-step gate against the oracle on the plan's exported factors
    ug = plan.to_device(u0.astype(np.complex64).astype(np.complex128))
    plan.step_lawson4(ug, 1)
    torch.cuda.synchronize()
    E = fo.FourierAction([plan.get_periodic_factor(mu, 0) for mu in range(3)])
    H = fo.FourierAction([plan.get_periodic_factor(mu, 1) for mu in range(3)])
    nl = steppers.CGLNonlinearity(p.coeffs.as_tuple())
    ref = steppers.lawson4_step(u0.astype(np.complex64).astype(np.complex128), E, H, p.tau, nl)
    got = plan.to_host(ug)
    gate = (metrics.rel_l2(got, ref), metrics.rel_linf(got, ref))
    split_state = u.clone()
    plan.destroy()
    fp64 = None
    traj = None
    if not args.no_fp64:
        plan64, u64, t64 = timed("fp64")
        ms64 = float(np.median(t64))
        d = split_state.to(torch.complex128) - u64
        traj = {"rel_l2": float(torch.linalg.vector_norm(d).item()
                                / torch.linalg.vector_norm(u64).item()),
                "rel_linf": float(d.abs().max().item() / u64.abs().max().item())}
        fp64 = {"value": p.N * K / (ms64 * 1e-3), "ms_per_step": ms64 / K, "replays_ms": t64,
                "hbm_gbs": 2.0 * alg_bytes / (ms64 / K * 1e-3) / 1e9,
                "frac": 2.0 * alg_bytes / (ms64 / K * 1e-3) / 1e9 / MI355X_PEAK_HBM_GBS}
        plan64.destroy()
    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        Eo, Ho = fo.actions_for(p, p.tau), fo.actions_for(p, 0.5 * p.tau)
        v = u0.copy()
        nsteps = 0
        while nsteps == 0 or (time.perf_counter() - t0 < args.cpu_budget_s and nsteps < 50):
            v = steppers.lawson4_step(v, Eo, Ho, p.tau, nl)
            nsteps += 1
        dt = time.perf_counter() - t0
        cpu = {"value": p.N * nsteps / dt, "unit": "grid-point-steps/s",
               "cores": _blas_threads(), "kind": "oracle",
               "sample": f"{nsteps} literal Lawson4 steps of the full 128^3 grid (numpy FFT, "
                         f"FP64); {dt:.2f} s"}
    rec = {
        "metric": "grid-point-steps/s at rel-L2 <=1e-6 vs FP64 oracle; HBM % of peak",
        "value": p.N * K / (ms * 1e-3), "unit": "grid-point-steps/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": ms / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 FFT (state c64)",
        "data": "synthetic (the paper's deterministic necklace-ring datum)",
        "config": {"workload": f"{p.name}: 3-D cubic-quintic CGL 128^3 periodic (Fourier), "
                               f"Lawson4, tau={p.tau:.6g}", "grid": list(p.n),
                   "method": "lawson4", "parallelism": "single-gpu"},
        "replays_ms": times,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": MI355X_PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / MI355X_PEAK_HBM_GBS, "traffic": None,
                     "kernel": "k_pass_fft<float, 128> (12 Fourier passes per step, two actions "
                               "per round as concurrent branches)",
                     "alg_bytes_per_step": alg_bytes},
        "accuracy": {"one_step_rel_l2_vs_fp64_oracle": gate[0],
                     "one_step_rel_linf_vs_fp64_oracle": gate[1], "gate": 1e-6,
                     "trajectory_vs_fp64_form": traj, "trajectory_steps": K},
        "fp64_form": fp64, "cpu_baseline": cpu, "paper_context": PAPER_TABLE4,
    }
    print(json.dumps(rec))


PAPER_TABLE5 = {
    "source": "Table 5: 2-D coupled cubic-quintic CGL, periodic, 700 x 350 Fourier modes, "
              "if4 (Lawson4), 2500 steps, T = 3",
    "hardware": "Intel Core i7-10750H (6 cores), MATLAB R2022a with FFTW, FP64",
    "if4_steps": 2500, "if4_time_s": 167.7, "grid_points": 2 * 700 * 350,
    "gp_steps_per_s": 2 * 700 * 350 * 2500 / 167.7,
}


def bench_coupled(args):
    """The Table 5 workload: the coupled two-field system (Section 4.4) on
    700 x 350 periodic modes (no Fourier pass at these lengths: each
    direction's exponential is a dense circulant on the mu-mode product
    kernels, the four independent field actions of a Lawson round run on
    four streams), the soliton datum, Lawson4 with the paper's 2500-step tau,
    both precisions.  A grid point is counted per field."""
    import torch
    import cgl_inputs as ci
    from oracle import coupled as co, fourier as fo, steppers
    from paper_2403_02816_amd import cgl
    n, lo, hi, T, m = (700, 350), (0.0, 0.0), (70.0, 35.0), 3.0, 2500
    tau = T / m
    # the datum as Section 4.4 builds it, by the library: the 1-D cubic-quintic
    # equation from the Gaussian 2.25 exp(-(x - 17.5)^2 / 12.5), if4 with
    # 10000 steps to T = 25, then u0(x1, x2) = w(x1), v0 = w(70 - x1)
    c = co.PAPER
    p1 = cgl.Plan((n[0],), ci.Coeffs(c.a1, c.b1, c.a2, c.a3, c.b3, c.a4, c.b4), 25.0 / 10000,
                  precision="fp64")
    p1.set_periodic(0, lo[0], hi[0])
    x = lo[0] + (hi[0] - lo[0]) * np.arange(n[0]) / n[0]
    w1 = p1.to_device(2.25 * np.exp(-(x - 17.5) ** 2 / (2 * 2.5 ** 2)) + 0j)
    assert p1.run("lawson4", w1, 10000, 2500) == 0
    u1 = np.repeat(p1.to_host(w1)[:, None], n[1], axis=1)
    p1.destroy()
    W0 = np.stack([u1, np.roll(u1[::-1], 1, axis=0)])
    K, W, R = args.steps, args.warmup, args.replays
    pts = 2 * n[0] * n[1]

    def timed(precision):
        p = cgl.CoupledPlan(n, co.PAPER, tau, precision=precision)
        for mu in range(2):
            p.set_periodic(mu, lo[mu], hi[mu])
        w = p.to_device(W0)
        w0 = w.clone()
        p.step("lawson4", w, max(W, 1))
        torch.cuda.synchronize()
        times = []
        for _ in range(max(1, R)):
            w.copy_(w0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p.step("lawson4", w, K)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        assert p.status() == 0
        return p, w, times

    p, w, times = timed("split")
    ms = float(np.median(times))
    # one-step gate of the split form against the oracle on the plan's factors
    wg = p.to_device(W0.astype(np.complex64).astype(np.complex128))
    p.step("lawson4", wg, 1)
    torch.cuda.synchronize()
    acts = [[fo.FourierAction([p.get_factor(f, mu, which) for mu in range(2)]) for f in range(2)]
            for which in (0, 1)]
    E = lambda X: np.stack([acts[0][0](X[0]), acts[0][1](X[1])])  # noqa: E731
    H = lambda X: np.stack([acts[1][0](X[0]), acts[1][1](X[1])])  # noqa: E731
    ref = steppers.lawson4_step(W0.astype(np.complex64).astype(np.complex128), E, H, tau,
                                co.CoupledNonlinearity(co.PAPER))
    from oracle import metrics
    got = p.to_host(wg)
    gate = (metrics.rel_l2(got, ref), metrics.rel_linf(got, ref))
    split_state = p.to_host(w)
    p.destroy()
    # MFMA work of a step: 4 actions x 2 fields x (n1 + n2) x 8 N flops (FP64
    # embedding), six bf16 term products each in the split form
    alg = 4 * 2 * 8 * (n[0] * n[1]) * (n[0] + n[1])
    fp64 = None
    if not args.no_fp64:
        p64, w64, t64 = timed("fp64")
        ms64 = float(np.median(t64))
        traj = metrics.rel_linf(split_state, p64.to_host(w64))
        fp64 = {"value": pts * K / (ms64 * 1e-3), "ms_per_step": ms64 / K, "replays_ms": t64,
                "mfma_tflops": alg / (ms64 / K * 1e-3) / 1e12,
                "frac": alg / (ms64 / K * 1e-3) / 1e12 / MI355X_PEAK_FP64_TFLOPS,
                "split_vs_fp64_rel_linf_after_steps": traj}
        p64.destroy()
    rec = {
        "metric": "grid-point-steps/s (per field) at rel-L2 <=1e-6 vs FP64 oracle",
        "value": pts * K / (ms * 1e-3), "unit": "grid-point-steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": ms / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16x3->f32 (split), state c64",
        "data": "synthetic (the paper's soliton datum, computed by the library)",
        "config": {"workload": "t5_coupled_cq2d_700x350_periodic: coupled cubic-quintic CGL, "
                               f"Lawson4, tau={tau:.6g}", "grid": list(n), "fields": 2,
                   "method": "lawson4", "parallelism": "single-gpu"},
        "replays_ms": times,
        "roofline": {"bound": "mfma", "achieved": 6 * alg / (ms / K * 1e-3) / 1e12,
                     "peak": MI355X_PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": 6 * alg / (ms / K * 1e-3) / 1e12 / MI355X_PEAK_BF16_TFLOPS,
                     "traffic": None,
                     "kernel": "whole step: dense circulant mu-mode products (n = 700, 350) "
                               "and the coupled pointwise kernels"},
        "accuracy": {"one_step_rel_l2_vs_fp64_oracle": gate[0],
                     "one_step_rel_linf_vs_fp64_oracle": gate[1], "gate": 1e-6},
        "fp64_form": fp64, "paper_context": PAPER_TABLE5,
    }
    print(json.dumps(rec))


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: there is no multi-GPU path "
              "(a grid would be slab-decomposed along its slowest axis, one all-to-all "
              "transpose per exponential action)", file=sys.stderr)
        sys.exit(2)
    import torch
    import cgl_inputs as ci
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "c3":
        return bench_batched(args)
    if args.workload == "c4":
        return bench_surrogate(args)
    if args.workload == "t5":
        return bench_coupled(args)
    if args.workload == "t4":
        return bench_fourier(args)
    p, method = workload(args.workload)
    u0 = ci.initial_state(p)
    K, W, R = args.steps, args.warmup, args.replays
    if args.calibrate_copy:
        a = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.ones_like(a)
        a.copy_(b)
        torch.cuda.synchronize()
        del a, b

    plan, u, times = time_form(p, method, "split", K, W, u0, R)
    ms = float(np.median(times))
    value = p.N * K / (ms * 1e-3)
    roof = split_roofline(p, method, times, K)
    gate_l2, gate_linf = one_step_gate(p, method, plan)
    split_state = u.clone()
    plan.destroy()

    # the other method on the same grid and form (Strang beside Lawson4)
    extra = None
    if not args.no_extra and args.workload in ("c2_lawson4", "c2_strang"):
        m2 = "strang" if method == "lawson4" else "lawson4"
        plan2, u2, t2 = time_form(p, m2, "split", K, W, u0, R)
        ms2 = float(np.median(t2))
        r2 = split_roofline(p, m2, t2, K)
        g2 = one_step_gate(p, m2, plan2)
        plan2.destroy()
        del u2
        extra = {"method": m2, "value": p.N * K / (ms2 * 1e-3), "ms_per_step": ms2 / K,
                 "replays_ms": t2, "roofline_frac": r2["frac"], "launch_ms": r2["launch_ms"],
                 "kernel": r2["kernel"], "one_step_rel_l2_vs_fp64_oracle": g2[0],
                 "one_step_rel_linf_vs_fp64_oracle": g2[1]}

    fp64 = None
    traj = None
    if not args.no_fp64:
        plan64, u64, t64 = time_form(p, method, "fp64", K, W, u0, R)
        ms64 = float(np.median(t64))
        d = split_state.to(torch.complex128) - u64
        traj = {"rel_l2": float(torch.linalg.vector_norm(d).item()
                                / torch.linalg.vector_norm(u64).item()),
                "rel_linf": float(d.abs().max().item() / u64.abs().max().item())}
        nl64 = launches_per_step(method, p.d, False)
        alg_flops = 8.0 * p.N * p.n[0]
        fp64 = {"value": p.N * K / (ms64 * 1e-3), "ms_per_step": ms64 / K, "replays_ms": t64,
                "mfma_tflops": alg_flops / ((ms64 / (K * nl64)) * 1e-3) / 1e12,
                "peak_tflops": MI355X_PEAK_FP64_TFLOPS,
                "note": "two actions per Lawson4 round as concurrent graph branches; "
                        "TFLOP/s over the timed region"}
        fp64["frac"] = fp64["mfma_tflops"] / MI355X_PEAK_FP64_TFLOPS
        plan64.destroy()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(p, method, args.cpu_budget_s, args.cpu_max_steps)

    tkey = {"c1": "c1", "c2_lawson4": "c2_lawson4"}.get(args.workload)
    traffic = None
    if tkey in SPLIT_TRAFFIC and paired_lawson4(method) and \
            split_sources_digest() == SPLIT_TRAFFIC[tkey]["sources_sha256_16"]:
        traffic = SPLIT_TRAFFIC[tkey]["bytes_per_launch"]
    roof["traffic"] = traffic
    bc = "Neumann" if p.bc else "Dirichlet"
    rec = {
        "metric": "grid-point-steps/s at rel-L2 <=1e-6 vs FP64 oracle; MFMA util % of peak",
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3->f32 (split), state c64",
        "data": "synthetic",
        "config": {"workload": f"{p.name}: 3-D cubic-quintic CGL {'x'.join(map(str, p.n))} "
                               f"{bc}, 2nd-order FD, {method}, tau={p.tau}, split-precision form",
                   "grid": list(p.n), "method": method, "tau": p.tau,
                   "parallelism": "single-gpu"},
        "replays_ms": times,
        "roofline": roof,
        "accuracy": {"one_step_rel_l2_vs_fp64_oracle": gate_l2,
                     "one_step_rel_linf_vs_fp64_oracle": gate_linf, "gate": 1e-6,
                     "trajectory_vs_fp64_form": traj, "trajectory_steps": K},
        "other_method": extra,
        "fp64_form": fp64,
        "cpu_baseline": cpu,
        "paper_context": PAPER_TABLE3,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
