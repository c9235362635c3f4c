"""Learned surrogate: training data from the batched stepper, training with
the library's own kernels, and the gated run (orchestration only; every
forward, backward, loss, optimiser and stepper operation runs in libcgl).

The network maps u(t) to an estimate of u(t + M tau) for a 2-D cubic
instance on an n x n grid (the C ABI documents it); the plain stepper checks
it at run time and replaces it when it is off.  Its output is a correction
about a base state: u(t) itself ("input"), the exact linear flow
e^{M tau K} u(t) ("linear": the Lawson change of variables of Section 2.2,
one Tucker operator of a plan with step M tau) or one Strang step of size
M tau ("strang").
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

import cgl_inputs as ci

from . import cgl

C = 48
BLOCKS = 4
CIN = 7
KEYS = ("a1", "b1", "a2", "a3", "b3")


def _torch():
    import torch
    return torch


def layer_shapes():
    return [(C, CIN)] + [(C, C)] * BLOCKS + [(2, C)]


def init_params(seed: int, zero_output: bool = False) -> np.ndarray:
    """He-uniform weights (the residual and output layers scaled by 0.1, so
    the initial network is close to its base), zero biases; zero_output: the
    output layer starts at zero, so the initial network is its base."""
    rng = np.random.default_rng(seed)
    parts = []
    shapes = layer_shapes()
    for k, (co, cin) in enumerate(shapes):
        bound = math.sqrt(6.0 / (cin * 9)) * (1.0 if k == 0 else 0.1)
        w = rng.uniform(-bound, bound, size=co * cin * 9)
        if zero_output and k == len(shapes) - 1:
            w[:] = 0.0
        parts.append(w)
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def standardise(coeffs, ranges: Optional[Dict] = None) -> np.ndarray:
    """The five cubic coefficients mapped to [-1, 1] over the sweep's ranges."""
    ranges = ranges or ci.coeff_ranges()
    vals = dict(zip(KEYS, coeffs.as_tuple()[:5]))
    return np.array([2.0 * (vals[k] - ranges[k][0]) / (ranges[k][1] - ranges[k][0]) - 1.0
                     for k in KEYS])


@dataclass
class PairSet:
    """Snapshots s_0 .. s_K of B trajectories, M steps apart, as one device
    tensor of (K + 1) * B samples (sample k * B + j = trajectory j at
    snapshot k); pair (k, j) maps sample k * B + j to sample (k + 1) * B + j."""
    snaps: object                 # complex64 torch tensor ((K + 1) * B * P,)
    cstd: object                  # float32 torch tensor ((K + 1) * B, 5)
    B: int
    K: int
    n: int
    problems: List[ci.Problem] = field(default_factory=list)
    seconds: float = 0.0
    base: str = "input"
    bases: object = None          # complex64 (K * B * P,): base of source sample i

    def pair_ids(self, trajectories: Sequence[int]) -> np.ndarray:
        j = np.asarray(trajectories, dtype=np.int64)
        k = np.arange(self.K, dtype=np.int64)
        return (k[:, None] * self.B + j[None, :]).ravel().astype(np.int32)


def coarse_plan(probs, tau: float, jump: int, batched: bool = True):
    """The plan that propagates a base state: the same instances with step
    jump * tau (its E exponential is e^{jump tau K})."""
    if batched:
        plan = cgl.BatchedPlan([p.n for p in probs], [p.coeffs for p in probs], jump * tau,
                               precision="split")
        plan.set_fd_operators_batched(probs)
    else:
        p = probs[0]
        plan = cgl.Plan(p.n, p.coeffs, jump * tau, precision="split")
        plan.set_fd_operators(p.a, p.b, p.bc, p.coeffs)
    return plan


def apply_base(coarse, base: str, x, out) -> None:
    """out = the base state of x under ``base`` (asynchronous, library kernels)."""
    if base == "linear":
        coarse.tucker(0, x, out)
    elif base == "strang":
        out.copy_(x)
        coarse.step("strang", out, 1)
    else:
        raise ValueError(base)


def generate_pairs(count: int, seed: int, n: int = ci.C4_N, jump: int = ci.C4_JUMP,
                   burn_in: int = 100, pairs: int = 40, tau: float = ci.C3_TAU,
                   base: str = "input") -> PairSet:
    """Run the batched split-precision Lawson4 stepper on ``count`` instances
    of the sweep at n x n and keep a snapshot after the burn-in and every
    ``jump`` steps after it; with base "linear" or "strang", also the base
    state of every source snapshot."""
    torch = _torch()
    probs = ci.batched_sweep(count, seed, fixed_n=n)
    t0 = time.perf_counter()
    plan = cgl.BatchedPlan([p.n for p in probs], [p.coeffs for p in probs], tau, precision="split")
    plan.set_fd_operators_batched(probs)
    P = n * n
    if plan.offsets != [j * P for j in range(count)]:
        raise RuntimeError("instances are not packed back to back")
    u = plan.to_device_batched([ci.initial_state(p) for p in probs])
    st = plan.run("lawson4", u, burn_in)
    snaps = torch.empty(((pairs + 1) * count * P,), dtype=torch.complex64, device="cuda")
    snaps[:count * P].copy_(u)
    for k in range(1, pairs + 1):
        st = st or plan.run("lawson4", u, jump)
        snaps[k * count * P:(k + 1) * count * P].copy_(u)
    torch.cuda.synchronize()
    if st != 0:
        raise RuntimeError(f"stepper status {st} while generating training data")
    cs = np.stack([standardise(p.coeffs) for p in probs]).astype(np.float32)
    cstd = torch.from_numpy(np.tile(cs, (pairs + 1, 1))).to("cuda")
    plan.destroy()
    bases = None
    if base != "input":
        coarse = coarse_plan(probs, tau, jump)
        bases = torch.empty((pairs * count * P,), dtype=torch.complex64, device="cuda")
        for k in range(pairs):
            sl = slice(k * count * P, (k + 1) * count * P)
            apply_base(coarse, base, snaps[sl], bases[sl])
        torch.cuda.synchronize()
        coarse.destroy()
    return PairSet(snaps, cstd, count, pairs, n, probs, time.perf_counter() - t0, base, bases)


def correction_rms(data: PairSet, ids: np.ndarray) -> float:
    """Root mean square over the given pairs and points of |target - base|:
    the size of the correction the network has to learn (its output scale)."""
    torch = _torch()
    P = data.n * data.n
    tot, cnt = 0.0, 0
    for b0 in range(0, len(ids), 256):
        sel = torch.from_numpy(np.asarray(ids[b0:b0 + 256], dtype=np.int64)).to("cuda")
        src = data.snaps.view(-1, P)[sel] if data.bases is None else data.bases.view(-1, P)[sel]
        tgt = data.snaps.view(-1, P)[sel + data.B]
        tot += float(torch.sum(torch.abs(tgt - src) ** 2).item())
        cnt += int(sel.numel()) * P
    return math.sqrt(tot / max(cnt, 1))


def split_trajectories(B: int, frac_train: float = 0.9, seed: int = 0):
    rng = np.random.default_rng(seed)
    perm = rng.permutation(B)
    nt = int(round(frac_train * B))
    return np.sort(perm[:nt]), np.sort(perm[nt:])


def train(sur: cgl.Surrogate, data: PairSet, train_ids: np.ndarray, epochs: int,
          batch: int = 64, lr_max: float = 1e-3, lr_min: float = 1e-5, seed: int = 0,
          log=None) -> List[float]:
    """Adam with a cosine learning-rate decay over all steps; returns the mean
    training loss of every epoch."""
    torch = _torch()
    rng = np.random.default_rng(seed)
    per_epoch = len(train_ids) // batch
    total = max(1, epochs * per_epoch)
    losses = []
    step = 0
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(train_ids).astype(np.int32)).to("cuda")
        for b in range(per_epoch):
            lr = lr_min + 0.5 * (lr_max - lr_min) * (1.0 + math.cos(math.pi * step / total))
            sur.train_step(batch, data.snaps, data.cstd, order[b * batch:(b + 1) * batch],
                           data.B, lr, base=data.bases)
            step += 1
        losses.append(sur.take_loss())
        if log:
            log(f"epoch {ep} loss {losses[-1]:.3e}")
    return losses


def validation_error(sur: cgl.Surrogate, data: PairSet, ids: np.ndarray, batch: int = 64):
    """Relative L2 error of single jumps on the given pairs: (mean, max)."""
    torch = _torch()
    P = data.n * data.n
    batch = min(batch, sur.max_batch)
    errs = []
    out = torch.empty((batch * P,), dtype=torch.complex64, device="cuda")
    for b0 in range(0, len(ids), batch):
        sel = ids[b0:b0 + batch]
        S = len(sel)
        src = torch.cat([data.snaps[int(i) * P:(int(i) + 1) * P] for i in sel])
        tgt = torch.cat([data.snaps[(int(i) + data.B) * P:(int(i) + data.B + 1) * P] for i in sel])
        cs = data.cstd[torch.from_numpy(sel.astype(np.int64)).to("cuda")]
        bs = None
        if data.bases is not None:
            bs = torch.cat([data.bases[int(i) * P:(int(i) + 1) * P] for i in sel])
        sur.forward(S, src, cs, out, base=bs)
        d = (out[:S * P] - tgt).view(S, P)
        e = torch.linalg.vector_norm(d, dim=1) / torch.linalg.vector_norm(tgt.view(S, P), dim=1)
        errs.append(e.cpu().numpy())
    e = np.concatenate(errs)
    return float(e.mean()), float(e.max())
