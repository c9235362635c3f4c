"""GPU parity of the split-precision form (bf16x3 terms, FP32 accumulation)
against the FP64 oracle.

Kernel level (relative 2-norm): one mu-mode product / Tucker operator on the
complex64 input, compared with the FP64 product of the same input; the
error budget is the FP32 rounding of the result (~6e-8) plus the dropped
term products (~1e-7), so the bound is 1e-6.
Step level: one Strang / Lawson4 step from an identical input must stay
within 1e-6 of the FP64 oracle step (the split form's accuracy target);
trajectory errors over many steps are reported, not gated.
"""
import numpy as np
import pytest

import cgl_inputs as ci
from oracle import tensor
from tests._util import assert_close, errors, log, make_plan, oracle_run, plan_ops, require_gpu

pytestmark = pytest.mark.gpu

SHAPES = [(150,), (64, 45), (130, 70), (20, 33, 17), (64, 64, 40), (3, 5, 4), (128, 33, 9)]


def _c64(u):
    return u.astype(np.complex64).astype(np.complex128)


def _random_plan(shape, seed, master=False):
    from paper_2403_02816_amd import cgl
    p = cgl.Plan(shape, ci.C0.coeffs, 0.01, precision="split", master=master)
    Es, Hs = [], []
    for mu, n in enumerate(shape):
        E = ci.random_complex((n, n), seed + 10 * mu) / np.sqrt(n)
        H = ci.random_complex((n, n), seed + 10 * mu + 1) / np.sqrt(n)
        p.set_exponentials(mu, E, H)
        Es.append(E)
        Hs.append(H)
    return p, Es, Hs


@pytest.mark.parametrize("shape", SHAPES)
def test_split_mode_product_every_mu(shape):
    torch = require_gpu()
    p, Es, Hs = _random_plan(shape, 300)
    U = _c64(ci.random_complex(shape, 17))
    x = p.to_device(U, dtype=torch.complex64)
    out = torch.empty_like(x)
    for mu in range(len(shape)):
        for which, Ms in ((0, Es), (1, Hs)):
            log(f"split mode_product shape={shape} mu={mu} which={which}")
            p.mode_product(mu, which, x, out)
            torch.cuda.synchronize()
            assert_close(p.to_host(out), tensor.mode_product(U, Ms[mu], mu), 1e-6,
                         f"split mode {shape} mu={mu} which={which}")
    p.destroy()


@pytest.mark.parametrize("shape", SHAPES)
def test_split_tucker(shape):
    torch = require_gpu()
    p, Es, Hs = _random_plan(shape, 400)
    U = _c64(ci.random_complex(shape, 18))
    x = p.to_device(U, dtype=torch.complex64)
    out = torch.empty_like(x)
    p.tucker(1, x, out)
    torch.cuda.synchronize()
    assert_close(p.to_host(out), tensor.tucker(U, Hs), 1e-6, f"split tucker {shape}")


def _one_step_gate(p, method, master=False, rk4_flow=False, steps=1):
    torch = require_gpu()
    plan = make_plan(p, "split", master=master, rk4_flow=rk4_flow)
    u0 = ci.initial_state(p)
    if not master:
        u0 = _c64(u0)
    u = plan.to_device(u0)
    if method == "strang":
        plan.step_strang(u, steps)
    else:
        plan.step_lawson4(u, steps)
    torch.cuda.synchronize()
    assert plan.status() == 0
    E, H = plan_ops(plan)
    ref = oracle_run(p, u0, method, steps, E, H, rk4_flow=rk4_flow)
    got = plan.to_host(u)
    plan.destroy()
    l2, linf = errors(got, ref)
    log(f"split {p.name} {method} master={master} steps={steps} rel-L2 {l2:.3e} rel-Linf {linf:.3e}")
    return l2, linf


def _gate(p, method, **kw):
    """The split form's accuracy target for one step: both measures <= 1e-6."""
    l2, linf = _one_step_gate(p, method, **kw)
    assert l2 < 1e-6 and linf < 1e-6, (p.name, method, kw, l2, linf)


@pytest.mark.parametrize("method", ["strang", "lawson4"])
def test_split_one_step_gate_c0(method):
    _gate(ci.C0, method)


@pytest.mark.parametrize("method", ["strang", "lawson4"])
@pytest.mark.parametrize("master", [False, True])
def test_split_one_step_gate_c1_shape(method, master):
    _gate(ci.scaled(ci.C1, (40, 36, 44)), method, master=master)


@pytest.mark.parametrize("method", ["strang", "lawson4"])
def test_split_one_step_gate_c2_shape(method):
    _gate(ci.scaled(ci.C2, (48, 40, 52)), method)


def test_split_one_step_gate_c1_full_size():
    _gate(ci.C1, "lawson4")


@pytest.mark.parametrize("method", ["strang", "lawson4"])
def test_split_one_step_gate_c2_full_size(method):
    """256^3 Dirichlet cubic-quintic, the full grid (the oracle takes ~10 s)."""
    _gate(ci.C2, method)


def test_split_trajectory_error_is_reported():
    p = ci.scaled(ci.C1, (32, 32, 32))
    err = _one_step_gate(p, "lawson4", steps=40)
    errm = _one_step_gate(p, "lawson4", master=True, steps=40)
    log(f"split 32^3 Lawson4 40 steps: c64 state {err}, FP64 master {errm}")
    assert max(err + errm) < 1e-3


def test_split_graph_replay_equals_eager_bitwise():
    torch = require_gpu()
    p = ci.scaled(ci.C1, (20, 18, 22))
    plan = make_plan(p, "split")
    u0 = ci.initial_state(p)
    a = plan.to_device(u0)
    b = plan.to_device(u0)
    plan.step_lawson4(a, 12)
    assert plan.run("lawson4", b, 12, 5) == 0
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan.destroy()


@pytest.mark.parametrize("tile", ["0", "1", "2", "3"])
def test_split_every_tile_shape(tile, monkeypatch):
    """Every compiled tile shape (64 rows x 32-deep and 128 rows x 16-deep
    stages staged through registers; 64 x 16 and 128 x 16 copied straight to
    LDS), forced instead of autotuned: kernel parity on a ragged shape (the
    single mode products of the direct-to-LDS shapes run on the 128 x 16
    register shape: they need a contiguous axis) and the one-step gate."""
    monkeypatch.setenv("CGL_SPLIT_TILE", tile)
    torch = require_gpu()
    p, Es, Hs = _random_plan((130, 70, 9), 500)
    U = _c64(ci.random_complex((130, 70, 9), 19))
    x = p.to_device(U, dtype=torch.complex64)
    out = torch.empty_like(x)
    for mu in range(3):
        p.mode_product(mu, 1, x, out)
        torch.cuda.synchronize()
        assert_close(p.to_host(out), tensor.mode_product(U, Hs[mu], mu), 1e-6,
                     f"tile {tile} mode {mu}")
    p.tucker(0, x, out)
    torch.cuda.synchronize()
    assert_close(p.to_host(out), tensor.tucker(U, Es), 1e-6, f"tile {tile} tucker")
    p.destroy()
    # Lawson4 of the two-action form (the paired form ignores the tile
    # choice) and Strang run on the forced shape
    monkeypatch.setenv("CGL_LAWSON_PAIRED", "0")
    for method in ("strang", "lawson4"):
        _gate(ci.scaled(ci.C2, (64, 32, 48)), method)


@pytest.mark.parametrize("shape,method", [((96, 80, 40), "lawson4"), ((130, 70, 9), "strang"),
                                          ((256, 256), "lawson4")])
def test_dma_tiles_match_register_tiles_bitwise(shape, method, monkeypatch):
    """The direct-to-LDS shapes compute the same products in the same order as
    the register-staged shapes with the same rows per workgroup: 64 x 16
    against 64 x 32 and 128 x 16 against 128 x 16, bit for bit.  Lawson4 runs
    as two single-action passes per direction here (the paired pass has its
    own tile choice)."""
    torch = require_gpu()
    from paper_2403_02816_amd import cgl
    monkeypatch.setenv("CGL_LAWSON_PAIRED", "0")
    p = ci.scaled(ci.C1, shape) if len(shape) == 3 else ci.scaled(ci.C0, shape)
    u0 = ci.initial_state(p)
    out = {}
    for tile in ("0", "2", "1", "3"):
        monkeypatch.setenv("CGL_SPLIT_TILE", tile)
        plan = make_plan(p, "split")
        u = plan.to_device(u0)
        assert plan.run(method, u, 4, 4) == 0
        torch.cuda.synchronize()
        out[tile] = plan.to_host(u)
        plan.destroy()
    log(f"dma tiles {shape} {method}: 64-row equal {np.array_equal(out['0'], out['2'])}, "
        f"128-row equal {np.array_equal(out['1'], out['3'])}")
    assert np.array_equal(out["0"], out["2"])
    assert np.array_equal(out["1"], out["3"])


@pytest.mark.parametrize("shape,master", [((128, 128, 128), False), ((96, 80, 40), True),
                                          ((130, 70, 9), False), ((256, 256), False)])
def test_paired_lawson4_matches_concurrent_actions_bitwise(shape, master, monkeypatch):
    """Lawson4 with both actions of a round in one paired pass per direction
    computes the same products and stage combinations as the two concurrent
    actions: identical bits (complex64 and FP64-master states)."""
    torch = require_gpu()
    from paper_2403_02816_amd import cgl
    p = ci.scaled(ci.C1, shape) if len(shape) == 3 else ci.scaled(ci.C0, shape)
    u0 = ci.initial_state(p)
    out = {}
    for paired in ("0", "1"):
        monkeypatch.setenv("CGL_LAWSON_PAIRED", paired)
        plan = make_plan(p, "split", master=master)
        u = plan.to_device(u0)
        assert plan.run("lawson4", u, 3, 3) == 0
        plan.step_lawson4(u, 1)
        torch.cuda.synchronize()
        out[paired] = plan.to_host(u)
        plan.destroy()
    log(f"paired lawson4 {shape} master={master}: equal {np.array_equal(out['0'], out['1'])}")
    assert np.array_equal(out["0"], out["1"])


@pytest.mark.parametrize("shape,master", [((96, 80, 40), False), ((130, 70, 9), True),
                                          ((256, 256), False), ((200, 33, 17), False)])
def test_paired_tile_shapes_agree_bitwise(shape, master, monkeypatch):
    """The paired pass with 64-row tiles (4 waves) and 128-row tiles (8 waves)
    computes every output from the same 16-deep MFMA steps in the same order:
    Lawson4 and Lawson2b steps agree bit for bit."""
    torch = require_gpu()
    p = ci.scaled(ci.C1, shape) if len(shape) == 3 else ci.scaled(ci.C0, shape)
    u0 = ci.initial_state(p)
    out = {}
    for tile in ("2", "3"):
        monkeypatch.setenv("CGL_PAIR_TILE", tile)
        plan = make_plan(p, "split", master=master)
        u = plan.to_device(u0)
        assert plan.run("lawson4", u, 3, 3) == 0
        plan.step("lawson2", u, 2)
        torch.cuda.synchronize()
        out[tile] = plan.to_host(u)
        plan.destroy()
    log(f"paired tiles {shape} master={master}: equal {np.array_equal(out['2'], out['3'])}")
    assert np.array_equal(out["2"], out["3"])
