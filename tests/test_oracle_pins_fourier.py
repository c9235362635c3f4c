"""Pins of the oracle's Fourier path (periodic boundaries, Section 3.2):
Fourier modes are eigenfunctions with the exponential factor of the E
tensor; the per-direction exponential equals the matrix exponential of the
closed-form periodic spectral second-derivative matrix; the action through
the transforms equals the Tucker operator of those matrices; the steppers
are exact for g = 0; split4 and Lawson4 reach orders 4 on a periodic
problem; the Table 4 initial datum is the ten-bead necklace."""
import numpy as np
import pytest
import scipy.linalg

import cgl_inputs as ci
from oracle import fourier as fo, metrics, steppers, tensor


def test_fourier_modes_are_eigenfunctions():
    n, a, b, t = (12, 10), -3.0, 5.0, 0.07
    c = (1.3, -0.6, 0.4)
    x = fo.nodes(n[0], a, b)
    y = fo.nodes(n[1], a, b)
    L = b - a
    for k1, k2 in ((0, 0), (2, -3), (-5, 4), (6, 5)):  # 6 is the Nyquist mode of n = 12
        u = np.exp(2j * np.pi * (k1 * (x[:, None] - a) / L + k2 * (y[None, :] - a) / L))
        act = fo.FourierAction(fo.exp_factors(n, a, b, c, t))
        lam = complex(c[0], c[1]) * -((2 * np.pi / L) ** 2 * (k1 ** 2 + k2 ** 2)) + c[2]
        assert np.abs(act(u) - np.exp(t * lam) * u).max() < 1e-13


@pytest.mark.parametrize("n", [8, 16, 30])
def test_direction_exponential_is_expm_of_the_spectral_second_derivative(n):
    a, b, t, d = 0.0, 7.0, 0.03, 3
    c = (1.0, 0.7, -0.3)
    A = complex(c[0], c[1]) * fo.spectral_second_derivative(n, a, b) + (c[2] / d) * np.eye(n)
    assert np.abs(fo.circulant_exponential(n, a, b, c, d, t) - scipy.linalg.expm(t * A)).max() < 1e-12


def test_fourier_action_equals_tucker_of_the_direction_exponentials():
    shape, a, b, t = (8, 6, 10), -2.0, 4.0, 0.05
    c = (0.5, 0.5, -0.5)
    rng = np.random.default_rng(3)
    U = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    act = fo.FourierAction(fo.exp_factors(shape, a, b, c, t))
    Ms = [fo.circulant_exponential(n, a, b, c, 3, t) for n in shape]
    assert np.abs(act(U) - tensor.tucker(U, Ms)).max() / np.abs(U).max() < 1e-13


def _periodic(n, coeffs, tau):
    return ci.Problem("per", n, ci.PERIODIC, 0.0, 2.0 * np.pi, coeffs, tau, 0, "split4", 5)


def _run(p, method, m, T, u0):
    tau = T / m
    E = fo.actions_for(p, tau)
    H = fo.actions_for(p, 0.5 * tau)
    nl = steppers.CGLNonlinearity(p.coeffs.as_tuple())
    u, bad = steppers.run(u0, steppers.make_step(method, E, H, tau, nl), m)
    assert not bad
    return u


@pytest.mark.parametrize("method", ["strang", "split4", "lawson2", "lawson4"])
def test_steppers_with_g_zero_are_the_fourier_flow(method):
    c = ci.Coeffs(1.0, 0.4, 0.2, 0.0, 0.0)
    p = _periodic((12, 10), c, 0.05)
    rng = np.random.default_rng(4)
    u0 = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    out = _run(p, method, 3, 0.15, u0)
    ref = fo.actions_for(p, 0.15)(u0)
    assert np.abs(out - ref).max() / np.abs(ref).max() < 1e-13


def test_empirical_orders_on_a_periodic_problem():
    c = ci.Coeffs(1.0, 1.5, 0.5, -1.0, 1.0)
    p = _periodic((24, 20), c, 0.0)
    x = fo.nodes(24, 0.0, 2 * np.pi)
    y = fo.nodes(20, 0.0, 2 * np.pi)
    u0 = (0.8 + 0.3 * np.cos(x)[:, None] * np.sin(2 * y)[None, :]) * np.exp(1j * np.cos(y))[None, :]
    T = 0.4
    ref = _run(p, "lawson4", 640, T, u0)
    for method, ms, lo, hi in (("strang", (10, 20, 40), 1.85, 2.2), ("split4", (5, 10, 20), 3.5, 4.6),
                               ("lawson4", (10, 20, 40), 3.5, 4.6)):
        errs = [metrics.rel_linf(_run(p, method, m, T, u0), ref) for m in ms]
        orders = [metrics.observed_order(ms[i], errs[i], ms[i + 1], errs[i + 1]) for i in range(2)]
        assert all(lo < o < hi for o in orders), (method, errs, orders)


def test_table4_datum_is_the_ten_bead_necklace():
    """Section 4.3: delta sech(...) cos(5 theta) e^{3 i theta}: on the circle
    rho = rho0 in the plane z = 0 the modulus peaks at delta ten times."""
    theta = np.linspace(-np.pi, np.pi, 2000, endpoint=False)
    x, y = 6.0 * np.cos(theta), 6.0 * np.sin(theta)
    mod = 1.2 * np.abs(np.cos(5 * np.arctan2(y, x)))
    peaks = np.sum((mod > np.roll(mod, 1)) & (mod >= np.roll(mod, -1)))
    assert peaks == 10 and abs(mod.max() - 1.2) < 1e-6
    u = ci.initial_state(ci.scaled(ci.T4, (32, 32, 32)))
    assert abs(np.abs(u).max() - 1.2) < 0.2
    assert np.abs(u[0, 0, 0]) < 1e-2  # a corner of (-12, 12)^3 is far from the ring
