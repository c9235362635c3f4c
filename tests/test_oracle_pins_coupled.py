"""Pins of the oracle's coupled two-field system (Section 4.4, eq. coupled):
without advection and cross-coupling each field is the single-field Fourier
solution; pure advection over one grid spacing is an exact shift; the
cross-coupling term has the closed-form flow of |u|^2 = |v|^2 and conserves
|u|^2 - |v|^2 pointwise; the system's mirror symmetry (x1 -> L - x1 with
u <-> v) is preserved by every stepper; Strang / Lawson2b reach order 2 and
split4 / Lawson4 order 4; the soliton datum is stationary at T = 25."""
import numpy as np
import pytest

from oracle import coupled as co, fourier as fo, metrics, steppers


def _smooth(n1, n2, seed, lo=(0.0, 0.0), hi=(2 * np.pi, 2 * np.pi)):
    """A band-limited complex field (modes |k| <= 3, no Nyquist component)."""
    rng = np.random.default_rng(seed)
    x = fo.nodes(n1, lo[0], hi[0])
    y = fo.nodes(n2, lo[1], hi[1])
    L1, L2 = hi[0] - lo[0], hi[1] - lo[1]
    u = np.zeros((n1, n2), dtype=np.complex128)
    for k1 in range(-3, 4):
        for k2 in range(-2, 3):
            c = (rng.standard_normal() + 1j * rng.standard_normal()) / (1 + k1 * k1 + k2 * k2)
            u += c * np.exp(2j * np.pi * (k1 * (x[:, None] - lo[0]) / L1 + k2 * (y[None, :] - lo[1]) / L2))
    return u / np.abs(u).max()


def _run(c, n, lo, hi, method, m, T, W0):
    tau = T / m
    E = co.CoupledAction(n, lo, hi, c, tau)
    H = co.CoupledAction(n, lo, hi, c, 0.5 * tau)
    nl = co.CoupledNonlinearity(c)
    W, bad = steppers.run(W0, steppers.make_step(method, E, H, tau, nl), m)
    assert not bad
    return W


@pytest.mark.parametrize("method", ["strang", "split4", "lawson2", "lawson4"])
def test_uncoupled_fields_are_single_field_solutions(method):
    c = co.CoupledCoeffs(a0=0.0, a1=0.6, b1=0.9, a2=0.3, a3=-1.0, b3=0.7, a4=-0.2, b4=0.4, a5=0.0)
    n, lo, hi = (12, 10), (0.0, 0.0), (5.0, 4.0)
    W0 = np.stack([_smooth(*n, 1, lo, hi), _smooth(*n, 2, lo, hi)])
    W = _run(c, n, lo, hi, method, 4, 0.2, W0)
    cq = (c.a1, c.b1, c.a2, c.a3, c.b3, c.a4, c.b4)
    tau = 0.05
    for f in range(2):
        E = fo.FourierAction([fo.exp_factor(n[mu], lo[mu], hi[mu], cq, 2, tau) for mu in range(2)])
        H = fo.FourierAction([fo.exp_factor(n[mu], lo[mu], hi[mu], cq, 2, 0.5 * tau) for mu in range(2)])
        ref, _ = steppers.run(W0[f], steppers.make_step(method, E, H, tau, steppers.CGLNonlinearity(cq)), 4)
        assert metrics.rel_linf(W[f], ref) < 1e-14


def test_advection_over_one_grid_spacing_is_a_shift():
    """u_t = a0 d_1 u: u(t, x) = u0(x + a0 t); with a0 t = h the grid values
    move by one node (band-limited data, so the spectral derivative is exact)."""
    n1, n2, L = 16, 6, 2 * np.pi
    a0 = 0.7
    c = co.CoupledCoeffs(a0=a0, a1=0.0, b1=0.0, a2=0.0, a3=0.0, b3=0.0, a4=0.0, b4=0.0, a5=0.0)
    t = (L / n1) / a0
    act = co.CoupledAction((n1, n2), (0.0, 0.0), (L, L), c, t)
    u = _smooth(n1, n2, 3)
    W = act(np.stack([u, u]))
    assert np.abs(W[0] - np.roll(u, -1, axis=0)).max() < 1e-13   # u moves with +a0 d_1
    assert np.abs(W[1] - np.roll(u, 1, axis=0)).max() < 1e-13    # v with -a0 d_1


def test_cross_coupling_flow():
    """With only a5: d|u|^2/dt = 2 a5 |v|^2 |u|^2 and symmetrically, so
    |u|^2 - |v|^2 is conserved and, where |u| = |v| = r0,
    r^2 = r0^2 / (1 - 2 a5 r0^2 t); the phases do not move (a5 real)."""
    c = co.CoupledCoeffs(a0=0.0, a1=0.0, b1=0.0, a2=0.0, a3=0.0, b3=0.0, a4=0.0, b4=0.0, a5=0.5)
    nl = co.CoupledNonlinearity(c)
    r0 = np.array([0.2, 0.5, 0.8, 1.0])
    ph = np.array([0.3, -1.2, 2.0, 0.0])
    W = np.stack([r0 * np.exp(1j * ph), r0 * np.exp(-1j * ph)])
    t, m = 0.3, 200
    for _ in range(m):
        W = nl.flow(W, t / m)
    exact = r0 ** 2 / (1 - 2 * c.a5 * r0 ** 2 * t)
    assert np.abs(np.abs(W[0]) ** 2 - exact).max() < 1e-10
    assert np.abs(np.angle(W[0]) - ph).max() < 1e-12
    rng = np.random.default_rng(7)
    W0 = rng.standard_normal((2, 9)) + 1j * rng.standard_normal((2, 9))
    W1 = nl.flow(nl.flow(W0, 0.01), 0.01)
    d0 = np.abs(W0[0]) ** 2 - np.abs(W0[1]) ** 2
    d1 = np.abs(W1[0]) ** 2 - np.abs(W1[1]) ** 2
    assert np.abs(d1 - d0).max() < 1e-9 * np.abs(W0).max() ** 2


@pytest.mark.parametrize("method", ["strang", "split4", "lawson2", "lawson4"])
def test_mirror_symmetry_is_preserved(method):
    c = co.PAPER
    n, lo, hi = (16, 6), (0.0, 0.0), (70.0 / 5, 35.0 / 5)
    u0 = _smooth(*n, 4, lo, hi)
    W0 = np.stack([u0, co.mirror(u0)])
    W = _run(c, n, lo, hi, method, 5, 0.25, W0)
    assert np.abs(W[1] - co.mirror(W[0])).max() < 1e-13 * np.abs(W).max()
    assert metrics.rel_linf(W[0], u0) > 1e-3   # the system moved


def test_empirical_orders():
    c = co.PAPER
    n, lo, hi = (20, 8), (0.0, 0.0), (14.0, 7.0)
    u0 = _smooth(*n, 5, lo, hi)
    W0 = np.stack([u0, _smooth(*n, 6, lo, hi)])
    T = 0.4
    ref = _run(c, n, lo, hi, "lawson4", 640, T, W0)
    for method, ms, lo_o, hi_o in (("strang", (10, 20, 40), 1.85, 2.2), ("lawson2", (10, 20, 40), 1.8, 2.2),
                                   ("split4", (5, 10, 20), 3.5, 4.7), ("lawson4", (10, 20, 40), 3.5, 4.6)):
        errs = [metrics.rel_linf(_run(c, n, lo, hi, method, m, T, W0), ref) for m in ms]
        orders = [metrics.observed_order(ms[i], errs[i], ms[i + 1], errs[i + 1]) for i in range(2)]
        assert all(lo_o < o < hi_o for o in orders), (method, errs, orders)


def test_soliton_datum_is_stationary():
    """Section 4.4: after T_st = 25 the 1-D soliton no longer changes
    qualitatively; one more time unit moves |w| by well under 1%."""
    c = co.PAPER
    w = co.soliton_datum(700, 0.0, 70.0, c)
    w_more = co.soliton_datum(700, 0.0, 70.0, c, m=10400, T=26.0)
    assert np.abs(np.abs(w_more) - np.abs(w)).max() < 1e-2 * np.abs(w).max()
    assert 0.5 < np.abs(w).max() < 3.0     # a localised pulse, neither decayed nor blown up
    x = fo.nodes(700, 0.0, 70.0)
    assert np.abs(w)[np.abs(x - 17.5) > 20].max() < 1e-2 * np.abs(w).max()
