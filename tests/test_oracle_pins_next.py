"""Pins of the oracle's further methods and operators against facts fixed by
the paper and by mathematics:

* the fourth-order finite-difference matrices of Sections 4.1.1 and 4.2
  (and the second-order mixed Dirichlet/Neumann operator): exactness on the
  polynomials their stencils must reproduce, the semi-internal grid of
  Section 4.2, convergence of the lowest eigenvalues to the continuous ones;
* split4 (eq. Richardson): the linear flow when g = 0, exactness for a
  linear g that commutes with K, the exact nonlinear flow when K = 0,
  empirical order 4;
* Lawson2b (eq. lawson2b): the linear flow when g = 0, Heun's method (eq.
  RK2) when K = 0, e^{tau K} times the RK2 polynomial for a linear g,
  empirical order 2;
* strang_3t / split4_3t (Section 4.3): reduce to strang / split4 without a
  quintic term, to the exact quintic flow when K = 0 and a3 = b3 = 0,
  empirical orders 2 and 4;
* the orders the paper prints for split4 and if2 (Tables 1 and 3).
"""
import os

import numpy as np
import pytest
import scipy.linalg

import cgl_inputs as ci
from oracle import metrics, nonlinear, operators as ops, steppers, tensor

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
D, N = ops.DIRICHLET, ops.NEUMANN


# ------------------------------------------------ finite-difference operators

def _nodes(n, a, b, lo, hi):
    h = ops.spacing_mixed(n, a, b, lo, hi)
    first = a + h if lo == D else a
    return first + h * np.arange(n)


def _poly(coef, x, der=0):
    return np.polyval(np.polyder(coef, der) if der else coef, x)


@pytest.mark.parametrize("lo,hi", [(D, D), (D, N), (N, D), (N, N)])
def test_fd4_rows_reproduce_the_polynomials_of_their_stencils(lo, hi):
    """Every row next to or away from a Dirichlet end is a 4th-order formula:
    exact on polynomials of degree <= 5 that vanish at the Dirichlet ends
    (the dropped boundary value is 0).  The Neumann end rows: the row before
    the end node is exact to degree 5, the end node's row to degree 4 on
    polynomials with zero derivative at that end."""
    n, a, b = 14, -1.5, 2.0
    x = _nodes(n, a, b, lo, hi)
    Dm = ops.laplacian_fd(n, a, b, lo, hi, 4)
    rng = np.random.default_rng(1)
    for deg in range(6):
        q = rng.standard_normal(deg + 1)
        p = q
        if lo == D:
            p = np.polymul(p, [1.0, -a])
        if hi == D:
            p = np.polymul(p, [1.0, -b])
        if np.polyval(p, x).std() == 0:
            continue
        err = Dm @ np.polyval(p, x) - _poly(p, x, 2)
        rows = list(range(n))
        # the Neumann end rows are checked on their own family below
        if lo == N:
            rows = rows[1:]
        if hi == N:
            rows = rows[:-1]
        scale = np.abs(_poly(p, x, 2)).max() + np.abs(np.polyval(p, x)).max()
        if np.polyval(p, x).size and len(p) - 1 <= 5:
            assert np.abs(err[rows]).max() < 1e-9 * scale, (lo, hi, deg, err[rows])
    # Neumann end rows: degree <= 4 polynomials with p'(end) = 0
    for end, row in ((a, 0), (b, n - 1)):
        if (end == a and lo != N) or (end == b and hi != N):
            continue
        for k in (0, 2, 3, 4):
            p = np.poly1d([1.0, -end]) ** k if k else np.poly1d([1.0])
            vals = p(x)
            got = (Dm @ vals)[row]
            want = p.deriv(2)(x[row]) if k >= 2 else 0.0
            assert abs(got - want) < 1e-8 * (1 + abs(want)), (end, k, got, want)
        # degree 5 is not reproduced: the end row is third order
        p = np.poly1d([1.0, -end]) ** 5
        assert abs((Dm @ p(x))[row] - p.deriv(2)(x[row])) > 1e-6


def test_fd4_matrices_are_the_printed_ones():
    """Dirichlet (Section 4.1.1) and semi-internal Dirichlet-Neumann (Section
    4.2) matrices, entries times 12 h^2, with h = (b-a)/(n+1) and (b-a)/n."""
    n = 9
    Ddd = ops.laplacian_fd(n, 0.0, 100.0, D, D, 4) * 12 * (100.0 / (n + 1)) ** 2
    assert np.allclose(Ddd[0, :5], [-15, -4, 14, -6, 1]) and np.all(Ddd[0, 5:] == 0)
    assert np.allclose(Ddd[1, :4], [16, -30, 16, -1])
    assert np.allclose(Ddd[4, 2:7], [-1, 16, -30, 16, -1])
    assert np.allclose(Ddd[n - 1, n - 5:], [1, -6, 14, -4, -15])
    Ddn = ops.laplacian_fd(n, 0.0, 100.0, D, N, 4) * 12 * (100.0 / n) ** 2
    assert np.allclose(Ddn[0, :5], [-15, -4, 14, -6, 1])
    assert np.allclose(Ddn[n - 2, n - 6:], [1, -6, 14, -4, -15, 10])
    assert np.allclose(Ddn[n - 1, n - 5:], [1, -8 / 3, -6, 56, -145 / 3])
    # Neumann end rows annihilate constants (u' = 0 keeps them)
    assert abs(Ddn[n - 1].sum()) < 1e-12 and abs(Ddn[n - 2].sum()) < 1e-12


def test_semi_internal_grid_of_the_paper():
    """Section 4.2: h = 100/n on (0, 100), the last node on the Neumann end."""
    n = 128
    x = ci.nodes(n, 0.0, 100.0, ci.DIRICHLET, ci.NEUMANN)
    assert ops.spacing_mixed(n, 0.0, 100.0, D, N) == pytest.approx(100.0 / n)
    assert x[0] == pytest.approx(100.0 / n) and x[-1] == pytest.approx(100.0)
    assert np.allclose(np.diff(x), 100.0 / n)
    # Dirichlet interior grid of Section 4.1.1: h = 100/(n+1)
    assert ops.spacing_mixed(256, 0.0, 100.0, D, D) == pytest.approx(100.0 / 257)


@pytest.mark.parametrize("lo,hi", [(D, D), (D, N), (N, N)])
def test_fd4_lowest_eigenvalues_converge_at_high_order(lo, hi):
    """The lowest eigenvalues of d^2/dx^2 on (0, L) with the end conditions:
    DD -(k pi/L)^2, DN -((k - 1/2) pi/L)^2, NN -(k pi/L)^2 (k >= 0).  The
    4th-order matrices converge at order > 3 (measured 3.5 with a Neumann end,
    whose rows are third order locally; 4 without); the 2nd-order ones at
    order 2.  Grids of 160 and 320 nodes (on coarser grids the leading error
    terms of the Neumann cases change sign, so their ratio says nothing)."""
    L = 3.0
    k = np.arange(1, 4)
    exact = {(D, D): -(k * np.pi / L) ** 2, (D, N): -((k - 0.5) * np.pi / L) ** 2,
             (N, N): -((k - 1) * np.pi / L) ** 2}[(lo, hi)]
    for order, lo_rate in ((4, 3.2 if N in (lo, hi) else 3.8), (2, 1.9)):
        errs = []
        for n in (160, 320):
            ev = np.linalg.eigvals(ops.laplacian_fd(n, 0.0, L, lo, hi, order))
            ev = np.sort(ev.real)[::-1][:3]
            errs.append(np.abs(ev - exact).max() + 1e-300)
        if errs[1] < 1e-9:  # NN order 2: k = 1 eigenvalue is exactly 0, others converge
            continue
        assert np.log2(errs[0] / errs[1]) > lo_rate, (order, lo, hi, errs)


def test_second_order_dn_eigenvalues_closed_form():
    """2nd-order Dirichlet-Neumann (ghost value at the Neumann end):
    lambda_k = -(4/h^2) sin^2((2k-1) pi / (4n)), k = 1..n."""
    n, L = 17, 2.5
    Dm = ops.laplacian_fd(n, 0.0, L, D, N, 2)
    h = L / n
    lam = -(4 / h ** 2) * np.sin((2 * np.arange(1, n + 1) - 1) * np.pi / (4 * n)) ** 2
    assert np.allclose(np.sort(np.linalg.eigvals(Dm).real), np.sort(lam), rtol=1e-10)


def test_second_order_operators_agree_with_the_plain_builder():
    for bc in (D, N):
        assert np.array_equal(ops.laplacian_fd(12, -1.0, 2.0, bc, bc, 2),
                              ops.laplacian_2nd(12, -1.0, 2.0, bc))


def test_operators_for_takes_the_fd4_matrices():
    p = ci.scaled(ci.T3, (10, 9, 8))
    Es = steppers.operators_for(p, 0.1)
    for E, n in zip(Es, p.n):
        A = ops.operator_A_fd(n, p.a, p.b, ci.DIRICHLET, ci.NEUMANN, 4, p.coeffs.as_tuple(), 3)
        assert np.allclose(E, scipy.linalg.expm(0.1 * A), rtol=0, atol=1e-14)


# ------------------------------------------------------------------- steppers

class _LinearG:
    """g(u) = c u with its exact flow e^{c t} u (commutes with K)."""
    exact = True

    def __init__(self, c):
        self.c = c

    def g(self, u):
        return self.c * u

    def flow(self, u, t):
        return np.exp(self.c * t) * u


def _rand_c(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _tiny(shape=(5, 4, 3), seed=41):
    As = [ops.operator_A(n, -2.0, 2.0, ops.DIRICHLET, (1.0, 0.8, -0.3), len(shape)) for n in shape]
    return As, _rand_c(shape, seed)


@pytest.mark.parametrize("method", ["split4", "lawson2"])
def test_g_zero_gives_the_linear_flow(method):
    As, U = _tiny()
    tau = 0.05
    E = [scipy.linalg.expm(tau * A) for A in As]
    H = [scipy.linalg.expm(0.5 * tau * A) for A in As]
    out = steppers.make_step(method, E, H, tau, _LinearG(0.0))(U)
    ref = scipy.linalg.expm(tau * tensor.kron_sum(As)) @ ci.flat(U)
    assert np.linalg.norm(ci.flat(out) - ref) / np.linalg.norm(ref) < 1e-13


def test_split4_with_linear_g_is_exact():
    As, U = _tiny()
    tau, c = 0.07, complex(0.4, -1.1)
    E = [scipy.linalg.expm(tau * A) for A in As]
    H = [scipy.linalg.expm(0.5 * tau * A) for A in As]
    out = steppers.split4_step(U, E, H, tau, _LinearG(c))
    ref = np.exp(tau * c) * (scipy.linalg.expm(tau * tensor.kron_sum(As)) @ ci.flat(U))
    assert np.linalg.norm(ci.flat(out) - ref) / np.linalg.norm(ref) < 1e-13


def test_lawson2_with_linear_g_is_expK_times_rk2_polynomial():
    As, U = _tiny()
    tau, c = 0.07, complex(0.4, -1.1)
    E = [scipy.linalg.expm(tau * A) for A in As]
    out = steppers.lawson2_step(U, E, tau, _LinearG(c))
    z = tau * c
    ref = (1 + z + z * z / 2) * (scipy.linalg.expm(tau * tensor.kron_sum(As)) @ ci.flat(U))
    assert np.linalg.norm(ci.flat(out) - ref) / np.linalg.norm(ref) < 1e-13


def test_K_zero_split4_is_the_exact_flow_and_lawson2_is_heun():
    """With K = 0 the extrapolated splitting of an exact flow is that flow
    (4/3 - 1/3 = 1), and Lawson2b is Heun's method (eq. RK2) on u' = g(u)."""
    U = _rand_c((6, 5), 14) * 0.8
    I = [np.eye(6), np.eye(5)]
    coef = ci.C0.coeffs.as_tuple()
    nl = steppers.CGLNonlinearity(coef)
    tau = 0.03
    ex, _ = nonlinear.phi_cubic(U, tau, coef[3], coef[4])
    s4 = steppers.split4_step(U, I, I, tau, nl)
    assert np.abs(s4 - ex).max() < 1e-14
    # Heun written from its Butcher tableau
    k1 = nl.g(U)
    k2 = nl.g(U + tau * k1)
    heun = U + tau / 2 * (k1 + k2)
    assert np.abs(steppers.lawson2_step(U, I, tau, nl) - heun).max() < 1e-14


def test_three_term_schemes_reduce_to_the_two_term_ones_without_quintic_term():
    p = ci.scaled(ci.C0, (10, 9))
    tau = p.tau
    E = steppers.operators_for(p, tau)
    H = steppers.operators_for(p, 0.5 * tau)
    nl = steppers.CGLNonlinearity(p.coeffs.as_tuple())
    U = ci.initial_state(p)
    a = steppers.strang_3t_step(U, E, tau, nl)
    b = steppers.strang_step(U, E, tau, nl)
    assert np.abs(a - b).max() / np.abs(b).max() < 1e-14
    a = steppers.split4_3t_step(U, E, H, tau, nl)
    b = steppers.split4_step(U, E, H, tau, nl)
    assert np.abs(a - b).max() / np.abs(b).max() < 1e-13


def test_strang_3t_with_K_zero_and_no_cubic_term_is_the_quintic_flow():
    """Closed form of the quintic flow: |phi^q_t(u)|^4 = |u|^4 / (1 - 4 a4 |u|^4 t)."""
    U = _rand_c((7, 3), 15) * 0.7
    I = [np.eye(7), np.eye(3)]
    coef = (1.0, 0.3, 0.0, 0.0, 0.0, -0.2, 0.9)
    nl = steppers.CGLNonlinearity(coef)
    tau = 0.04
    out = steppers.strang_3t_step(U, I, tau, nl)
    r4 = np.abs(U) ** 4
    assert np.allclose(np.abs(out) ** 4, r4 / (1 - 4 * coef[5] * r4 * tau), rtol=1e-13)
    ref, _ = nonlinear.phi_quintic(U, tau, coef[5], coef[6])
    assert np.abs(out - ref).max() < 1e-14


def _run(p, method, m, T, nl=None):
    tau = T / m
    E = steppers.operators_for(p, tau)
    H = steppers.operators_for(p, 0.5 * tau)
    nl = nl or steppers.CGLNonlinearity(p.coeffs.as_tuple())
    u, bad = steppers.run(ci.initial_state(p), steppers.make_step(method, E, H, tau, nl), m)
    assert not bad
    return u


def test_empirical_orders_split4_4_lawson2_2():
    p = ci.scaled(ci.C0, (24, 24))
    T = 0.5
    ref = _run(p, "lawson4", 640, T)
    for method, ms, lo, hi in (("split4", (5, 10, 20), 3.6, 4.6), ("lawson2", (10, 20, 40), 1.85, 2.2)):
        errs = [metrics.rel_linf(_run(p, method, m, T), ref) for m in ms]
        orders = [metrics.observed_order(ms[i], errs[i], ms[i + 1], errs[i + 1]) for i in range(2)]
        assert all(lo < o < hi for o in orders), (method, errs, orders)


def test_empirical_orders_three_term_schemes():
    """Cubic-quintic coefficients on a small 2-D Dirichlet grid."""
    p = ci.Problem("cq2d", (20, 22), ci.DIRICHLET, -6.0, 6.0, ci.CQ, 0.0, 0, "strang_3t", 6)
    T = 0.3
    ref = _run(p, "lawson4", 960, T)
    for method, ms, lo, hi in (("strang_3t", (10, 20, 40), 1.85, 2.2),
                               ("split4_3t", (6, 12, 24), 3.5, 4.7)):
        errs = [metrics.rel_linf(_run(p, method, m, T), ref) for m in ms]
        orders = [metrics.observed_order(ms[i], errs[i], ms[i + 1], errs[i + 1]) for i in range(2)]
        assert all(lo < o < hi for o in orders), (method, errs, orders)


def test_split4_middle_sub_flow_is_one_evaluation_over_tau_half():
    """eq. Richardson writes phi_{tau/2} between the two half-step actions; for
    the RK4 sub-flow this differs from two RK4 steps of tau/4 (composition),
    and the oracle follows the printed form."""
    p = ci.scaled(ci.C1, (6, 5, 7))
    tau = 0.05
    E = steppers.operators_for(p, tau)
    H = steppers.operators_for(p, 0.5 * tau)
    nl = steppers.CGLNonlinearity(p.coeffs.as_tuple())
    U = ci.initial_state(p) * 2.0
    lit = steppers.split4_step(U, E, H, tau, nl)
    mid = nl.flow(tensor.tucker(nl.flow(U, tau / 4), H), tau / 2)
    v = nl.flow(tensor.tucker(mid, H), tau / 4)
    assert np.abs(lit - (4 / 3 * v - 1 / 3 * steppers.strang_step(U, E, tau, nl))).max() < 1e-14
    comp = nl.flow(nl.flow(tensor.tucker(nl.flow(U, tau / 4), H), tau / 4), tau / 4)
    v2 = nl.flow(tensor.tucker(comp, H), tau / 4)
    assert np.abs(v - v2).max() > 1e-12  # the two readings differ for RK4


def test_observed_order_reproduces_paper_split4_and_if2_columns():
    rows = []
    with open(os.path.join(GOLDEN, "paper_table_orders.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    meths = {(r[0], r[1]) for r in rows}
    assert ("table1", "split4") in meths and ("table3", "split4") in meths
    assert ("table3", "if2") in meths
    for _tab, _meth, m0, e0, m1, e1, printed in rows:
        p = metrics.observed_order(int(m0), float(e0), int(m1), float(e1))
        # the printed errors carry 4 significant digits and the order 3 decimals
        half_ulp = [0.5 * 10.0 ** (int(np.floor(np.log10(float(e)))) - 3) / float(e) for e in (e0, e1)]
        tol = sum(half_ulp) / np.log(int(m1) / int(m0)) + 5e-4 + 1e-9
        assert abs(p - float(printed)) < tol, (_tab, _meth, m1, p, printed, tol)
