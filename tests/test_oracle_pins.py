"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks an oracle function against something other than itself:
closed forms, textbook eigen-decompositions, brute-force exp(tau K) on tiny
grids, invariants, special cases that reduce to known maps, and the orders
the paper prints in its tables.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg

import cgl_inputs as ci
from oracle import metrics, nonlinear, operators as ops, steppers, tensor

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
COEF2 = ci.C0.coeffs.as_tuple()
COEF3 = ci.CQ.as_tuple()


# ---------------------------------------------------------------- operators

@pytest.mark.parametrize("bc", [ops.DIRICHLET, ops.NEUMANN])
@pytest.mark.parametrize("n", [5, 17, 64])
def test_laplacian_eigenpairs(bc, n):
    """The sine / cosine bases diagonalise the 2nd-order FD Laplacian."""
    D = ops.laplacian_2nd(n, -3.0, 4.0, bc)
    lam, V = ops.eigen_2nd(n, -3.0, 4.0, bc)
    res = np.linalg.norm(D @ V - V * lam) / (np.linalg.norm(D) * np.linalg.norm(V))
    assert res < 1e-14
    # eigenvalues also agree with a dense symmetric/general eigensolver
    ev = np.sort(np.linalg.eigvals(D).real)
    assert np.allclose(np.sort(lam), ev, rtol=1e-10, atol=1e-10 * abs(lam).max())


def test_neumann_rows_annihilate_constants_and_trapezoid_weights():
    """Neumann rows: D2 1 = 0 (u' = 0 keeps constants) and w^T D2 = 0 for the
    trapezoid weights w = (1/2, 1, ..., 1, 1/2) (discrete mass balance)."""
    n = 11
    D = ops.laplacian_2nd(n, 0.0, 1.0, ops.NEUMANN)
    assert np.abs(D @ np.ones(n)).max() < 1e-12
    w = np.ones(n)
    w[0] = w[-1] = 0.5
    assert np.abs(w @ D).max() < 1e-12
    E = ops.exp_closed_form(n, 0.0, 1.0, ops.NEUMANN, (1.0, 0.7, 0.3), 2, 0.05)
    assert np.allclose(E @ np.ones(n), np.exp(0.05 * 0.3 / 2) * np.ones(n), rtol=1e-13, atol=0)


def test_dirichlet_operator_is_tridiagonal_with_diagonal_shift():
    c = (1.3, -0.4, 0.6)
    A = ops.operator_A(7, 0.0, 8.0, ops.DIRICHLET, c, 3)
    h = 1.0
    assert A[3, 3] == pytest.approx(complex(1.3, -0.4) * (-2.0) / h ** 2 + 0.2)
    assert A[3, 4] == pytest.approx(complex(1.3, -0.4) / h ** 2)
    assert A[0, 2] == 0 and A[6, 4] == 0


@pytest.mark.parametrize("bc", [ops.DIRICHLET, ops.NEUMANN])
@pytest.mark.parametrize("n,t", [(8, 0.3), (64, 1e-2), (128, 5e-3), (33, 2.0)])
def test_exp_closed_form_vs_scipy_expm(bc, n, t):
    A = ops.operator_A(n, -10.0, 10.0, bc, COEF3, 3)
    E1 = ops.exp_closed_form(n, -10.0, 10.0, bc, COEF3, 3, t)
    E2 = ops.exp_scipy(A, t)
    assert np.linalg.norm(E1 - E2) / np.linalg.norm(E2) < 5e-15


# ---------------------------------------------------------------- tensors

def _rand_c(shape, seed):
    return ci.random_complex(shape, seed)


def test_mode_product_matches_elementwise_definition():
    U = _rand_c((3, 4, 2), 1)
    M = _rand_c((4, 4), 2)
    Y = tensor.mode_product(U, M, 1)
    ref = np.zeros_like(U)
    for i in range(3):
        for k in range(4):
            for l in range(2):
                ref[i, k, l] = sum(M[k, j] * U[i, j, l] for j in range(4))
    assert np.abs(Y - ref).max() < 1e-14


@pytest.mark.parametrize("shape", [(6,), (4, 5), (4, 5, 3)])
def test_tucker_equals_bruteforce_expm_of_kronecker_sum(shape):
    """eq. (Tucker): exp(tau K) vec(U) = vec(U x_1 e^{tau A_1} ... x_d e^{tau A_d})
    with K the Kronecker sum of eq. (ODEs) and column-stacking vec."""
    As = [_rand_c((n, n), 10 + i) * 0.3 for i, n in enumerate(shape)]
    tau = 0.7
    U = _rand_c(shape, 3)
    K = tensor.kron_sum(As)
    lhs = scipy.linalg.expm(tau * K) @ ci.flat(U)
    rhs = ci.flat(tensor.tucker(U, [scipy.linalg.expm(tau * A) for A in As]))
    assert np.linalg.norm(lhs - rhs) / np.linalg.norm(lhs) < 1e-13


@pytest.mark.parametrize("shape", [(6,), (4, 5), (4, 5, 3)])
def test_kronsumv_equals_assembled_K(shape):
    As = [_rand_c((n, n), 20 + i) for i, n in enumerate(shape)]
    U = _rand_c(shape, 4)
    lhs = tensor.kron_sum(As) @ ci.flat(U)
    rhs = ci.flat(tensor.kronsumv(U, As))
    assert np.linalg.norm(lhs - rhs) / np.linalg.norm(lhs) < 1e-13


def test_tucker_mode_order_invariance_and_d1_matvec():
    shape = (5, 4, 6)
    Ms = [_rand_c((n, n), 30 + i) for i, n in enumerate(shape)]
    U = _rand_c(shape, 5)
    ref = tensor.tucker(U, Ms)
    for order in [(2, 1, 0), (1, 0, 2), (0, 2, 1)]:
        Y = U
        for mu in order:
            Y = tensor.mode_product(Y, Ms[mu], mu)
        assert np.abs(Y - ref).max() < 1e-12
    v = _rand_c((7,), 6)
    M = _rand_c((7, 7), 7)
    assert np.abs(tensor.tucker(v, [M]) - M @ v).max() < 1e-13


# ---------------------------------------------------------------- nonlinear

def _fine_rk4(u, t, g, m=4000):
    h = t / m
    for _ in range(m):
        u = nonlinear.rk4_flow(u, h, g)
    return u


@pytest.mark.parametrize("a3,b3,t", [(-1.0, 0.2, 0.05), (-1.0, 1.0, 0.05), (1.2, 1.0, 1e-3), (0.4, -0.7, 0.3)])
def test_exact_cubic_flow_vs_fine_rk4_and_modulus_law(a3, b3, t):
    u0 = _rand_c((50,), 8) * 0.6
    v, bad = nonlinear.phi_cubic(u0, t, a3, b3)
    assert not bad.any()
    ref = _fine_rk4(u0, t, lambda w: nonlinear.g_cgl(w, (0, 0, 0, a3, b3)))
    assert np.abs(v - ref).max() / np.abs(ref).max() < 1e-12
    r0 = np.abs(u0) ** 2
    assert np.allclose(np.abs(v) ** 2, r0 / (1.0 - 2.0 * a3 * r0 * t), rtol=1e-13, atol=0)


def test_exact_cubic_flow_limits_and_domain():
    u0 = _rand_c((20,), 9)
    v0, _ = nonlinear.phi_cubic(u0, 0.1, 0.0, 0.8)
    assert np.allclose(v0, np.exp(1j * 0.8 * np.abs(u0) ** 2 * 0.1) * u0, rtol=1e-14)
    v1, _ = nonlinear.phi_cubic(u0, 0.1, 1e-9, 0.8)
    assert np.abs(v1 - v0).max() < 1e-8
    # semigroup property of an exact flow
    a, _ = nonlinear.phi_cubic(u0, 0.07, -1.0, 0.3)
    b, _ = nonlinear.phi_cubic(a, 0.05, -1.0, 0.3)
    c, _ = nonlinear.phi_cubic(u0, 0.12, -1.0, 0.3)
    assert np.abs(b - c).max() < 1e-13
    # outside the domain 1 - 2 a3 |u|^2 t > 0 the mask is raised
    _, bad = nonlinear.phi_cubic(np.array([2.0 + 0j, 0.1 + 0j]), 0.5, 1.0, 0.0)
    assert bad.tolist() == [True, False]


def test_exact_quintic_flow_vs_fine_rk4():
    u0 = _rand_c((40,), 10) * 0.7
    a4, b4, t = -0.1, -0.5, 0.08
    v, bad = nonlinear.phi_quintic(u0, t, a4, b4)
    assert not bad.any()
    ref = _fine_rk4(u0, t, lambda w: nonlinear.g_cgl(w, (0, 0, 0, 0, 0, a4, b4)))
    assert np.abs(v - ref).max() / np.abs(ref).max() < 1e-12
    r0 = np.abs(u0) ** 4
    assert np.allclose(np.abs(v) ** 4, r0 / (1.0 - 4.0 * a4 * r0 * t), rtol=1e-12)


def test_rk4_flow_linear_stability_polynomial():
    """For g(u) = c u one RK4 step is R(c t) u with R(z) = sum_{k<=4} z^k/k!."""
    c = complex(-0.3, 1.7)
    t = 0.4
    u = _rand_c((9,), 11)
    z = c * t
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    assert np.abs(nonlinear.rk4_flow(u, t, lambda w: c * w) - R * u).max() < 1e-14


def test_rk4_flow_local_error_is_fifth_order():
    u0 = _rand_c((30,), 12) * 0.8
    gfun = lambda w: nonlinear.g_cgl(w, (0, 0, 0, -1.0, 0.5))
    errs = []
    for t in (0.08, 0.04, 0.02):
        exact, _ = nonlinear.phi_cubic(u0, t, -1.0, 0.5)
        errs.append(np.abs(nonlinear.rk4_flow(u0, t, gfun) - exact).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(4.6 < r < 5.4 for r in rates), rates


# ---------------------------------------------------------------- steppers

class _LinearG:
    """Test nonlinearity g(u) = c u with exact flow e^{c t} u."""

    def __init__(self, c):
        self.c = c

    def g(self, u):
        return self.c * u

    def flow(self, u, t):
        return np.exp(self.c * t) * u


def _tiny_problem(shape=(5, 4, 3), seed=40):
    As = [ops.operator_A(n, -2.0, 2.0, ops.DIRICHLET, (1.0, 0.8, -0.3), len(shape)) for n in shape]
    return As, _rand_c(shape, seed)


@pytest.mark.parametrize("method", ["strang", "lawson4"])
def test_steppers_with_g_zero_are_exact_linear_flow(method):
    As, U = _tiny_problem()
    tau = 0.05
    E = [scipy.linalg.expm(tau * A) for A in As]
    H = [scipy.linalg.expm(0.5 * tau * A) for A in As]
    step = steppers.make_step(method, E, H, tau, _LinearG(0.0))
    ref = scipy.linalg.expm(tau * tensor.kron_sum(As)) @ ci.flat(U)
    assert np.linalg.norm(ci.flat(step(U)) - ref) / np.linalg.norm(ref) < 1e-13


def test_lawson4_with_linear_g_is_expK_times_rk4_polynomial():
    """g(u) = c u commutes with K, so Lawson4 gives e^{tau K} R(tau c) u exactly."""
    As, U = _tiny_problem()
    tau, c = 0.07, complex(0.4, -1.1)
    E = [scipy.linalg.expm(tau * A) for A in As]
    H = [scipy.linalg.expm(0.5 * tau * A) for A in As]
    out = steppers.lawson4_step(U, E, H, tau, _LinearG(c))
    z = tau * c
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    ref = R * (scipy.linalg.expm(tau * tensor.kron_sum(As)) @ ci.flat(U))
    assert np.linalg.norm(ci.flat(out) - ref) / np.linalg.norm(ref) < 1e-13


def test_strang_with_linear_g_is_exact():
    As, U = _tiny_problem()
    tau, c = 0.07, complex(0.4, -1.1)
    E = [scipy.linalg.expm(tau * A) for A in As]
    out = steppers.strang_step(U, E, tau, _LinearG(c))
    ref = np.exp(tau * c) * (scipy.linalg.expm(tau * tensor.kron_sum(As)) @ ci.flat(U))
    assert np.linalg.norm(ci.flat(out) - ref) / np.linalg.norm(ref) < 1e-13


def test_lawson4_with_K_zero_is_classical_rk4_and_strang_is_exact_flow():
    """Lawson methods are RK methods for w = e^{-tK} u (Section 2.2): with
    K = 0 Lawson4 is classical RK4; Strang with E = I is phi_{tau/2} o phi_{tau/2} = phi_tau."""
    U = _rand_c((6, 5), 13) * 0.8
    I = [np.eye(6), np.eye(5)]
    nl = steppers.CGLNonlinearity(COEF2)
    tau = 0.03
    l4 = steppers.lawson4_step(U, I, I, tau, nl)
    # textbook RK4 written with a Butcher tableau, independent of rk4_flow
    A_t = [[0, 0, 0, 0], [0.5, 0, 0, 0], [0, 0.5, 0, 0], [0, 0, 1, 0]]
    b_t = [1 / 6, 1 / 3, 1 / 3, 1 / 6]
    ks = []
    for i in range(4):
        ks.append(nl.g(U + tau * sum(A_t[i][j] * ks[j] for j in range(i))))
    rk = U + tau * sum(b_t[i] * ks[i] for i in range(4))
    assert np.abs(l4 - rk).max() < 1e-14
    st = steppers.strang_step(U, I, tau, nl)
    ex, _ = nonlinear.phi_cubic(U, tau, COEF2[3], COEF2[4])
    assert np.abs(st - ex).max() < 1e-14


def test_lawson4_regrouped_schedule_equals_literal():
    """The 4-half-action schedule (P = H u, Q = H g(u), X, Y) is algebraically
    eq. (lawson4) because e^{tau K} = e^{tau K/2} e^{tau K/2}."""
    p = ci.scaled(ci.C0, (12, 10))
    tau = p.tau
    E = steppers.operators_for(p, tau)
    H = steppers.operators_for(p, 0.5 * tau)
    nl = steppers.CGLNonlinearity(p.coeffs.as_tuple())
    U = ci.initial_state(p)
    lit = steppers.lawson4_step(U, E, H, tau, nl)
    P = tensor.tucker(U, H)
    Q = tensor.tucker(nl.g(U), H)
    u2 = P + 0.5 * tau * Q
    g2 = nl.g(u2)
    u3 = P + 0.5 * tau * g2
    g3 = nl.g(u3)
    X = P + tau * g3
    Y = P + tau / 6 * Q + tau / 3 * (g2 + g3)
    reg = tensor.tucker(Y, H) + tau / 6 * nl.g(tensor.tucker(X, H))
    assert np.abs(lit - reg).max() / np.abs(lit).max() < 1e-13


def _c0_small(nn=24):
    return ci.scaled(ci.C0, (nn, nn))


def _run(p, method, m, T):
    tau = T / m
    E = steppers.operators_for(p, tau)
    H = steppers.operators_for(p, 0.5 * tau)
    nl = steppers.CGLNonlinearity(p.coeffs.as_tuple())
    u, bad = steppers.run(ci.initial_state(p), steppers.make_step(method, E, H, tau, nl), m)
    assert not bad
    return u


def test_empirical_orders_strang_2_lawson4_4():
    p = _c0_small()
    T = 0.5
    ref = _run(p, "lawson4", 640, T)
    for method, ms, lo, hi in (("strang", (10, 20, 40), 1.85, 2.15), ("lawson4", (10, 20, 40), 3.6, 4.5)):
        errs = [metrics.rel_linf(_run(p, method, m, T), ref) for m in ms]
        orders = [metrics.observed_order(ms[i], errs[i], ms[i + 1], errs[i + 1]) for i in range(2)]
        assert all(lo < o < hi for o in orders), (method, errs, orders)


def test_observed_order_reproduces_paper_tables():
    rows = []
    with open(os.path.join(GOLDEN, "paper_table_orders.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    assert len(rows) >= 16
    for _tab, _meth, m0, e0, m1, e1, printed in rows:
        p = metrics.observed_order(int(m0), float(e0), int(m1), float(e1))
        # the printed errors carry 4 significant digits and the order 3 decimals
        half_ulp = [0.5 * 10.0 ** (int(np.floor(np.log10(float(e)))) - 3) / float(e) for e in (e0, e1)]
        tol = sum(half_ulp) / np.log(int(m1) / int(m0)) + 5e-4 + 1e-9
        assert abs(p - float(printed)) < tol, (_tab, _meth, m1, p, printed, tol)


def test_rel_norms():
    b = np.array([3 + 4j, 0, 0])
    a = np.array([3 + 4j, 1, 0])
    assert metrics.rel_l2(a, b) == pytest.approx(0.2)
    assert metrics.rel_linf(a, b) == pytest.approx(0.2)


def test_cubic_exact_flow_blowup_is_counted():
    nl = steppers.CGLNonlinearity((1.0, 0.0, 0.0, 1.0, 0.0))
    nl.flow(np.array([10.0 + 0j]), 0.1)
    assert nl.blowups == 1
