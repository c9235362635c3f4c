"""Strang, split4, Lawson2 and Lawson4 steps and the three-term splittings,
written exactly as in the paper (oracle; test infrastructure only).

* Strang (eq. Strang): u_{n+1} = phi_{tau/2}( e^{tau K} phi_{tau/2}(u_n) ).
  Both half flows are evaluated; consecutive half flows of two steps are not
  merged.
* Lawson4 (eq. lawson4), six exponential actions per step:
      u2 = e^{tau K/2}(u + tau/2 g(u))
      u3 = e^{tau K/2} u + tau/2 g(u2)
      u4 = e^{tau K} u + tau e^{tau K/2} g(u3)
      u_{n+1} = e^{tau K}(u + tau/6 g(u)) + tau/3 e^{tau K/2}(g(u2) + g(u3)) + tau/6 g(u4)
  where e^{tau K} and e^{tau K/2} act through the Tucker operator (eq. Tucker)
  with the matrices E_mu = exp(tau A_mu) and H_mu = exp(tau A_mu / 2).

* split4 (eq. Richardson, the explicit form of eq. richextrap):
      u_n2 = phi_{tau/2}(e^{tau K} phi_{tau/2}(u_n))
      u_{n+1} = 4/3 phi_{tau/4}(e^{tau K/2} phi_{tau/2}(e^{tau K/2} phi_{tau/4}(u_n))) - 1/3 u_n2
  (the middle sub-flow is one evaluation of phi over tau/2, as printed).
* Lawson2b (eq. lawson2b):
      u_n2 = e^{tau K}(u_n + tau g(u_n))
      u_{n+1} = e^{tau K}(u_n + tau/2 g(u_n)) + tau/2 g(u_n2)
* strang_3t (Section 4.3): S3_tau(u) = phi^q_{tau/2}(phi^c_{tau/2}(e^{tau K}
  phi^c_{tau/2}(phi^q_{tau/2}(u)))) with the exact cubic and quintic flows;
  split4_3t = 4/3 S3_{tau/2}(S3_{tau/2}(u)) - 1/3 S3_tau(u), composed as
  written (S3_{tau/2} uses e^{tau K/2}).

The nonlinear part is an object with ``g(u)`` and ``flow(u, t)`` (and, for
the three-term schemes, ``phi_c`` / ``phi_q``) so that the same steppers run
the CGL nonlinearity and the closed-form test problems.
"""
from __future__ import annotations

from typing import Callable, List, Sequence

import numpy as np

from . import nonlinear
from .tensor import tucker as _tucker


def tucker(u: np.ndarray, M) -> np.ndarray:
    """The exponential action: the Tucker operator of eq. (Tucker) for a list
    of matrices, or a callable action (the Fourier path of Section 3.2)."""
    return M(u) if callable(M) else _tucker(u, M)


class CGLNonlinearity:
    """g of eq. (cqCGL) and its sub-flow phi_t.

    Cubic case (a4 = b4 = 0): phi_t is the exact flow of eq. (exsolcub).
    Cubic-quintic case: phi_t is one RK4 step of u' = g(u) (Sections 4.3/4.4).
    ``force_rk4`` selects the RK4 sub-flow also for the cubic case.
    Points that leave the exact flow's domain are counted in ``blowups``.
    """

    def __init__(self, coeffs, force_rk4: bool = False):
        c = tuple(float(v) for v in coeffs)
        self.coeffs = c + (0.0,) * (7 - len(c))
        self.cubic = self.coeffs[5] == 0.0 and self.coeffs[6] == 0.0
        self.exact = self.cubic and not force_rk4
        self.blowups = 0

    def g(self, u: np.ndarray) -> np.ndarray:
        return nonlinear.g_cgl(u, self.coeffs)

    def flow(self, u: np.ndarray, t: float) -> np.ndarray:
        if self.exact:
            return self.phi_c(u, t)
        return nonlinear.rk4_flow(u, t, self.g)

    def phi_c(self, u: np.ndarray, t: float) -> np.ndarray:
        """Exact flow of the cubic part (eq. exsolcub)."""
        v, bad = nonlinear.phi_cubic(u, t, self.coeffs[3], self.coeffs[4])
        self.blowups += int(np.count_nonzero(bad))
        return v

    def phi_q(self, u: np.ndarray, t: float) -> np.ndarray:
        """Exact flow of the quintic part (Section 4.3)."""
        v, bad = nonlinear.phi_quintic(u, t, self.coeffs[5], self.coeffs[6])
        self.blowups += int(np.count_nonzero(bad))
        return v


def strang_step(u: np.ndarray, E: Sequence[np.ndarray], tau: float, nl) -> np.ndarray:
    v = nl.flow(u, 0.5 * tau)
    w = tucker(v, E)
    return nl.flow(w, 0.5 * tau)


def lawson4_step(u: np.ndarray, E: Sequence[np.ndarray], H: Sequence[np.ndarray],
                 tau: float, nl) -> np.ndarray:
    g1 = nl.g(u)
    u2 = tucker(u + 0.5 * tau * g1, H)
    g2 = nl.g(u2)
    u3 = tucker(u, H) + 0.5 * tau * g2
    g3 = nl.g(u3)
    u4 = tucker(u, E) + tau * tucker(g3, H)
    g4 = nl.g(u4)
    return (tucker(u + (tau / 6.0) * g1, E) + (tau / 3.0) * tucker(g2 + g3, H)
            + (tau / 6.0) * g4)


def split4_step(u: np.ndarray, E: Sequence[np.ndarray], H: Sequence[np.ndarray],
                tau: float, nl) -> np.ndarray:
    un2 = nl.flow(tucker(nl.flow(u, 0.5 * tau), E), 0.5 * tau)
    v = nl.flow(u, 0.25 * tau)
    v = tucker(v, H)
    v = nl.flow(v, 0.5 * tau)
    v = tucker(v, H)
    v = nl.flow(v, 0.25 * tau)
    return (4.0 / 3.0) * v - (1.0 / 3.0) * un2


def lawson2_step(u: np.ndarray, E: Sequence[np.ndarray], tau: float, nl) -> np.ndarray:
    g1 = nl.g(u)
    un2 = tucker(u + tau * g1, E)
    return tucker(u + 0.5 * tau * g1, E) + 0.5 * tau * nl.g(un2)


def strang_3t_step(u: np.ndarray, E: Sequence[np.ndarray], tau: float, nl) -> np.ndarray:
    t = 0.5 * tau
    v = nl.phi_c(nl.phi_q(u, t), t)
    w = tucker(v, E)
    return nl.phi_q(nl.phi_c(w, t), t)


def split4_3t_step(u: np.ndarray, E: Sequence[np.ndarray], H: Sequence[np.ndarray],
                   tau: float, nl) -> np.ndarray:
    full = strang_3t_step(u, E, tau, nl)
    half = strang_3t_step(strang_3t_step(u, H, 0.5 * tau, nl), H, 0.5 * tau, nl)
    return (4.0 / 3.0) * half - (1.0 / 3.0) * full


def rk4_step_nonlinear(u: np.ndarray, tau: float, nl) -> np.ndarray:
    """Classical RK4 (eq. RK4) for u' = g(u), i.e. with K = 0."""
    return nonlinear.rk4_flow(u, tau, nl.g)


def make_step(method: str, E, H, tau: float, nl) -> Callable[[np.ndarray], np.ndarray]:
    if method == "strang":
        return lambda u: strang_step(u, E, tau, nl)
    if method == "lawson4":
        return lambda u: lawson4_step(u, E, H, tau, nl)
    if method == "split4":
        return lambda u: split4_step(u, E, H, tau, nl)
    if method == "lawson2":
        return lambda u: lawson2_step(u, E, tau, nl)
    if method == "strang_3t":
        return lambda u: strang_3t_step(u, E, tau, nl)
    if method == "split4_3t":
        return lambda u: split4_3t_step(u, E, H, tau, nl)
    raise ValueError(method)


def run(u0: np.ndarray, step: Callable[[np.ndarray], np.ndarray], m: int,
        stop_on_nonfinite: bool = True):
    """Apply ``step`` m times.  Returns (u_m, nonfinite_flag)."""
    u = np.array(u0, dtype=np.complex128, copy=True)
    for _ in range(m):
        u = step(u)
        if stop_on_nonfinite and not np.all(np.isfinite(u)):
            return u, True
    return u, not np.all(np.isfinite(u))


def operators_for(problem, t: float, route: str = "closed") -> List[np.ndarray]:
    """exp(t A_mu) for every direction of a workload (closed form or scipy).
    Workloads with fourth-order or mixed-boundary operators have no closed
    form here and always take the scipy route."""
    from . import operators as ops
    order = getattr(problem, "order", 2)
    bc_hi = getattr(problem, "bc_hi", None)
    if order != 2 or (bc_hi is not None and bc_hi != problem.bc):
        hi = problem.bc if bc_hi is None else bc_hi
        return [ops.exp_scipy(ops.operator_A_fd(n, problem.a, problem.b, problem.bc, hi, order,
                                                problem.coeffs.as_tuple(), problem.d), t)
                for n in problem.n]
    out = []
    for n in problem.n:
        if route == "closed":
            out.append(ops.exp_closed_form(n, problem.a, problem.b, problem.bc,
                                           problem.coeffs.as_tuple(), problem.d, t))
        else:
            A = ops.operator_A(n, problem.a, problem.b, problem.bc,
                               problem.coeffs.as_tuple(), problem.d)
            out.append(ops.exp_scipy(A, t))
    return out
