"""The coupled two-field cubic-quintic CGL system of Section 4.4, eq. (coupled)
(oracle; test infrastructure only).

Two fields u, v on one periodic 2-D grid:
    u_t =  a0 d_1 u + (a1 + i b1) Lap u + a2 u + (a3 + i b3)|u|^2 u + (a4 + i b4)|u|^4 u + a5 |v|^2 u
    v_t = -a0 d_1 v + (a1 + i b1) Lap v + a2 v + (a3 + i b3)|v|^2 v + (a4 + i b4)|v|^4 v + a5 |u|^2 v
K = diag(K^u, K^v) is block diagonal, so the exponential acts on each field
with its own Kronecker sum: direction 1 of u carries +a0 d_1, of v -a0 d_1.
The pseudospectral discretisation diagonalises both: the first derivative
multiplies mode k by i k, the second by -k^2.  Reading: for an even number
of nodes the first-derivative symbol of the Nyquist mode is 0 (the sampled
Nyquist mode is a cosine whose derivative vanishes at every node; this keeps
the operator real and the system's mirror symmetry exact).

The state is the stacked array W = [u, v] (shape (2, n1, n2)); the steppers
of ``steppers`` apply unchanged with ``CoupledAction`` as the exponential
action and ``CoupledNonlinearity`` as g and its sub-flow (one classical RK4
step of W' = g(W): no exact flow exists once the fields are coupled).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Sequence

import numpy as np

from . import fourier, nonlinear


@dataclass(frozen=True)
class CoupledCoeffs:
    a0: float
    a1: float
    b1: float
    a2: float
    a3: float
    b3: float
    a4: float
    b4: float
    a5: float


# Section 4.4's parameter set
PAPER = CoupledCoeffs(a0=-0.4, a1=0.125, b1=0.5, a2=-0.9, a3=1.0, b3=0.8, a4=-0.1, b4=-0.6, a5=0.5)


def first_derivative_wavenumbers(n: int, a: float, b: float) -> np.ndarray:
    """Wave numbers for the first-derivative symbol i k: those of the
    transform with the Nyquist mode (even n) set to 0."""
    k = fourier.wavenumbers(n, a, b)
    if n % 2 == 0:
        k[n // 2] = 0.0
    return k


def exp_factor(n: int, a: float, b: float, c: CoupledCoeffs, mu: int, sign: float,
               t: float) -> np.ndarray:
    """Diagonal of exp(t A_mu) for one field of the 2-D system: A_1 carries
    sign * a0 d_1 (sign +1 for u, -1 for v), both carry (a1 + i b1) d_mu^2 + a2/2."""
    k = fourier.wavenumbers(n, a, b)
    lam = complex(c.a1, c.b1) * -(k ** 2) + c.a2 / 2.0
    if mu == 0:
        lam = lam + sign * c.a0 * 1j * first_derivative_wavenumbers(n, a, b)
    return np.exp(t * lam)


class CoupledAction:
    """W -> [e^{t K^u} u, e^{t K^v} v], each by the Fourier route."""

    def __init__(self, n: Sequence[int], lo: Sequence[float], hi: Sequence[float],
                 c: CoupledCoeffs, t: float):
        self.fields = [fourier.FourierAction([exp_factor(n[mu], lo[mu], hi[mu], c, mu, s, t)
                                              for mu in range(2)]) for s in (1.0, -1.0)]

    def __call__(self, W: np.ndarray) -> np.ndarray:
        return np.stack([self.fields[0](W[0]), self.fields[1](W[1])])


class CoupledNonlinearity:
    """g(W) of eq. (coupled) and its sub-flow (RK4)."""

    def __init__(self, c: CoupledCoeffs):
        self.c = c
        self.exact = False
        self.blowups = 0

    def g(self, W: np.ndarray) -> np.ndarray:
        c = self.c
        u, v = W[0], W[1]
        ru = u.real * u.real + u.imag * u.imag
        rv = v.real * v.real + v.imag * v.imag
        gu = complex(c.a3, c.b3) * ru * u + complex(c.a4, c.b4) * ru * ru * u + c.a5 * rv * u
        gv = complex(c.a3, c.b3) * rv * v + complex(c.a4, c.b4) * rv * rv * v + c.a5 * ru * v
        return np.stack([gu, gv])

    def flow(self, W: np.ndarray, t: float) -> np.ndarray:
        return nonlinear.rk4_flow(W, t, self.g)


def mirror(u: np.ndarray) -> np.ndarray:
    """u(L - x_1, x_2) on the periodic grid x_1 = a + j h: node j -> node -j mod n1
    (with a = 0, the paper's domain)."""
    return np.roll(u[::-1], 1, axis=0)


def soliton_datum(n1: int, lo: float, hi: float, c: CoupledCoeffs, m: int = 10000,
                  T: float = 25.0, delta: float = 2.25, chi: float = 17.5,
                  sigma: float = 2.5) -> np.ndarray:
    """Section 4.4's stationary soliton: the 1-D cubic-quintic CGL equation
    (eq. cqgl1d: the coupled system's coefficients without a0 and a5) from
    the Gaussian delta exp(-(x - chi)^2 / (2 sigma^2)), periodic on (lo, hi)
    with n1 Fourier modes, stepped by if4 (Lawson4) with m steps to T."""
    from . import steppers
    x = fourier.nodes(n1, lo, hi)
    w = (delta * np.exp(-(x - chi) ** 2 / (2.0 * sigma ** 2))).astype(np.complex128)
    tau = T / m
    cq = (c.a1, c.b1, c.a2, c.a3, c.b3, c.a4, c.b4)

    def act(t):
        return fourier.FourierAction([fourier.exp_factor(n1, lo, hi, cq, 1, t)])

    nl = steppers.CGLNonlinearity(cq)
    w, bad = steppers.run(w, steppers.make_step("lawson4", act(tau), act(0.5 * tau), tau, nl), m)
    if bad:
        raise FloatingPointError("the 1-D soliton run became non-finite")
    return w


def initial_state(w: np.ndarray, n2: int) -> np.ndarray:
    """u0(x1, x2) = w(x1), v0(x1, x2) = w(L - x1) (Section 4.4), as W (2, n1, n2)."""
    u0 = np.repeat(w[:, None], n2, axis=1)
    return np.stack([u0, mirror(u0)])
