"""Periodic boundaries: the pseudospectral Fourier discretisation of Section 3.2
(oracle; test infrastructure only).

On (a, b) with period L = b - a and n equispaced nodes x_j = a + j L / n,
j = 0..n-1, the Fourier basis functions are eigenfunctions of the second
derivative, so each A_mu is diagonal in coefficient space:
    A_mu = diag((a1 + i b1)(-k^2) + a2/d)  over the wave numbers k of the grid,
and the action of exp(t K) is the pointwise product of the coefficient tensor
with E = exp(t ((a1 + i b1)(-sum_mu k_mu^2) + a2)) between a forward and an
inverse d-dimensional discrete Fourier transform.  The wave numbers are those
of the discrete transform of an n-point grid, 2 pi / L times
0, 1, ..., n/2, -n/2 + 1, ..., -1 (Section 3.2 prints them as 0 .. n-1 on
(0, 2 pi); the symmetric set is the reading under which K is the periodic
spectral Laplacian).  The nonlinear term is evaluated pointwise on grid
values, g applied between an inverse and a forward transform as in the
paper; the steppers here keep the state as grid values, which is the same
method with the transforms moved to the exponential actions.

``numpy.fft`` is the transform (a library primitive).  ``FourierAction``
objects are callables that the steppers accept in place of the lists of
exponential matrices.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def wavenumbers(n: int, a: float, b: float) -> np.ndarray:
    """Wave numbers of an n-point periodic grid on (a, b), in the order of the
    discrete transform's coefficients."""
    L = b - a
    return 2.0 * np.pi * np.fft.fftfreq(n, d=1.0 / n) / L


def nodes(n: int, a: float, b: float) -> np.ndarray:
    return a + (b - a) * np.arange(n, dtype=np.float64) / n


def exp_factor(n: int, a: float, b: float, coeffs, d: int, t: float) -> np.ndarray:
    """Diagonal of exp(t A_mu) for one direction of a d-dimensional problem."""
    a1, b1, a2 = coeffs[0], coeffs[1], coeffs[2]
    return np.exp(t * (complex(a1, b1) * -(wavenumbers(n, a, b) ** 2) + a2 / d))


def exp_factors(ns: Sequence[int], a: float, b: float, coeffs, t: float):
    """Per-direction diagonals of exp(t A_mu): the E tensor of Section 3.2 is
    their outer product (K is a Kronecker sum of the diagonal A_mu)."""
    return [exp_factor(n, a, b, coeffs, len(ns), t) for n in ns]


class FourierAction:
    """u -> F^{-1}(E * F(u)) with E the outer product of the factors."""

    def __init__(self, factors):
        self.factors = [np.asarray(f, dtype=np.complex128) for f in factors]
        E = self.factors[0]
        for f in self.factors[1:]:
            E = np.multiply.outer(E, f)
        self.E = E

    def __call__(self, u: np.ndarray) -> np.ndarray:
        return np.fft.ifftn(self.E * np.fft.fftn(u))


def actions_for(problem, t: float) -> FourierAction:
    return FourierAction(exp_factors(problem.n, problem.a, problem.b, problem.coeffs.as_tuple(), t))


def circulant_exponential(n: int, a: float, b: float, coeffs, d: int, t: float) -> np.ndarray:
    """The same one-direction exponential as a dense n x n matrix acting on
    grid values, F^{-1} diag(e) F, assembled column by column (it is the
    exponential of the periodic spectral second-derivative matrix)."""
    e = exp_factor(n, a, b, coeffs, d, t)
    eye = np.eye(n)
    return np.stack([np.fft.ifft(e * np.fft.fft(eye[:, j])) for j in range(n)], axis=1)


def spectral_second_derivative(n: int, a: float, b: float) -> np.ndarray:
    """The periodic Fourier second-derivative matrix on an even n-point grid,
    from its closed form (entries depend on j - k only):
      diagonal  -pi^2/(3 h^2) - 1/6,   off-diagonal  -(-1)^(j-k) / (2 sin^2((j-k) h/2)),
    for the period 2 pi with h = 2 pi / n, scaled by (2 pi / L)^2."""
    if n % 2:
        raise ValueError("even n only")
    h = 2.0 * np.pi / n
    j = np.arange(n)
    diff = j[:, None] - j[None, :]
    with np.errstate(divide="ignore"):
        D = -((-1.0) ** diff) / (2.0 * np.sin(diff * h / 2.0) ** 2)
    D[diff == 0] = -np.pi ** 2 / (3.0 * h * h) - 1.0 / 6.0
    return D * (2.0 * np.pi / (b - a)) ** 2
