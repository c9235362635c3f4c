"""Pointwise nonlinear terms and flows (oracle; test infrastructure only).

* g(u) = (a3 + i b3)|u|^2 u + (a4 + i b4)|u|^4 u: the nonlinear part of
  eq. (cqCGL) evaluated pointwise.
* Exact cubic flow of u' = (a3 + i b3)|u|^2 u (eq. exsolcub):
  phi^c_t(u0) = exp(-(a3 + i b3)/(2 a3) * log|1 - 2 a3 |u0|^2 t|) u0.
  Its domain is 1 - 2 a3 |u0|^2 t > 0; at or beyond it the flow has blown up
  (the absolute value in the paper's formula would silently continue it), so
  ``phi_cubic`` also returns a mask of points outside the domain.
* Exact quintic flow of u' = (a4 + i b4)|u|^4 u (Section 4.3):
  phi^q_t(u0) = exp(-(a4 + i b4)/(4 a4) * log|1 - 4 a4 |u0|^4 t|) u0.
* When no exact flow is used (cubic-quintic g), the sub-flow phi_t is one
  step of the classical RK4 scheme (eq. RK4) applied to u' = g(u), as in the
  cubic-quintic experiments of Sections 4.3 and 4.4.
"""
from __future__ import annotations

from typing import Callable, Tuple

import numpy as np


def g_cgl(u: np.ndarray, coeffs) -> np.ndarray:
    a3, b3 = coeffs[3], coeffs[4]
    a4, b4 = (coeffs[5], coeffs[6]) if len(coeffs) > 5 else (0.0, 0.0)
    r = (u.real * u.real + u.imag * u.imag)
    return complex(a3, b3) * r * u + complex(a4, b4) * (r * r) * u


def phi_cubic(u: np.ndarray, t: float, a3: float, b3: float) -> Tuple[np.ndarray, np.ndarray]:
    """Exact cubic flow and a boolean mask of points where 1 - 2 a3 |u|^2 t <= 0."""
    r = u.real * u.real + u.imag * u.imag
    s = 1.0 - 2.0 * a3 * r * t
    bad = s <= 0.0
    if a3 == 0.0:
        return np.exp(1j * b3 * r * t) * u, bad
    # log|s| written as log1p(-2 a3 r t) inside the domain (same value, no
    # cancellation for small a3 r t); the paper's absolute value outside it
    with np.errstate(invalid="ignore", divide="ignore"):
        L = np.where(bad, np.log(np.abs(s)), np.log1p(-2.0 * a3 * r * t))
    return np.exp(-complex(a3, b3) / (2.0 * a3) * L) * u, bad


def phi_quintic(u: np.ndarray, t: float, a4: float, b4: float) -> Tuple[np.ndarray, np.ndarray]:
    """Exact quintic flow and a boolean mask of points where 1 - 4 a4 |u|^4 t <= 0."""
    r = u.real * u.real + u.imag * u.imag
    s = 1.0 - 4.0 * a4 * r * r * t
    bad = s <= 0.0
    if a4 == 0.0:
        return np.exp(1j * b4 * r * r * t) * u, bad
    with np.errstate(invalid="ignore", divide="ignore"):
        L = np.where(bad, np.log(np.abs(s)), np.log1p(-4.0 * a4 * r * r * t))
    return np.exp(-complex(a4, b4) / (4.0 * a4) * L) * u, bad


def rk4_flow(u: np.ndarray, t: float, g: Callable[[np.ndarray], np.ndarray]) -> np.ndarray:
    """One classical RK4 step (eq. RK4 with K = 0) of w' = g(w) over time t."""
    k1 = g(u)
    k2 = g(u + 0.5 * t * k1)
    k3 = g(u + 0.5 * t * k2)
    k4 = g(u + t * k3)
    return u + (t / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
