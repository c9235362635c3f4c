"""1-D operators A_mu and their exponentials (oracle; test infrastructure only).

The semi-discretised system is u' = K u + g(u) with K the Kronecker sum of
A_mu ~ (a1 + i b1) d^2/dx_mu^2 + a2/d (eq. ODEs and the display after it).
The workloads use 2nd-order central differences:

* Dirichlet, interior nodes, h = (b-a)/(n+1):  D2 = tridiag(1, -2, 1) / h^2.
* Neumann, vertex grid, h = (b-a)/(n-1): interior rows (1, -2, 1)/h^2; the
  boundary rows use the ghost value of the centred u' = 0 condition, which
  gives (-2, 2)/h^2 in the first row and (2, -2)/h^2 in the last row.

The exponentials exp(t A_mu) are needed once per run (Section 3.1: computed
once and for all when the step size is constant).  Two independent routes:

* ``exp_closed_form``: the textbook eigen-decomposition of the 2nd-order
  Laplacian (sine basis for Dirichlet, cosine basis for Neumann).
* ``exp_scipy``: ``scipy.linalg.expm`` (Pade with scaling and squaring, the
  method the paper cites for its small exponentials).

General boundaries and the paper's fourth-order matrices (``laplacian_fd``):
each end of a direction is Dirichlet or Neumann on its own.

* Grid: a Dirichlet end is not a node (its value is 0), a Neumann end is the
  first or last node.  n unknowns: DD interior nodes h = (b-a)/(n+1); DN the
  semi-internal grid of Section 4.2, x_j = a + j h, j = 1..n, h = (b-a)/n
  (x_n = b); ND its mirror; NN the vertex grid h = (b-a)/(n-1).
* 2nd order: rows (1, -2, 1)/h^2; a Neumann end row is (-2, 2)/h^2 from the
  centred ghost value.
* 4th order (Sections 4.1.1 and 4.2, displayed matrices, times 1/(12 h^2)):
  interior rows (-1, 16, -30, 16, -1) with the Dirichlet boundary value 0
  dropped; next to a Dirichlet end the one-sided row (-15, -4, 14, -6, 1);
  at a Neumann end the last two rows (1, -6, 14, -4, -15, 10) and
  (1, -8/3, -6, 56, -145/3) (mirrored at the left end).  The paper prints
  DD and DN; ND and NN are the same rows mirrored.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

DIRICHLET = 0
NEUMANN = 1


def spacing(n: int, a: float, b: float, bc: int) -> float:
    if bc == DIRICHLET:
        return (b - a) / (n + 1)
    if bc == NEUMANN:
        return (b - a) / (n - 1)
    raise ValueError("bc")


def laplacian_2nd(n: int, a: float, b: float, bc: int) -> np.ndarray:
    """Dense n x n 2nd-order finite-difference second derivative (real)."""
    h = spacing(n, a, b, bc)
    D = np.zeros((n, n))
    for j in range(n):
        D[j, j] = -2.0
        if j > 0:
            D[j, j - 1] = 1.0
        if j < n - 1:
            D[j, j + 1] = 1.0
    if bc == NEUMANN:
        # ghost node u_{-1} = u_{1} (and u_{n} = u_{n-2}) from the centred u' = 0
        D[0, 1] = 2.0
        D[n - 1, n - 2] = 2.0
    return D / (h * h)


def operator_A(n: int, a: float, b: float, bc: int, coeffs, d: int) -> np.ndarray:
    """A_mu = (a1 + i b1) D2 + (a2/d) I, complex128 (display after eq. ODEs)."""
    a1, b1, a2 = coeffs[0], coeffs[1], coeffs[2]
    D = laplacian_2nd(n, a, b, bc)
    return (complex(a1, b1) * D + (a2 / d) * np.eye(n)).astype(np.complex128)


def eigen_2nd(n: int, a: float, b: float, bc: int):
    """Eigenvalues and eigenvector matrix of ``laplacian_2nd``.

    Dirichlet: V_jk = sqrt(2/(n+1)) sin(pi j k/(n+1)), j,k = 1..n (orthogonal,
    symmetric), lambda_k = -(4/h^2) sin^2(pi k / (2(n+1))).
    Neumann (vertex grid): C_jk = cos(pi j k/(n-1)), j,k = 0..n-1,
    lambda_k = -(4/h^2) sin^2(pi k / (2(n-1))).
    """
    h = spacing(n, a, b, bc)
    # sin / cos are 2 pi periodic: reduce the integer j*k modulo the period
    # before scaling, so large arguments lose no accuracy
    if bc == DIRICHLET:
        j = np.arange(1, n + 1)
        jk = np.outer(j, j) % (2 * (n + 1))
        V = np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * jk / (n + 1))
        lam = -(4.0 / (h * h)) * np.sin(np.pi * j / (2.0 * (n + 1))) ** 2
        return lam, V
    j = np.arange(0, n)
    jk = np.outer(j, j) % (2 * (n - 1))
    C = np.cos(np.pi * jk / (n - 1))
    lam = -(4.0 / (h * h)) * np.sin(np.pi * j / (2.0 * (n - 1))) ** 2
    return lam, C


def exp_closed_form(n: int, a: float, b: float, bc: int, coeffs, d: int, t: float) -> np.ndarray:
    """exp(t A_mu) from the eigen-decomposition: V diag(exp(t((a1+ib1) lam + a2/d))) V^{-1}."""
    a1, b1, a2 = coeffs[0], coeffs[1], coeffs[2]
    lam, V = eigen_2nd(n, a, b, bc)
    w = np.exp(t * (complex(a1, b1) * lam + a2 / d))
    if bc == DIRICHLET:
        return (V * w) @ V.T
    # inverse of the cosine basis: C^{-1} = (2/(n-1)) W C W, W = diag(1/2, 1, ..., 1, 1/2)
    # (discrete orthogonality of cos(pi j k/(n-1)) with trapezoid weights)
    W = np.ones(n)
    W[0] = W[-1] = 0.5
    Cinv = (2.0 / (n - 1)) * (W[:, None] * V * W[None, :])
    return (V * w) @ Cinv


def exp_scipy(A: np.ndarray, t: float) -> np.ndarray:
    """exp(t A) by scipy.linalg.expm (any dense A)."""
    return scipy.linalg.expm(t * np.asarray(A, dtype=np.complex128))


def spacing_mixed(n: int, a: float, b: float, bc_lo: int, bc_hi: int) -> float:
    """Grid step for n unknowns with the given end conditions (see module docstring)."""
    nodes_at_ends = (bc_lo == NEUMANN) + (bc_hi == NEUMANN)
    if bc_lo not in (DIRICHLET, NEUMANN) or bc_hi not in (DIRICHLET, NEUMANN):
        raise ValueError("bc")
    return (b - a) / (n + 1 - nodes_at_ends)


def laplacian_fd(n: int, a: float, b: float, bc_lo: int, bc_hi: int, order: int) -> np.ndarray:
    """Dense n x n finite-difference second derivative (real) of order 2 or 4
    with a Dirichlet or Neumann condition at each end."""
    h = spacing_mixed(n, a, b, bc_lo, bc_hi)
    D = np.zeros((n, n))
    if order == 2:
        for j in range(n):
            D[j, j] = -2.0
            if j > 0:
                D[j, j - 1] = 1.0
            if j < n - 1:
                D[j, j + 1] = 1.0
        if bc_lo == NEUMANN:
            D[0, 1] = 2.0
        if bc_hi == NEUMANN:
            D[n - 1, n - 2] = 2.0
        return D / (h * h)
    if order != 4:
        raise ValueError("order must be 2 or 4")
    if n < 6:
        raise ValueError("the 4th-order rows need n >= 6")
    centred = (-1.0, 16.0, -30.0, 16.0, -1.0)
    for j in range(n):
        for k, c in zip(range(j - 2, j + 3), centred):
            if 0 <= k < n:  # columns outside are Dirichlet zeros (or replaced below)
                D[j, k] = c
    dir_row = (-15.0, -4.0, 14.0, -6.0, 1.0)          # next to a Dirichlet end
    neu_rows = ((1.0, -6.0, 14.0, -4.0, -15.0, 10.0),  # the node before a Neumann end node
                (1.0, -8.0 / 3.0, -6.0, 56.0, -145.0 / 3.0))  # the Neumann end node
    if bc_hi == DIRICHLET:
        D[n - 1, :] = 0.0
        D[n - 1, n - 5:] = dir_row[::-1]
    else:
        D[n - 2, :] = 0.0
        D[n - 2, n - 6:] = neu_rows[0]
        D[n - 1, :] = 0.0
        D[n - 1, n - 5:] = neu_rows[1]
    if bc_lo == DIRICHLET:
        D[0, :] = 0.0
        D[0, :5] = dir_row
    else:
        D[1, :] = 0.0
        D[1, :6] = neu_rows[0][::-1]
        D[0, :] = 0.0
        D[0, :5] = neu_rows[1][::-1]
    return D / (12.0 * h * h)


def operator_A_fd(n: int, a: float, b: float, bc_lo: int, bc_hi: int, order: int, coeffs,
                  d: int) -> np.ndarray:
    """A_mu = (a1 + i b1) D2 + (a2/d) I with ``laplacian_fd``."""
    a1, b1, a2 = coeffs[0], coeffs[1], coeffs[2]
    D = laplacian_fd(n, a, b, bc_lo, bc_hi, order)
    return (complex(a1, b1) * D + (a2 / d) * np.eye(n)).astype(np.complex128)
