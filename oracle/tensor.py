"""mu-mode product and Tucker operator (oracle; test infrastructure only).

A tensor U in C^{n1 x ... x nd} is a NumPy array of shape (n1, ..., nd); its
``vec`` stacks columns, so index 1 runs fastest (Section 3.1).

* mu-mode product (Section 3.1): (U x_mu M)[.., i_mu, ..] = sum_j M[i_mu, j] U[.., j, ..],
  i.e. M multiplies every mu-fibre of U.
* Tucker operator (eq. Tucker): exp(tau K) vec(U) = vec(U x_1 e^{tau A_1} x_2 ... x_d e^{tau A_d}).
* K u (eq. kronsumv): vec(sum_mu U x_mu A_mu).
* K itself (eq. ODEs): K = sum_mu I_d (x) ... (x) I_{mu+1} (x) A_mu (x) I_{mu-1} (x) ... (x) I_1,
  only for brute-force checks on tiny grids.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def mode_product(U: np.ndarray, M: np.ndarray, mu: int) -> np.ndarray:
    """U x_mu M with mu zero-based (mu = 0 is the paper's index 1)."""
    Y = np.tensordot(M, U, axes=([1], [mu]))
    return np.moveaxis(Y, 0, mu)


def tucker(U: np.ndarray, Ms: Sequence[np.ndarray]) -> np.ndarray:
    """U x_1 M_1 x_2 ... x_d M_d, modes applied in the order 1..d."""
    Y = U
    for mu, M in enumerate(Ms):
        Y = mode_product(Y, M, mu)
    return Y


def kronsumv(U: np.ndarray, As: Sequence[np.ndarray]) -> np.ndarray:
    """K u computed as sum_mu U x_mu A_mu (eq. kronsumv), returned as a tensor."""
    out = np.zeros(U.shape, dtype=np.result_type(U, *As))
    for mu, A in enumerate(As):
        out = out + mode_product(U, A, mu)
    return out


def kron_sum(As: Sequence[np.ndarray]) -> np.ndarray:
    """Assemble K = A_d (+) ... (+) A_1 (eq. ODEs) as a dense N x N matrix."""
    ns = [A.shape[0] for A in As]
    N = int(np.prod(ns))
    K = np.zeros((N, N), dtype=np.complex128)
    d = len(As)
    for mu in range(d):
        # factor list from index d down to index 1: I_d (x) ... (x) A_mu (x) ... (x) I_1
        term = np.ones((1, 1), dtype=np.complex128)
        for nu in range(d - 1, -1, -1):
            F = As[nu] if nu == mu else np.eye(ns[nu])
            term = np.kron(term, F)
        K += term
    return K
