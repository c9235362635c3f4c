"""Error measures and observed order (oracle; test infrastructure only).

* relative infinity-norm error against a reference solution: the accuracy
  measure of the paper's experiments (Section 4, introductory paragraphs);
* relative 2-norm error over all complex entries: the parity measure;
* observed order between consecutive runs with m_{k-1} and m_k steps:
  p = log(e_{k-1}/e_k) / log(m_k/m_{k-1}), the "order" column of Tables 1-5.
"""
from __future__ import annotations

import numpy as np


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / den) if den > 0 else float(np.linalg.norm(a.ravel()))


def rel_linf(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a)))


def observed_order(steps_prev: int, err_prev: float, steps: int, err: float) -> float:
    return float(np.log(err_prev / err) / np.log(steps / steps_prev))
