"""Thin Python binding of the CGL stepper (same names as the C ABI).

PyTorch provides device memory and the stream; the library does all of the
work.  State tensors are 1-D complex torch tensors of N = prod(n) elements
holding the column-stacked (index 1 fastest) grid function; ``to_device`` /
``to_host`` convert from / to NumPy arrays of shape n.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _lib as L
from ._lib import CGLError, check

PRECISIONS = {"fp64": L.FP64, "split": L.SPLIT_BF16}
METHODS = {"strang": L.STRANG, "lawson4": L.LAWSON4, "split4": L.SPLIT4, "lawson2": L.LAWSON2}


def _coeffs(c) -> L.Coeffs:
    v = tuple(float(x) for x in (c.as_tuple() if hasattr(c, "as_tuple") else c))
    v = v + (0.0,) * (7 - len(v))
    return L.Coeffs(*v)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def fd_operator(n: int, a: float, b: float, bc: int, coeffs, d: int) -> np.ndarray:
    """cgl_fd_operator: 2nd-order FD A_mu as a complex128 (n, n) array."""
    out = np.zeros((n, n), dtype=np.complex128, order="F")
    c = _coeffs(coeffs)
    check(L.lib().cgl_fd_operator(n, a, b, bc, C.byref(c), d, _dptr(out)), "cgl_fd_operator")
    return out


def fd_operator_ex(n: int, a: float, b: float, bc_lo: int, bc_hi: int, order: int, coeffs,
                   d: int) -> np.ndarray:
    """cgl_fd_operator_ex: FD A_mu of order 2 or 4 with a condition at each end."""
    out = np.zeros((n, n), dtype=np.complex128, order="F")
    c = _coeffs(coeffs)
    check(L.lib().cgl_fd_operator_ex(n, a, b, bc_lo, bc_hi, order, C.byref(c), d, _dptr(out)),
          "cgl_fd_operator_ex")
    return out


def problem_operators(p) -> list:
    """The operators A_mu of a workload description (grid n, domain (a, b),
    boundary types bc / bc_hi, FD order, coefficients)."""
    hi = p.bc if getattr(p, "bc_hi", None) is None else p.bc_hi
    order = getattr(p, "order", 2)
    return [fd_operator_ex(nm, p.a, p.b, p.bc, hi, order, p.coeffs, len(p.n)) for nm in p.n]


def expm(A: np.ndarray, t: float) -> np.ndarray:
    """cgl_expm: the library's Pade exponential of a host matrix."""
    A = np.asfortranarray(A, dtype=np.complex128)
    out = np.zeros_like(A, order="F")
    check(L.lib().cgl_expm(A.shape[0], _dptr(A), float(t), _dptr(out)), "cgl_expm")
    return out


def _torch():
    import torch
    return torch


def current_stream_handle() -> int:
    torch = _torch()
    return torch.cuda.current_stream().cuda_stream


class Plan:
    """cgl_plan + the calls that take it."""

    def __init__(self, n: Sequence[int], coeffs, tau: float, precision: str = "fp64",
                 master: bool = False, rk4_flow: bool = False, stream: Optional[int] = None,
                 three_term: bool = False):
        self.n = tuple(int(v) for v in n)
        self.d = len(self.n)
        self.N = int(np.prod(self.n))
        self.tau = float(tau)
        self.precision = precision
        self.master = bool(master)
        flags = ((L.FLAG_FP64_MASTER if master else 0) | (L.FLAG_RK4_FLOW if rk4_flow else 0)
                 | (L.FLAG_THREE_TERM if three_term else 0))
        if stream is None:
            stream = current_stream_handle()
        self._stream = stream
        arr = (C.c_int64 * self.d)(*self.n)
        c = _coeffs(coeffs)
        h = C.c_void_p()
        check(L.lib().cgl_plan(C.byref(h), self.d, arr, C.byref(c), self.tau,
                               PRECISIONS[precision], flags, C.c_void_p(stream)), "cgl_plan")
        self._h = h

    # -- element types -------------------------------------------------------
    @property
    def state_dtype(self):
        torch = _torch()
        return torch.complex128 if (self.precision == "fp64" or self.master) else torch.complex64

    @property
    def stage_dtype(self):
        torch = _torch()
        return torch.complex128 if self.precision == "fp64" else torch.complex64

    def to_device(self, u: np.ndarray, dtype=None):
        torch = _torch()
        flat = np.ascontiguousarray(np.asarray(u).reshape(-1, order="F"))
        return torch.from_numpy(flat.astype(np.complex128)).to(
            device="cuda", dtype=dtype or self.state_dtype)

    def to_host(self, t) -> np.ndarray:
        return t.detach().to("cpu").numpy().astype(np.complex128).reshape(self.n, order="F")

    # -- setup ---------------------------------------------------------------
    def set_operators(self, mu: int, A: np.ndarray) -> None:
        A = np.asfortranarray(A, dtype=np.complex128)
        check(L.lib().cgl_set_operators(self._h, mu, _dptr(A)), "cgl_set_operators")

    def set_exponentials(self, mu: int, E: np.ndarray, H: np.ndarray) -> None:
        E = np.asfortranarray(E, dtype=np.complex128)
        H = np.asfortranarray(H, dtype=np.complex128)
        check(L.lib().cgl_set_exponentials(self._h, mu, _dptr(E), _dptr(H)), "cgl_set_exponentials")

    def set_fd_operators(self, a: float, b: float, bc: int, coeffs) -> None:
        self.set_operators_all([fd_operator(nm, a, b, bc, coeffs, self.d) for nm in self.n])

    def set_problem_operators(self, p) -> None:
        """The operators of a workload description: FD (order and both ends)
        or, for periodic boundaries, the Fourier discretisation."""
        if p.bc == L.PERIODIC:
            for mu in range(self.d):
                self.set_periodic(mu, p.a, p.b)
            return
        self.set_operators_all(problem_operators(p))

    def set_periodic(self, mu: int, a: float, b: float) -> None:
        """cgl_set_periodic: direction mu periodic on (a, b), Fourier route."""
        check(L.lib().cgl_set_periodic(self._h, mu, float(a), float(b)), "cgl_set_periodic")

    def get_periodic_factor(self, mu: int, which: int) -> np.ndarray:
        out = np.zeros(self.n[mu], dtype=np.complex128)
        check(L.lib().cgl_get_periodic_factor(self._h, mu, which, _dptr(out)),
              "cgl_get_periodic_factor")
        return out

    def set_operators_all(self, As) -> None:
        """cgl_set_operators_all: every operator at once (parallel exponentials)."""
        mats = [np.asfortranarray(A, dtype=np.complex128) for A in As]
        arr = (C.POINTER(C.c_double) * len(mats))(*[_dptr(m) for m in mats])
        check(L.lib().cgl_set_operators_all(self._h, arr), "cgl_set_operators_all")

    def get_operator(self, mu: int, which: int) -> np.ndarray:
        nm = self.n[mu]
        out = np.zeros((nm, nm), dtype=np.complex128, order="F")
        check(L.lib().cgl_get_operator(self._h, mu, which, _dptr(out)), "cgl_get_operator")
        return out

    def split_terms(self):
        a, b = C.c_int(), C.c_int()
        check(L.lib().cgl_split_terms(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    # -- device work ---------------------------------------------------------
    def mode_product(self, mu: int, which: int, x, out) -> None:
        check(L.lib().cgl_mode_product(self._h, mu, which, C.c_void_p(x.data_ptr()),
                                       C.c_void_p(out.data_ptr())), "cgl_mode_product")

    def tucker(self, which: int, x, out) -> None:
        check(L.lib().cgl_tucker(self._h, which, C.c_void_p(x.data_ptr()),
                                 C.c_void_p(out.data_ptr())), "cgl_tucker")

    def step_strang(self, u, nsteps: int = 1) -> None:
        check(L.lib().cgl_step_strang(self._h, C.c_void_p(u.data_ptr()), int(nsteps)), "cgl_step_strang")

    def step_lawson4(self, u, nsteps: int = 1) -> None:
        check(L.lib().cgl_step_lawson4(self._h, C.c_void_p(u.data_ptr()), int(nsteps)),
              "cgl_step_lawson4")

    def step(self, method: str, u, nsteps: int = 1) -> None:
        """cgl_step: nsteps eager steps of any method."""
        check(L.lib().cgl_step(self._h, METHODS[method], C.c_void_p(u.data_ptr()), int(nsteps)),
              "cgl_step")

    def run(self, method: str, u, nsteps: int, check_every: int = 0) -> int:
        """cgl_run; returns the status code (CGL_ENONFINITE etc. are not raised)."""
        st = L.lib().cgl_run(self._h, METHODS[method], C.c_void_p(u.data_ptr()), int(nsteps),
                             int(check_every))
        if st not in (L.OK, L.ENONFINITE, L.EBLOWUP):
            raise CGLError(st, "cgl_run")
        return st

    def status(self) -> int:
        return L.lib().cgl_status(self._h)

    def clear_status(self) -> None:
        check(L.lib().cgl_clear_status(self._h))

    def destroy(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().cgl_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class BatchedPlan(Plan):
    """cgl_plan_batched: independent instances with their own grids and
    coefficients, stepped together.  State tensors are 1-D complex torch
    tensors holding every instance's column-stacked grid function at the
    offsets ``self.offsets``."""

    def __init__(self, grids, coeffs, tau: float, precision: str = "split",
                 master: bool = False, rk4_flow: bool = False, stream: Optional[int] = None,
                 three_term: bool = False):
        grids = [tuple(int(v) for v in g) for g in grids]
        self.grids = grids
        self.batch = len(grids)
        d = len(grids[0])
        assert all(len(g) == d for g in grids)
        self.n = grids[0]
        self.d = d
        self.tau = float(tau)
        self.precision = precision
        self.master = bool(master)
        flags = ((L.FLAG_FP64_MASTER if master else 0) | (L.FLAG_RK4_FLOW if rk4_flow else 0)
                 | (L.FLAG_THREE_TERM if three_term else 0))
        if stream is None:
            stream = current_stream_handle()
        self._stream = stream
        flat = [v for g in grids for v in g]
        arr = (C.c_int64 * len(flat))(*flat)
        carr = (L.Coeffs * self.batch)(*[_coeffs(c) for c in coeffs])
        h = C.c_void_p()
        check(L.lib().cgl_plan_batched(C.byref(h), self.batch, d, arr, carr, self.tau,
                                       PRECISIONS[precision], flags, C.c_void_p(stream)),
              "cgl_plan_batched")
        self._h = h
        self.offsets = []
        for j in range(self.batch):
            off = C.c_int64()
            check(L.lib().cgl_instance_offset(self._h, j, C.byref(off)))
            self.offsets.append(off.value)
        self.N = int(sum(int(np.prod(g)) for g in grids))

    def set_fd_operators_batched(self, problems) -> None:
        """FD operators of every instance (problems[j] with n, a, b, bc, coeffs)."""
        mats = []
        for p in problems:
            for nm in p.n:
                mats.append(fd_operator(nm, p.a, p.b, p.bc, p.coeffs, len(p.n)))
        self.set_operators_all(mats)

    def get_instance_operator(self, j: int, mu: int, which: int) -> np.ndarray:
        nm = self.grids[j][mu]
        out = np.zeros((nm, nm), dtype=np.complex128, order="F")
        check(L.lib().cgl_get_instance_operator(self._h, j, mu, which, _dptr(out)))
        return out

    def to_device_batched(self, states, dtype=None):
        torch = _torch()
        flat = np.concatenate([np.asarray(u).reshape(-1, order="F") for u in states])
        return torch.from_numpy(flat.astype(np.complex128)).to(device="cuda",
                                                                 dtype=dtype or self.state_dtype)

    def to_host_batched(self, t):
        v = t.detach().to("cpu").numpy().astype(np.complex128)
        out = []
        for j, g in enumerate(self.grids):
            Nj = int(np.prod(g))
            out.append(v[self.offsets[j]:self.offsets[j] + Nj].reshape(g, order="F"))
        return out


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def sur_param_count() -> int:
    n = C.c_int64()
    check(L.lib().cgl_sur_param_count(C.byref(n)))
    return n.value


class Surrogate:
    """cgl_sur_*: the residual conv net on an n1 x n2 grid.  States are 1-D
    complex64 torch tensors of batch * n1 * n2 elements (sample-major, each
    sample column-stacked); coefficient tensors are float32 (batch, 5) on the
    device; index tensors int32."""

    def __init__(self, n1: int, n2: int, max_batch: int, stream: Optional[int] = None):
        self.n1, self.n2, self.max_batch = int(n1), int(n2), int(max_batch)
        self.P = self.n1 * self.n2
        if stream is None:
            stream = current_stream_handle()
        h = C.c_void_p()
        check(L.lib().cgl_sur_create(C.byref(h), self.n1, self.n2, self.max_batch,
                                     C.c_void_p(stream)), "cgl_sur_create")
        self._h = h
        self.count = sur_param_count()

    def set_params(self, params: np.ndarray) -> None:
        a = np.ascontiguousarray(params, dtype=np.float32)
        assert a.size == self.count
        check(L.lib().cgl_sur_set_params(self._h, _fptr(a)), "cgl_sur_set_params")

    def set_loss(self, kind: str) -> None:
        """"mse" or "rel" (mean squared relative L2 error per sample)."""
        check(L.lib().cgl_sur_set_loss(self._h, {"mse": L.SUR_LOSS_MSE, "rel": L.SUR_LOSS_REL}[kind]),
              "cgl_sur_set_loss")

    def set_output_scale(self, scale: float) -> None:
        """y = base + scale * (network correction)."""
        check(L.lib().cgl_sur_set_output_scale(self._h, float(scale)), "cgl_sur_set_output_scale")

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.count, dtype=np.float32)
        check(L.lib().cgl_sur_get_params(self._h, _fptr(out)), "cgl_sur_get_params")
        return out

    def forward(self, batch: int, u, cstd, out, base=None) -> None:
        """out = network(u) about base (None: about u)."""
        check(L.lib().cgl_sur_forward(self._h, int(batch), _ptr(u), _ptr(cstd), _ptr(base),
                                      _ptr(out)), "cgl_sur_forward")

    def grad(self, batch: int, src, cstd, idx, target_offset: int, base=None):
        g = np.zeros(self.count, dtype=np.float32)
        loss = C.c_double()
        check(L.lib().cgl_sur_grad(self._h, int(batch), _ptr(src), _ptr(cstd), _ptr(idx),
                                   int(target_offset), _ptr(base), _fptr(g), C.byref(loss)),
              "cgl_sur_grad")
        return g, loss.value

    def train_step(self, batch: int, src, cstd, idx, target_offset: int, lr: float,
                   base=None) -> None:
        check(L.lib().cgl_sur_train_step(self._h, int(batch), _ptr(src), _ptr(cstd), _ptr(idx),
                                         int(target_offset), _ptr(base), float(lr)),
              "cgl_sur_train_step")

    def take_loss(self) -> float:
        v = C.c_double()
        check(L.lib().cgl_sur_take_loss(self._h, C.byref(v)), "cgl_sur_take_loss")
        return v.value

    def destroy(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().cgl_sur_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


SUR_BASES = {"input": L.SUR_BASE_INPUT, "linear": L.SUR_BASE_LINEAR, "strang": L.SUR_BASE_STRANG}


def run_surrogate(plan: Plan, sur: Surrogate, u, cstd, njumps: int, steps_per_jump: int,
                  check_every: int, tol: float, coarse: Optional[Plan] = None,
                  base: str = "input"):
    """cgl_run_surrogate; returns (status, dict of counters).  base "linear" or
    "strang" takes the jump's base from ``coarse`` (a plan of the same problem
    with step steps_per_jump * tau)."""
    c = np.ascontiguousarray(cstd, dtype=np.float64)
    stats = (C.c_int64 * 4)()
    st = L.lib().cgl_run_surrogate(plan._h, sur._h, _ptr(u), _dptr(c), int(njumps),
                                   int(steps_per_jump), int(check_every), float(tol),
                                   coarse._h if coarse is not None else None, SUR_BASES[base],
                                   stats)
    if st not in (L.OK, L.ENONFINITE, L.EBLOWUP):
        raise CGLError(st, "cgl_run_surrogate")
    return st, {"accepted": stats[0], "rejected": stats[1], "checks": stats[2],
                "plain_steps": stats[3]}


class CoupledPlan:
    """cgl_coupled_*: the two-field system of Section 4.4 on a periodic 2-D
    grid.  ``c`` has the fields a0, a1, b1, a2, a3, b3, a4, b4, a5; states are
    1-D complex torch tensors of 2 N elements (u then v, each column-stacked)."""

    def __init__(self, n: Sequence[int], c, tau: float, precision: str = "fp64",
                 stream: Optional[int] = None):
        self.n = tuple(int(v) for v in n)
        self.N = self.n[0] * self.n[1]
        self.precision = precision
        if stream is None:
            stream = current_stream_handle()
        cc = L.CoupledCoeffs(*(float(getattr(c, k)) for k in
                               ("a0", "a1", "b1", "a2", "a3", "b3", "a4", "b4", "a5")))
        nn = (C.c_int64 * 2)(*self.n)
        h = C.c_void_p()
        check(L.lib().cgl_coupled_plan(C.byref(h), nn, C.byref(cc), float(tau),
                                       L.FP64 if precision == "fp64" else L.SPLIT_BF16,
                                       C.c_void_p(stream)), "cgl_coupled_plan")
        self._h = h

    @property
    def dtype(self):
        torch = _torch()
        return torch.complex128 if self.precision == "fp64" else torch.complex64

    def set_periodic(self, mu: int, a: float, b: float) -> None:
        check(L.lib().cgl_coupled_set_periodic(self._h, int(mu), float(a), float(b)),
              "cgl_coupled_set_periodic")

    def get_factor(self, field: int, mu: int, which: int) -> np.ndarray:
        out = np.zeros(2 * self.n[mu], dtype=np.float64)
        check(L.lib().cgl_coupled_get_factor(self._h, int(field), int(mu), int(which), _dptr(out)),
              "cgl_coupled_get_factor")
        return out[0::2] + 1j * out[1::2]

    def to_device(self, W: np.ndarray):
        """W (2, n1, n2) -> device state (u then v, index 1 fastest)."""
        torch = _torch()
        flat = np.concatenate([np.asarray(W[k]).reshape(-1, order="F") for k in range(2)])
        return torch.from_numpy(flat.astype(np.complex128)).to(device="cuda", dtype=self.dtype)

    def to_host(self, t) -> np.ndarray:
        a = t.detach().to("cpu").numpy().astype(np.complex128)
        return np.stack([a[k * self.N:(k + 1) * self.N].reshape(self.n, order="F")
                         for k in range(2)])

    def step(self, method: str, w, nsteps: int = 1) -> None:
        check(L.lib().cgl_coupled_step(self._h, METHODS[method], C.c_void_p(w.data_ptr()),
                                       int(nsteps)), "cgl_coupled_step")

    def status(self) -> int:
        return L.lib().cgl_coupled_status(self._h)

    def destroy(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().cgl_coupled_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
