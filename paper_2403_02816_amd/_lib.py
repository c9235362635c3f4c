"""ctypes declarations of libcgl.so (the C ABI in include/cgl.h).

Argument marshalling only: every step of the stepper runs in the library.
Loading fails loudly when the built library is missing; there is no other
implementation to fall back to.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcgl.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTREADY, ENONFINITE, EBLOWUP, EGATE, ESCRATCH = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
FP64, SPLIT_BF16 = 0, 1
STRANG, LAWSON4, SPLIT4, LAWSON2 = 0, 1, 2, 3
DIRICHLET, NEUMANN, PERIODIC = 0, 1, 2
E, H = 0, 1
FLAG_FP64_MASTER = 1
FLAG_RK4_FLOW = 2
FLAG_THREE_TERM = 4
SUR_LOSS_MSE, SUR_LOSS_REL = 0, 1
SUR_BASE_INPUT, SUR_BASE_LINEAR, SUR_BASE_STRANG = 0, 1, 2


class Coeffs(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("a1", "b1", "a2", "a3", "b3", "a4", "b4")]


class CoupledCoeffs(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("a0", "a1", "b1", "a2", "a3", "b3", "a4", "b4", "a5")]


_P = C.c_void_p
_I64 = C.c_int64
_D = C.c_double
_DP = C.POINTER(C.c_double)
_I = C.c_int

SIGNATURES = {
    "cgl_plan": (_I, [C.POINTER(_P), _I, C.POINTER(_I64), C.POINTER(Coeffs), _D, _I, C.c_uint, _P]),
    "cgl_set_operators": (_I, [_P, _I, _DP]),
    "cgl_set_exponentials": (_I, [_P, _I, _DP, _DP]),
    "cgl_fd_operator": (_I, [_I64, _D, _D, _I, C.POINTER(Coeffs), _I, _DP]),
    "cgl_fd_operator_ex": (_I, [_I64, _D, _D, _I, _I, _I, C.POINTER(Coeffs), _I, _DP]),
    "cgl_expm": (_I, [_I64, _DP, _D, _DP]),
    "cgl_get_operator": (_I, [_P, _I, _I, _DP]),
    "cgl_set_periodic": (_I, [_P, _I, _D, _D]),
    "cgl_get_periodic_factor": (_I, [_P, _I, _I, _DP]),
    "cgl_mode_product": (_I, [_P, _I, _I, _P, _P]),
    "cgl_tucker": (_I, [_P, _I, _P, _P]),
    "cgl_tucker_noalloc": (_I, [_P, _I, _P, _P]),
    "cgl_step_strang": (_I, [_P, _P, _I64]),
    "cgl_step_lawson4": (_I, [_P, _P, _I64]),
    "cgl_step": (_I, [_P, _I, _P, _I64]),
    "cgl_run": (_I, [_P, _I, _P, _I64, _I64]),
    "cgl_status": (_I, [_P]),
    "cgl_clear_status": (_I, [_P]),
    "cgl_destroy": (None, [_P]),
    "cgl_strerror": (C.c_char_p, [_I]),
    "cgl_split_terms": (_I, [_P, C.POINTER(_I), C.POINTER(_I)]),
    "cgl_set_operators_all": (_I, [_P, C.POINTER(_DP)]),
    "cgl_plan_batched": (_I, [C.POINTER(_P), _I, _I, C.POINTER(_I64), C.POINTER(Coeffs), _D, _I,
                              C.c_uint, _P]),
    "cgl_batch_size": (_I, [_P, C.POINTER(_I)]),
    "cgl_instance_offset": (_I, [_P, _I, C.POINTER(_I64)]),
    "cgl_set_instance_operators": (_I, [_P, _I, _I, _DP]),
    "cgl_get_instance_operator": (_I, [_P, _I, _I, _I, _DP]),
    "cgl_sur_param_count": (_I, [C.POINTER(_I64)]),
    "cgl_sur_create": (_I, [C.POINTER(_P), _I64, _I64, _I, _P]),
    "cgl_sur_set_params": (_I, [_P, C.POINTER(C.c_float)]),
    "cgl_sur_get_params": (_I, [_P, C.POINTER(C.c_float)]),
    "cgl_sur_set_loss": (_I, [_P, _I]),
    "cgl_sur_forward": (_I, [_P, _I, _P, _P, _P, _P]),
    "cgl_sur_set_output_scale": (_I, [_P, C.c_float]),
    "cgl_sur_grad": (_I, [_P, _I, _P, _P, _P, _I64, _P, C.POINTER(C.c_float), _DP]),
    "cgl_sur_train_step": (_I, [_P, _I, _P, _P, _P, _I64, _P, C.c_float]),
    "cgl_sur_take_loss": (_I, [_P, _DP]),
    "cgl_sur_destroy": (None, [_P]),
    "cgl_run_surrogate": (_I, [_P, _P, _P, _DP, _I64, _I64, _I64, _D, _P, _I, C.POINTER(_I64)]),
    "cgl_coupled_plan": (_I, [C.POINTER(_P), C.POINTER(_I64), C.POINTER(CoupledCoeffs), _D, _I, _P]),
    "cgl_coupled_set_periodic": (_I, [_P, _I, _D, _D]),
    "cgl_coupled_get_factor": (_I, [_P, _I, _I, _I, _DP]),
    "cgl_coupled_step": (_I, [_P, _I, _P, _I64]),
    "cgl_coupled_status": (_I, [_P]),
    "cgl_coupled_destroy": (None, [_P]),
}

_lib = None


def lib() -> C.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2403_02816_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class CGLError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        msg = lib().cgl_strerror(status).decode()
        super().__init__(f"{where}: {msg} ({status})" if where else f"{msg} ({status})")


def check(status: int, where: str = "") -> int:
    if status != OK:
        raise CGLError(status, where)
    return status
