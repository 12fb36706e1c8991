"""ctypes view of the C ABI in include/mdd.h (libmdd.so, built in-tree).

Loading fails loudly if the library has not been built: there is no fallback
implementation of any step in Python.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libmdd.so")

MDD_OK, MDD_EINVAL, MDD_ESHAPE, MDD_ENOMEM, MDD_EHIP, MDD_EUNSUPPORTED, MDD_ESTATE = \
    0, -1, -2, -3, -4, -5, -6
MDD_ELIMIT = -7
NOALLOC_WORKSPACE_BYTES = 64 << 20
PREC = {"fp32": 0, "bf16x3": 1, "fp16x3": 2, "bf16": 3, "fp32_cgemm": 4}
FLAG_STORE_RF = 1
FLAG_FULL_GRAD = 2
FLAG_STREAM_KERNEL = 4
FLAG_STREAM_DATA = 8
OPT = {"sgd": 0, "adam": 1, "nsgd": 2}
KC_NAMES = ("fft_model", "gemm", "update", "reduce", "data_fft", "reciprocity")

# Entry points the header declares (checked by the test-suite against the .so).
EXPORTS = ("mdd_workspace_bytes", "mdd_plan_create", "mdd_plan_destroy", "mdd_plan_set_stream",
           "mdd_set_kernel", "mdd_stage_kernel", "mdd_set_data", "mdd_stage_data", "mdd_set_mask", "mdc_forward",
           "mdc_adjoint", "mdc_forward_rec", "mdc_adjoint_rec",
           "mdd_stoch_grad", "mdd_stoch_grad_noalloc", "mdd_step", "mdd_full_grad", "mdd_full_step",
           "mdd_reciprocity", "mdd_check_batch_host", "mdd_invalidate_model_spectra",
           "mdd_sigma_max2",
           "mdd_profile_enable", "mdd_profile_read", "mdd_calibrate_update", "mdd_calibrate_rows",
           "mdd_status_string", "mdd_plan_last_hip_error")


class Dims(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int32), ("nr", ctypes.c_int32), ("nvs", ctypes.c_int32),
                ("nt", ctypes.c_int32), ("nf", ctypes.c_int32), ("nb_max", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_int32)]


class Opt(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("mu", ctypes.c_double), ("t", ctypes.c_int64)]


class MddError(RuntimeError):
    def __init__(self, fn, status, hip=0):
        self.status = status
        msg = f"{fn} failed: {status_string(status)} ({status})"
        if hip:
            msg += f", hipError_t {hip}"
        super().__init__(msg)


_lib = None
_P = ctypes.c_void_p
_I32 = ctypes.c_int32


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2202_04486_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "mdd_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Dims)]),
        "mdd_plan_create": (_I32, [ctypes.POINTER(Dims), _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
        "mdd_plan_destroy": (_I32, [_P]),
        "mdd_plan_set_stream": (_I32, [_P, _P]),
        "mdd_set_kernel": (_I32, [_P, _P]),
        "mdd_stage_kernel": (_I32, [_P, _P, _I32]),
        "mdd_set_data": (_I32, [_P, _P]),
        "mdd_stage_data": (_I32, [_P, _P, _I32]),
        "mdd_set_mask": (_I32, [_P, _P]),
        "mdc_forward": (_I32, [_P, _P, _P, _I32, _P]),
        "mdc_adjoint": (_I32, [_P, _P, _P, _I32, _P]),
        "mdc_forward_rec": (_I32, [_P, _P, _P, _I32, _P]),
        "mdc_adjoint_rec": (_I32, [_P, _P, _P, _I32, _P]),
        "mdd_stoch_grad": (_I32, [_P, _P, _P, _I32, _P, _P, _P]),
        "mdd_stoch_grad_noalloc": (_I32, [ctypes.POINTER(Dims), _P, _P, _P, _P, _P, _I32, _P, _P,
                                          _P, _P]),
        "mdd_step": (_I32, [_P, _P, _P, _P, ctypes.POINTER(Opt), _P, _I32, _P, _P]),
        "mdd_full_grad": (_I32, [_P, _P, _P, _P, _P]),
        "mdd_full_step": (_I32, [_P, _P, _P, _P, ctypes.POINTER(Opt), _P, _P]),
        "mdd_reciprocity": (_I32, [_P, _P, _I32, _I32, _P]),
        "mdd_check_batch_host": (_I32, [_P, _I32, _I32, _I32]),
        "mdd_invalidate_model_spectra": (_I32, [_P]),
        "mdd_sigma_max2": (_I32, [_P, _I32, _P]),
        "mdd_profile_enable": (_I32, [_P, _I32, _I32]),
        "mdd_profile_read": (_I32, [_P, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64)]),
        "mdd_calibrate_update": (_I32, [_P, _P, _P, _P, _I32, _I32, _I32, _I32, _I32, _P]),
        "mdd_calibrate_rows": (_I32, [_P, _P, _P, _I32, _I32, _I32, _I32, _I32, _P]),
        "mdd_status_string": (ctypes.c_char_p, [_I32]),
        "mdd_plan_last_hip_error": (_I32, [_P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().mdd_status_string(int(status)).decode()


def check(fn: str, status: int, plan=None) -> None:
    if status != MDD_OK:
        hip = load().mdd_plan_last_hip_error(plan) if plan else 0
        raise MddError(fn, status, hip)


def make_dims(ns, nr, nvs, nt, nf, nb_max, precision="fp32", flags=0) -> Dims:
    prec = PREC[precision] if isinstance(precision, str) else int(precision)
    return Dims(ns, nr, nvs, nt, nf, nb_max, prec, flags)


def workspace_bytes(dims: Dims) -> int:
    return int(load().mdd_workspace_bytes(ctypes.byref(dims)))
