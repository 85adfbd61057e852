"""ctypes binding of libcaspt2.so (argument marshalling only).

Every step of the computation runs in the HIP library; this module only
converts arguments.  Importing it fails loudly if the library was not built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcaspt2.so")

OK, E_ARG, E_NOMEM, E_DEVICE, E_NOCONV, E_INDEFINITE, E_NOTIMPL, E_STATE = 0, -1, -2, -3, -4, -5, -6, -7
MSMR, SSSR = 0, 1
FP64, MIXED = 0, 1
ENTRY_NAMES = ["ccvv+", "ccvv-", "cavv+", "cavv-", "aavv+", "aavv-", "ccav+", "ccav-",
               "ccaa+", "ccaa-", "aaav", "caaa", "caav"]


class Dims(ctypes.Structure):
    _fields_ = [("nclosed", ctypes.c_int32), ("nact", ctypes.c_int32), ("nvirt", ctypes.c_int32),
                ("naux", ctypes.c_int32), ("nstates", ctypes.c_int32), ("nelec", ctypes.c_int32),
                ("scheme", ctypes.c_int32), ("xms", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("shift", ctypes.c_double),
                ("ovl_thresh", ctypes.c_double)]


class Inputs(ctypes.Structure):
    _fields_ = [("fock", ctypes.c_void_p), ("hcore", ctypes.c_void_p), ("dfB", ctypes.c_void_p),
                ("ci", ctypes.c_void_p), ("eref", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("flags", ctypes.c_int32), ("resnorm", ctypes.c_double),
                ("e0", ctypes.c_double), ("min_denom", ctypes.c_double),
                ("emin_kept", ctypes.c_double), ("emax_dropped", ctypes.c_double),
                ("refinements", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)

SIGNATURES = {
    "caspt2_create": (ctypes.c_int, [ctypes.POINTER(Dims), ctypes.POINTER(Inputs), ctypes.c_int, _P,
                                     ctypes.POINTER(_P)]),
    "caspt2_create_many": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(Dims), ctypes.POINTER(Inputs), ctypes.c_int,
                                          ctypes.POINTER(_P), ctypes.c_int32, ctypes.POINTER(_P),
                                          ctypes.POINTER(ctypes.c_int32)]),
    "caspt2_destroy": (ctypes.c_int, [_P]),
    "caspt2_set_precision": (ctypes.c_int, [_P, ctypes.c_int32]),
    "caspt2_set_streams": (ctypes.c_int, [_P, ctypes.c_int32]),
    "caspt2_autotune": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.c_int32]),
    "caspt2_tune_entry": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "caspt2_vector_length": (ctypes.c_int64, [_P]),
    "caspt2_layout": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "caspt2_residual": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "caspt2_residual_all": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    "caspt2_residual_all_many": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_P), ctypes.c_int32,
                                                ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_int32)]),
    "caspt2_solve_amplitudes": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int32, _P, ctypes.POINTER(Info)]),
    "caspt2_get_amplitudes": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "xms_rotate": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _D, _D, _D, _D]),
    "caspt2_get_xms": (ctypes.c_int, [_P, _D, _D]),
    "xms_rotate_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P]),
    "xms_heff": (ctypes.c_int, [_P, _D, _D, _D]),
    "caspt2_solve_lambda": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _P,
                                           ctypes.POINTER(Info)]),
    "caspt2_get_lambda": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "caspt2_batch_solve": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.c_double, ctypes.c_int32, ctypes.POINTER(Info),
                                          ctypes.POINTER(Info)]),
    "caspt2_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "caspt2_profile": (ctypes.c_int, [_P, ctypes.c_int32]),
    "caspt2_profile_entry": (ctypes.c_int, [_P, ctypes.c_int32, _D, ctypes.POINTER(ctypes.c_int64), _D]),
    "caspt2_debug_gemm": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                         _P, _P, _P]),
    "caspt2_debug_gemm_f32": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                             _P, _P, _P]),
    "caspt2_debug_entry": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _D]),
    "caspt2_debug_source": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P]),
    "caspt2_debug_eigh": (ctypes.c_int, [ctypes.c_int32, _P, _D, _P]),
    "caspt2_debug_residual_f32": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    "caspt2_set_verbose": (ctypes.c_int, [_P, ctypes.c_int32]),
    "caspt2_debug_eigh_method": (ctypes.c_int, [ctypes.c_int32, _P, _D, _P, ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_int32)]),
    "caspt2_debug_eigh_abs": (ctypes.c_int, [ctypes.c_int32, _P, _D, _P, ctypes.c_int32, ctypes.c_double,
                                             ctypes.POINTER(ctypes.c_int32)]),
    "caspt2_debug_ccvv_passes": (ctypes.c_int, [ctypes.c_int32]),
    "caspt2_debug_ccvv_passes_used": (ctypes.c_int, [_P, ctypes.c_int32]),
    "caspt2_profile_stage": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_char_p, ctypes.c_int32, _D,
                                            ctypes.POINTER(ctypes.c_int64)]),
    "caspt2_densities": (ctypes.c_int, [_P, _D, _P, _D, _D, _D]),
    "caspt2_density2_length": (ctypes.c_int64, [_P]),
    "caspt2_density2_layout": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                              ctypes.POINTER(ctypes.c_int32)]),
    "caspt2_last_error": (ctypes.c_char_p, []),
}


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


class Caspt2Error(RuntimeError):
    def __init__(self, code: int, where: str, text: str):
        super().__init__(f"{where}: status {code} ({text})")
        self.code = code
