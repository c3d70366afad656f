"""ctypes binding of libexx.so: argument marshalling only.

Loading fails loudly when the library has not been built; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libexx.so")

# enums mirrored from include/exx.h
BC_PERIODIC, BC_FREE, BC_SURFACE, BC_WIRE = 0, 1, 2, 3
KERNEL_COULOMB, KERNEL_SCREENED, KERNEL_ISF = 0, 1, 2
PREC_FP32, PREC_FP64_PLAIN, PREC_FP64_FUSED = 0, 1, 2
MODE_ENERGY, MODE_KPSI, MODE_ENERGY_KPSI = 1, 2, 3
FLAG_ACCUMULATE = 1
PLAN_COMPLEX = 1
BATCH_GRAPH, BATCH_COMPLEX, BATCH_MERGE = 1, 2, 4

ERRORS = {
    0: "EXX_OK", -1: "EXX_ERR_INVALID_ARG", -2: "EXX_ERR_UNSUPPORTED_SIZE", -3: "EXX_ERR_CAPACITY",
    -4: "EXX_ERR_WORKSPACE", -5: "EXX_ERR_ALIGNMENT", -6: "EXX_ERR_HIP",
    -7: "EXX_ERR_NOT_PREPARED", -8: "EXX_ERR_INTERNAL",
}


class ExxGrid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double),
                ("bc", C.c_int), ("kernel", C.c_int), ("R", C.c_double), ("omega", C.c_double)]


class ExxTuning(C.Structure):
    _fields_ = [("tile", C.c_int), ("batch_slots", C.c_int), ("slab_threads", C.c_int),
                ("streams", C.c_int), ("slab_form", C.c_int)]


SLAB_FORMS = {"shared": 1, "wave": 2}


PASS_KINDS = ["convert", "zero", "pass_a", "pass_b", "pass_c", "finalize", "plain_fft",
              "plain_other"]


class ExxPassTimes(C.Structure):
    _fields_ = [("ms", C.c_double * 8), ("launches", C.c_longlong * 8)]


class ExxSystem(C.Structure):
    _fields_ = [("psi", C.c_void_p), ("occ", C.c_void_p), ("ex_out", C.c_void_p),
                ("kpsi", C.c_void_p), ("pair_e", C.c_void_p)]


# name -> (restype, argtypes); every symbol declared in include/exx.h
SIGNATURES = {
    "exx_plan_create": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(ExxGrid), C.c_int, C.c_int, C.c_uint]),
    "exx_plan_destroy": (None, [C.c_void_p]),
    "exx_plan_prepare": (C.c_int, [C.c_void_p, C.c_int]),
    "exx_workspace_bytes": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_size_t)]),
    "exx_compute": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_uint,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "exx_gradient": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                               C.c_void_p]),
    "exx_compute_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                      C.c_uint, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "exx_plan_get_tuning": (C.c_int, [C.c_void_p, C.POINTER(ExxTuning)]),
    "exx_plan_set_tuning": (C.c_int, [C.c_void_p, C.POINTER(ExxTuning)]),
    "exx_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                               C.c_size_t, C.c_void_p, C.c_int, C.c_char_p]),
    "exx_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(ExxGrid), C.POINTER(C.c_int),
                                   C.c_int, C.c_int, C.c_uint]),
    "exx_batch_destroy": (None, [C.c_void_p]),
    "exx_batch_workspace_bytes": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "exx_batch_compute": (C.c_int, [C.c_void_p, C.POINTER(ExxSystem), C.c_int, C.c_uint, C.c_void_p,
                                    C.c_size_t, C.c_void_p]),
    "exx_batch_autotune": (C.c_int, [C.c_void_p, C.POINTER(ExxSystem), C.c_void_p, C.c_size_t,
                                     C.c_void_p, C.c_int, C.c_char_p]),
    "exx_batch_get_tuning": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(ExxTuning)]),
    "exx_error_string": (C.c_char_p, [C.c_int]),
    "exx_last_error": (C.c_char_p, []),
    "exx_plan_schedule_info": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_longlong),
                                         C.POINTER(C.c_longlong)]),
    "exx_version": (C.c_char_p, []),
    "exx_plan_enable_profiling": (C.c_int, [C.c_void_p, C.c_int]),
    "exx_plan_read_profile": (C.c_int, [C.c_void_p, C.POINTER(ExxPassTimes)]),
}

_lib = None


class ExxError(RuntimeError):
    def __init__(self, code: int, where: str, message: str):
        super().__init__(f"{where}: {ERRORS.get(code, code)}: {message}")
        self.code = code


def lib() -> C.CDLL:
    """The loaded library (raises if libexx.so is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -m paper_1712_07973_amd.build` "
                "(the HIP library is required, there is no fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code: int, where: str) -> None:
    if code != 0:
        msg = lib().exx_last_error()
        raise ExxError(code, where, msg.decode() if msg else "")
