"""ctypes binding of liboecdg.so (the C ABI in include/oecdg.h).

Argument marshalling only: every step of the method runs in the HIP
library.  The first use (lib(), hence every solver handle) fails loudly if
the library is not built; there is no other implementation to fall back on.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboecdg.so")

OK, EINVAL, ENOMEM, EHIP, ENONFINITE, ENONPHYSICAL, EUNSUPPORTED, ETIMEOUT, ETOOBIG = 0, -1, -2, -3, -4, -5, -6, -7, -8
MODE_AUTO, MODE_EAGER, MODE_GRAPH, MODE_PERSISTENT = 0, 1, 2, 3
FLAG_ALLOW_NEGATIVE_PRESSURE = 1
OPT_MODE, OPT_TILE, OPT_GRAPH_STEPS, OPT_GRID, OPT_FOLD = 1, 2, 3, 4, 5

# every symbol include/oecdg.h declares
EXPORTS = ("oecdg_state_size", "oecdg_init", "oecdg_batch_offsets", "oecdg_set_option", "oecdg_dt",
           "oecdg_stage", "oecdg_run", "oecdg_run_noalloc", "oecdg_run_nonuniform", "oecdg_set_inflow", "oecdg_adjoint", "oecdg_destroy", "oecdg_strerror",
           "oecdg_last_error")


class Desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("k", C.c_int32), ("flux", C.c_int32), ("bc", C.c_int32),
                ("nx", C.c_int64), ("ny", C.c_int64),
                ("xlo", C.c_double), ("xhi", C.c_double), ("ylo", C.c_double), ("yhi", C.c_double),
                ("flux_param", C.c_double * 2), ("cfl", C.c_double),
                ("oe", C.c_int32), ("rk", C.c_int32),
                ("space", C.c_int32), ("flags", C.c_int32)]


class OECDGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(msg)
        self.code = code


_lib = None


def lib():
    """Load liboecdg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    H = C.c_void_p
    D = C.c_void_p          # device pointers
    L.oecdg_state_size.argtypes = [C.POINTER(Desc), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.oecdg_init.argtypes = [C.POINTER(Desc), C.c_int32, C.c_void_p, C.POINTER(H)]
    L.oecdg_batch_offsets.argtypes = [H, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.oecdg_set_option.argtypes = [H, C.c_int32, C.c_int64]
    L.oecdg_dt.argtypes = [H, D, D, C.POINTER(C.c_double)]
    L.oecdg_set_inflow.argtypes = [H, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.oecdg_stage.argtypes = [H, C.c_int32, C.c_double, C.c_double, D, D, D, D, D, D]
    L.oecdg_run.argtypes = [H, D, D, C.c_double, C.c_int64, C.c_double, C.POINTER(C.c_double),
                            C.POINTER(C.c_int64)]
    L.oecdg_run_noalloc.argtypes = [C.POINTER(Desc), C.c_void_p, D, D, C.c_double, C.c_int64, C.c_double,
                                    C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.oecdg_run_nonuniform.argtypes = [H, D, D, D, C.c_double, C.c_int64, C.c_double, C.POINTER(C.c_double),
                                       C.POINTER(C.c_int64)]
    L.oecdg_adjoint.argtypes = [H, D, D, C.c_int64, C.c_double, D, D, D, D, C.c_int32]
    L.oecdg_destroy.argtypes = [H]
    L.oecdg_destroy.restype = None
    L.oecdg_strerror.argtypes = [C.c_int]
    L.oecdg_strerror.restype = C.c_char_p
    L.oecdg_last_error.argtypes = [H]
    L.oecdg_last_error.restype = C.c_char_p
    _lib = L
    return L


def check(rc: int, handle=None, where: str = ""):
    if rc != OK:
        L = lib()
        msg = L.oecdg_strerror(rc).decode()
        if handle is not None:
            detail = L.oecdg_last_error(handle).decode()
            if detail:
                msg = f"{msg}: {detail}"
        raise OECDGError(rc, f"{where}: {msg}" if where else msg)
