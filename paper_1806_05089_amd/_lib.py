"""ctypes declarations of libpond's C ABI (include/pond.h).  Marshalling only."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpond.so")

POND_OK = 0
POND_E_INVALID = -1
POND_E_NULL = -2
POND_E_ALIAS = -3
POND_E_STATE = -4
POND_E_HIP = -5
POND_E_UNSUPPORTED = -6

POND_F64 = 0
POND_F32_MIXED = 1
POND_OP_STEP = 0
POND_OP_STEP_ADJOINT = 1
POND_PERIODIC = 0
POND_ZERO_GRADIENT = 1

POND_ITERS_MASK = 0x3F
POND_ITERS_NONCONVERGED = 0x40
POND_ITERS_BAD = 0x80

EXPORTED = ("pond_init", "pond_step", "pond_moments", "pond_step_adjoint", "pond_last_error",
            "pond_abi_version", "pond_tape_bytes", "pond_step_record",
            "pond_step_adjoint_recorded", "pond_workspace_bytes", "pond_init_adjoint",
            "pond_step_noalloc")


class pond_config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("q1d", C.c_int32),
                ("precision", C.c_int32), ("isothermal", C.c_int32), ("bc_x", C.c_int32),
                ("bc_y", C.c_int32), ("max_iter", C.c_int32), ("fixed_iter", C.c_int32),
                ("seed_mode", C.c_int32), ("tau", C.c_double), ("eps_abs", C.c_double),
                ("eps_rel", C.c_double)]


class pond_state(C.Structure):
    _fields_ = [("f", C.c_void_p), ("g", C.c_void_p), ("iters", C.c_void_p)]


class pond_stats(C.Structure):
    _fields_ = [("nonconverged", C.c_int64), ("bad_state", C.c_int64), ("max_iters", C.c_int32),
                ("mean_iters", C.c_double), ("iter_hist", C.c_int64 * (POND_ITERS_MASK + 1))]


class PondError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libpond error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str | None = None):
    """Load libpond.so (built in-tree by paper_1806_05089_amd.build, or the file
    named by POND_LIBRARY).  No fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        path = os.environ.get("POND_LIBRARY", LIB_PATH)
    if not os.path.exists(path):
        raise ImportError(f"libpond.so not found at {path}; build it with "
                          "`python -m paper_1806_05089_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(path)
    cp = C.POINTER(pond_config)
    sp = C.POINTER(pond_state)
    dp = C.c_void_p
    lib.pond_init.argtypes = [cp, dp, dp, dp, dp, sp, dp]
    lib.pond_init.restype = C.c_int
    lib.pond_step.argtypes = [cp, sp, sp, C.c_int32, dp, C.POINTER(pond_stats)]
    lib.pond_step.restype = C.c_int
    lib.pond_moments.argtypes = [cp, sp, dp, dp, dp, dp, dp, dp]
    lib.pond_moments.restype = C.c_int
    lib.pond_step_adjoint.argtypes = [cp, sp, sp, sp, sp, dp, dp, C.c_int64, dp]
    lib.pond_step_adjoint.restype = C.c_int
    lib.pond_tape_bytes.argtypes = [cp, C.POINTER(C.c_int64)]
    lib.pond_tape_bytes.restype = C.c_int
    lib.pond_step_record.argtypes = [cp, sp, sp, dp, dp]
    lib.pond_step_record.restype = C.c_int
    lib.pond_step_adjoint_recorded.argtypes = [cp, sp, sp, dp, sp, sp, dp, dp]
    lib.pond_step_adjoint_recorded.restype = C.c_int
    lib.pond_workspace_bytes.argtypes = [cp, C.c_int32, C.POINTER(C.c_int64)]
    lib.pond_workspace_bytes.restype = C.c_int
    lib.pond_init_adjoint.argtypes = [cp, dp, dp, dp, dp, dp, dp, dp]
    lib.pond_init_adjoint.restype = C.c_int
    lib.pond_step_noalloc.argtypes = [cp, sp, sp, C.c_int32, dp, C.POINTER(pond_stats)]
    lib.pond_step_noalloc.restype = C.c_int
    lib.pond_last_error.argtypes = []
    lib.pond_last_error.restype = C.c_char_p
    lib.pond_abi_version.argtypes = []
    lib.pond_abi_version.restype = C.c_int
    _lib = lib
    return lib


def check(rc: int):
    if rc != POND_OK:
        msg = load().pond_last_error().decode(errors="replace")
        raise PondError(rc, msg)
