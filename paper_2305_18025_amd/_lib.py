"""ctypes binding of libpimdb.so (the C ABI in include/pimdb.h).

Argument marshalling only: every computation happens in the HIP library.
The library is loaded from this package directory; if it is missing the
import of any GPU entry point raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libpimdb.so")

PIMDB_OK = 0
PIMDB_EINVAL = -1
PIMDB_ENOSYS = -2
PIMDB_EWORKSPACE = -3
PIMDB_EDEVICE = -4
PIMDB_ENONFINITE = -5
PIMDB_ERANGE = -6

PIMDB_FP64 = 0
PIMDB_MIXED = 1
PIMDB_FP64_DIRECT = 2
PIMDB_ALG_FAST = 0
PIMDB_ALG_ORIGINAL = 1
PIMDB_SHIFT_MIN = 0
PIMDB_SHIFT_TWO_TERM = 1

STATUS_NONFINITE_INPUT = 1
STATUS_NONFINITE_OUTPUT = 2
STATUS_RANGE = 4
STATUS_PRECISION = 8
STATUS_TIMEOUT = 16

DEBUG_PROBABILITIES = 1
DEBUG_CYCLE_ENERGIES = 2
DEBUG_FORWARD = 3
DEBUG_BACKWARD = 4

MAX_N = 4096
MAX_BATCH = 65536
STATIC_SCRATCH_BYTES = 16 << 20

_c_int, _c_i32, _c_i64 = ctypes.c_int, ctypes.c_int32, ctypes.c_int64
_c_dbl, _c_sz, _vp = ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
_pi64, _pi32, _pdbl = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
_handle = ctypes.c_void_p

# name -> (restype, argtypes); kept in the order of include/pimdb.h
SIGNATURES = {
    "pimdb_create": (_c_int, [ctypes.POINTER(_handle), _c_int, _vp]),
    "pimdb_destroy": (_c_int, [_handle]),
    "pimdb_set_stream": (_c_int, [_handle, _vp]),
    "pimdb_set_system": (_c_int, [_handle, _c_i64, _c_i32, _c_dbl, _c_dbl, _c_dbl]),
    "pimdb_set_batch": (_c_int, [_handle, _c_i32, _pi64, _pi32, _pdbl, _pdbl, _pdbl]),
    "pimdb_set_box": (_c_int, [_handle, _c_dbl]),
    "pimdb_set_trap": (_c_int, [_handle, _c_dbl]),
    "pimdb_set_precision": (_c_int, [_handle, _c_int]),
    "pimdb_set_algorithm": (_c_int, [_handle, _c_int, _c_int]),
    "pimdb_set_pair_gaussian": (_c_int, [_handle, ctypes.c_double, ctypes.c_double]),
    "pimdb_pair_forces": (_c_int, [_handle, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pimdb_get_algorithm": (_c_int, [_handle, ctypes.POINTER(_c_int), ctypes.POINTER(_c_int)]),
    "pimdb_set_tuning": (_c_int, [_handle, _c_int, _c_int]),
    "pimdb_set_timing": (_c_int, [_handle, _c_int]),
    "pimdb_last_timing": (_c_int, [_handle, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "pimdb_set_split": (_c_int, [_handle, _c_int]),
    "pimdb_get_split": (_c_int, [_handle, ctypes.POINTER(_c_int), ctypes.POINTER(_c_int), ctypes.POINTER(_c_int)]),
    "pimdb_get_tuning": (_c_int, [_handle, ctypes.POINTER(_c_int), ctypes.POINTER(_c_int)]),
    "pimdb_system_offset": (_c_i64, [_handle, _c_i32]),
    "pimdb_total_elements": (_c_i64, [_handle]),
    "pimdb_workspace_bytes": (_c_sz, [_handle]),
    "pimdb_bind_workspace": (_c_int, [_handle, _vp, _c_sz]),
    "pimdb_exchange_energy": (_c_int, [_handle, _vp, _vp]),
    "pimdb_exchange_forces": (_c_int, [_handle, _vp, _vp, _vp]),
    "pimdb_exchange_forces_batched": (_c_int, [_handle, _vp, _vp, _vp, _vp]),
    "pimdb_exchange_forces_static": (_c_int, [_handle, _vp, _vp, _vp]),
    "pimdb_state_bytes": (_c_sz, [_handle]),
    "pimdb_exchange_energy_save": (_c_int, [_handle, _vp, _vp, _vp]),
    "pimdb_exchange_adjoint": (_c_int, [_handle, _vp, _vp, _vp, _vp]),
    "pimdb_md_step": (_c_int, [_handle, _vp, _vp, _vp, _vp, _c_dbl]),
    "pimdb_distinguishable_forces": (_c_int, [_handle, _vp, _vp, _vp]),
    "pimdb_debug_get": (_c_int, [_handle, _vp, _c_i32, _c_int, _vp]),
    "pimdb_endpoint_springs": (_c_int, [_handle, _vp, _c_i32, _c_int, _vp]),
    "pimdb_status": (_c_int, [_handle, _pi32]),
    "pimdb_strerror": (ctypes.c_char_p, [_c_int]),
    "pimdb_last_error": (ctypes.c_char_p, [_handle]),
}

_lib = None


class PimdbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("pimdb error %d (%s)%s" % (code, strerror(code) if _lib else "", (": " + msg) if msg else ""))
        self.code = code


def load():
    """Load libpimdb.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise OSError("libpimdb.so not found at %s; run paper_2305_18025_amd.build" % SO_PATH)
        lib = ctypes.CDLL(SO_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def strerror(code) -> str:
    return load().pimdb_strerror(int(code)).decode()


def check(rc, handle=None):
    if rc != PIMDB_OK:
        msg = ""
        if handle is not None and _lib is not None:
            raw = _lib.pimdb_last_error(handle)
            msg = raw.decode() if raw else ""
        raise PimdbError(rc, msg)
    return rc
