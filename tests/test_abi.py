"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function that include/pimdb.h declares, the binding covers them, the
constants agree, and host validation rejects bad arguments without touching
a device."""
import ctypes
import os
import re

import pytest

from paper_2305_18025_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pimdb.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pimdb_[a-z_]+)\s*\(", text)))


def _defines():
    out = {}
    for name, val in re.findall(r"#define\s+(PIMDB_[A-Z0-9_]+)\s+\(?(-?\d+)\)?", open(HEADER).read()):
        out[name] = int(val)
    return out


def test_library_loads_and_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n


def test_binding_signatures_cover_header():
    assert sorted(_lib.SIGNATURES) == _declared()


def test_constants_match_header():
    d = _defines()
    for name in ["OK", "EINVAL", "ENOSYS", "EWORKSPACE", "EDEVICE", "ENONFINITE", "ERANGE", "FP64", "MIXED",
                 "FP64_DIRECT"]:
        assert getattr(_lib, "PIMDB_" + name) == d["PIMDB_" + name]
    assert _lib.MAX_N == d["PIMDB_MAX_N"]
    assert _lib.MAX_BATCH == d["PIMDB_MAX_BATCH"]
    assert _lib.STATIC_SCRATCH_BYTES == d["PIMDB_STATIC_SCRATCH_BYTES"]
    assert _lib.DEBUG_PROBABILITIES == d["PIMDB_DEBUG_PROBABILITIES"]
    assert _lib.DEBUG_BACKWARD == d["PIMDB_DEBUG_BACKWARD"]
    assert _lib.STATUS_RANGE == d["PIMDB_STATUS_RANGE"]
    assert _lib.STATUS_PRECISION == d["PIMDB_STATUS_PRECISION"]


def test_strerror_texts():
    for code in range(0, -7, -1):
        assert _lib.strerror(code) and _lib.strerror(code) != "unknown error"
    assert _lib.strerror(-99) == "unknown error"


def test_null_handle_is_rejected():
    lib = _lib.load()
    assert lib.pimdb_set_system(None, 8, 4, 1.0, 1.0, 1.0) == _lib.PIMDB_EINVAL
    assert lib.pimdb_exchange_forces(None, None, None, None) == _lib.PIMDB_EINVAL
    assert lib.pimdb_exchange_forces_static(None, None, None, None) == _lib.PIMDB_EINVAL
    assert lib.pimdb_exchange_energy(None, None, None) == _lib.PIMDB_EINVAL
    assert lib.pimdb_status(None, None) == _lib.PIMDB_EINVAL
    assert lib.pimdb_workspace_bytes(None) == 0
    assert lib.pimdb_system_offset(None, 0) == -1
    assert lib.pimdb_destroy(None) == _lib.PIMDB_OK
    assert lib.pimdb_create(None, 0, None) == _lib.PIMDB_EINVAL


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    lib = _lib.load()
    h = ctypes.c_void_p(123)
    assert lib.pimdb_create(ctypes.byref(h), 0, None) == _lib.PIMDB_EDEVICE
    assert h.value is None
