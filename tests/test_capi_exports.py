"""The C interface library loads and exports every function include/gsr.h declares
(no GPU needed: nothing is called except pure host helpers)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsr.h")
LIB = os.path.join(ROOT, "paper_2503_22863_amd", "libgsr.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gsr_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2503_22863_amd import build

        build.build()
    import torch  # noqa: F401  (same HIP runtime as the package uses)

    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_host_helpers(lib):
    lib.gsr_cov_bytes.restype = ctypes.c_int64
    lib.gsr_cov_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64]
    assert lib.gsr_cov_bytes(3, 20, 10) == -1
    lib.gsr_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.gsr_version()


def test_num_unknowns_rejects_bad_dims(lib):
    class Dims(ctypes.Structure):
        _fields_ = [("n_stars", ctypes.c_int64), ("m", ctypes.c_int64), ("n_att", ctypes.c_int64),
                    ("n_instr", ctypes.c_int64), ("n_glob", ctypes.c_int32), ("value_type", ctypes.c_int32)]

    f = lib.gsr_num_unknowns
    f.restype = ctypes.c_int64
    f.argtypes = [ctypes.c_void_p]
    assert f(ctypes.byref(Dims(1000, 20000, 64, 32, 1, 0))) == 5225
    assert f(ctypes.byref(Dims(10**6, 0, 40000, 200, 1, 0))) == 5120201
    assert f(ctypes.byref(Dims(1, 1, 3, 6, 1, 0))) == -1
    assert f(ctypes.byref(Dims(1, 1, 4, 6, 2, 0))) == -1
    assert f(None) == -1
