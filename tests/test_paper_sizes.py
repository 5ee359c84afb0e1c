"""Sizes the paper prints, checked against the library's Eq. (5) / Eq. (6) helper
and the 24-coefficient row form (golden values in tests/golden/paper_sizes.json)."""
import ctypes
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_sizes.json")))


@pytest.fixture(scope="module")
def cov_bytes():
    lib_path = os.path.join(ROOT, "paper_2503_22863_amd", "libgsr.so")
    if not os.path.exists(lib_path):
        from paper_2503_22863_amd import build

        build.build()
    import torch  # noqa: F401

    f = ctypes.CDLL(lib_path).gsr_cov_bytes
    f.restype = ctypes.c_int64
    f.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64]
    return f


def test_cycle_sizes(cov_bytes):
    v1, v2 = GOLD["cycle_v1"], GOLD["cycle_v2"]
    b1 = cov_bytes(1, v1["itn_cov_cp"], v1["n_unk"])
    b2 = cov_bytes(2, v2["itn_cov_cp"], v2["n_cov_indexes"])
    assert round(b1 / 1e9, 1) == v1["printed_gb"]
    assert round(b2 / 1e9, 1) == v2["printed_gb"]
    tot = GOLD["total_over_run"]
    cycles = tot["n_iter"] // v1["itn_cov_cp"]
    assert round(b1 * cycles / 1e12) == tot["printed_tb_v1"]
    assert round(b2 * cycles / 1e12) == tot["printed_tb_v2"]
    assert cov_bytes(0, 1, 1) == -1 and cov_bytes(1, -1, 1) == -1


def test_counts():
    n = GOLD["n_cov_full"]["n_unk"]
    assert abs(n * (n - 1) // 2 - GOLD["n_cov_full"]["printed"]) / GOLD["n_cov_full"]["printed"] < 0.01
    d = GOLD["dense_matrix"]
    assert round(d["rows"] * d["per_row"] * 8 / 1e12) == d["printed_tb"]
    # the 4,000 selected unknowns of the large workload give the paper's ~8e6 covariance threshold (Sec. 3)
    assert 4000 * 3999 // 2 == 7_998_000
