"""Error behaviour of the C interface: bad arguments, bad index data, calls out of
order and after destroy come back as error codes with a message, never as a
device fault."""
import ctypes as C

import numpy as np
import pytest
import torch

import gsr_synth

pytestmark = pytest.mark.gpu

GSR_EINVAL, GSR_ENOMEM, GSR_EHIP, GSR_ESTATE = -1, -2, -3, -4


@pytest.fixture(scope="module")
def dev():
    import paper_2503_22863_amd as gsr

    gsr.lib()
    return gsr


@pytest.fixture(scope="module")
def small(dev):
    g = gsr_synth.make_system(30, 10, 8, 6, 1, seed=31)
    return g, dev.System.from_generated(g)


def _code(fn):
    with pytest.raises(Exception) as ei:
        fn()
    return getattr(ei.value, "code", None), str(ei.value)


def test_bad_dims_and_pointers(dev):
    L = dev.lib()
    h = C.c_void_p()
    t = torch.zeros(16, dtype=torch.float64, device="cuda")
    rp = torch.zeros(2, dtype=torch.int64, device="cuda")
    for dims in [dev.Dims(1, 0, 3, 6, 1, 0), dev.Dims(1, 0, 4, 5, 1, 0), dev.Dims(1, 0, 4, 6, 2, 0),
                 dev.Dims(-1, 0, 4, 6, 1, 0), dev.Dims(1, 0, 4, 6, 1, 7)]:
        rc = L.gsr_create(C.byref(h), C.byref(dims), C.c_void_p(t.data_ptr()), C.c_void_p(rp.data_ptr()), None, None,
                          None)
        assert rc == GSR_EINVAL
        assert L.gsr_last_error()
    assert L.gsr_create(None, C.byref(dev.Dims(1, 0, 4, 6, 1, 0)), None, None, None, None, None) == GSR_EINVAL
    # rows without the index arrays
    rc = L.gsr_create(C.byref(h), C.byref(dev.Dims(1, 4, 4, 6, 1, 0)), C.c_void_p(t.data_ptr()),
                      C.c_void_p(rp.data_ptr()), None, None, None)
    assert rc == GSR_EINVAL


def test_star_row_ptr_must_cover_rows(dev):
    g = gsr_synth.make_system(10, 5, 8, 6, 1, seed=32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    rp = g.star_row_ptr.copy()
    rp[-1] -= 1  # last star stops one row short of m
    with pytest.raises(dev.GsrError) as ei:
        dev.System(t(g.vals), t(rp), t(g.att_start), t(g.instr_col), 8, 6, 1)
    assert ei.value.code == GSR_EINVAL


def test_wrong_argument_kinds(dev, small):
    g, S = small
    host = torch.zeros(g.dims.n, dtype=torch.float64)
    with pytest.raises(dev.GsrError) as ei:
        S.aprod1(host)
    assert ei.value.code == GSR_EINVAL and "device pointer" in str(ei.value)
    with pytest.raises(dev.GsrError):
        S.lsqr_solve(torch.zeros(g.dims.m, dtype=torch.float64, device="cuda"), itmax=-1)
    with pytest.raises(dev.GsrError):
        S.lsqr_solve(torch.zeros(g.dims.m, dtype=torch.float64, device="cuda"), damp=-1.0)
    with pytest.raises(dev.GsrError):
        S.cov_request([0, g.dims.n], block=64)  # index out of range
    with pytest.raises(dev.GsrError):
        S.cov_request([0, 1], block=0)
    with pytest.raises(dev.GsrError):
        S.cov_get()  # no selection
    with pytest.raises(dev.GsrError):
        S.lsqr_refine(torch.zeros(g.dims.m, dtype=torch.float64, device="cuda"))  # FP64 system
    with pytest.raises(dev.GsrError):
        S.set_tuning(0)


def test_calls_out_of_order(dev, small):
    g, S = small
    with pytest.raises(dev.GsrError) as ei:
        S.lsqr_iterate(1)
    assert ei.value.code == GSR_ESTATE
    with pytest.raises(dev.GsrError) as ei:
        S.lsqr_end()
    assert ei.value.code == GSR_ESTATE


def test_calls_after_destroy(dev):
    g = gsr_synth.make_system(10, 5, 8, 6, 1, seed=33)
    S = dev.System.from_generated(g)
    h = S._h
    S.close()
    L = dev.lib()
    x = torch.zeros(g.dims.n, dtype=torch.float64, device="cuda")
    y = torch.zeros(g.dims.m, dtype=torch.float64, device="cuda")
    assert L.gsr_aprod1(h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), 0.0, 0, None) == GSR_EINVAL
    assert b"destroyed" in L.gsr_last_error()
    assert L.gsr_destroy(None) == 0


def test_nan_known_terms_do_not_hang(dev, small):
    g, S = small
    b = torch.full((g.dims.m,), float("nan"), dtype=torch.float64, device="cuda")
    x, _, r = S.lsqr_solve(b, itmax=20)
    # NaN propagates; the solve ends (stop tests never pass, itmax does)
    assert r["itn"] <= 20


def test_mlp_bad_sizes(dev):
    L = dev.lib()
    h = C.c_void_p()
    p = np.zeros(10)
    assert L.gsr_mlp_create(C.byref(h), 0, 4, 1, p.ctypes.data) == GSR_EINVAL
    assert L.gsr_mlp_create(C.byref(h), 2, 4, 1, None) == GSR_EINVAL
