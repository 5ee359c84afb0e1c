"""gsr_aprod1_noalloc (aprod 1 with its workspace in the library's static device
scratch) against gsr_aprod1 on the same handle and inputs, through the C
interface: two calls in a row, the second on a smaller system, so the second
runs over what the first left in the shared scratch.  The kernels are the
same, so the outputs must agree bit for bit; the oracle's aprod 1 (Eq. 2)
is held to the 1e-13 normwise product bar as well."""
import ctypes as C

import numpy as np
import pytest
import torch

import gsr_synth

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _case(oracle_lib, stars, obs, n_att, n_instr, seed, scale):
    import paper_2503_22863_amd as gsr

    print(f"[no-alloc] {stars} stars x {obs} obs, n_att={n_att}, scale={scale}", flush=True)
    g = gsr_synth.make_system(stars, obs, n_att, n_instr, 1, seed=seed)
    S = gsr.System.from_generated(g, device="cuda:0")
    rng = np.random.default_rng(seed + 1)
    x = rng.standard_normal(g.dims.n)
    y0 = rng.standard_normal(g.dims.m)
    xd = torch.from_numpy(x).cuda()
    y_ref_gpu = torch.from_numpy(y0).cuda()
    y_na = torch.from_numpy(y0).cuda()
    L = gsr.lib()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.gsr_aprod1_noalloc(S._h, C.c_void_p(xd.data_ptr()), C.c_void_p(y_na.data_ptr()), C.c_double(scale),
                              gsr.PROD_F64, st)
    assert rc == 0, L.gsr_last_error()
    rc = L.gsr_aprod1(S._h, C.c_void_p(xd.data_ptr()), C.c_void_p(y_ref_gpu.data_ptr()), C.c_double(scale),
                      gsr.PROD_F64, st)
    assert rc == 0, L.gsr_last_error()
    torch.cuda.synchronize()
    a, b = y_na.cpu().numpy(), y_ref_gpu.cpu().numpy()
    assert np.array_equal(a, b), np.abs(a - b).max()
    o = oracle_lib.OSystem(g)
    ref = oracle_lib.aprod1(o, x, y=y0, scale=scale)
    e = _rel(a, ref)
    print(f"  equal to gsr_aprod1; vs oracle {e:.2e}", flush=True)
    assert e <= 1e-13
    S.close()


def test_noalloc_aprod1_two_calls(oracle_lib):
    torch.cuda.set_device(0)
    _case(oracle_lib, 400, 50, 6000, 40, seed=71, scale=0.5)
    _case(oracle_lib, 120, 20, 64, 16, seed=72, scale=1.0)


def test_noalloc_rejects_too_large_attitude_block():
    import paper_2503_22863_amd as gsr

    g = gsr_synth.make_system(4, 8, 180000, 8, 1, seed=5)
    S = gsr.System.from_generated(g, device="cuda:0")
    x = torch.zeros(g.dims.n, dtype=torch.float64, device="cuda:0")
    y = torch.zeros(g.dims.m, dtype=torch.float64, device="cuda:0")
    with pytest.raises(gsr.GsrError, match="scratch"):
        S.aprod1_noalloc(x, y)
    S.close()
