"""Parity at the large one-GPU share with covariances (3*10^6 stars x U[50,90]
observations, m ~ 2.1e8, n = 15,360,501; covariances of 4,000 selected unknowns)
in the launch configuration bench.py times (rows placed by the caller in the
regrouped order, graph replay).  The oracle runs the whole share on the host CPU,
so every output is compared: the iteration's one-pass product at the 1e-13
normwise bar per block and element by element at 64 eps of the absolute-value
sums, and five column-scaled LSQR iterations (x, variances per block and the
4,000 x 4,000 covariance block) at max(1e-13, 10 s), s the oracle's own
response to last-bit perturbations (tests/_checks.py; unscaled iterates at
these sizes depend on the summation order of the long instrumental and global
column sums past the second iteration)."""
import numpy as np
import pytest
import torch

import gsr_synth
from _checks import abs_system, blocks, check_aprod1, check_aprod2, rel, sensitivity

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(1200)
def test_full_share_3m(oracle_lib):
    import paper_2503_22863_amd as gsr

    print("[full 3m] generating the 3*10^6-star share", flush=True)
    g = gsr_synth.share_3m()
    d = g.dims
    k = 4000
    nst = (k * 3 // 5) // 5
    sel = gsr_synth.covariance_selection(d, nst, k * 3 // 10 // 3, k - 5 * nst - 3 * (k * 3 // 10 // 3), seed=19)
    assert sel.size == k
    o = oracle_lib.OSystem(g)
    print("[full 3m] packing the rows in the regrouped order", flush=True)
    S = gsr.System.packed_from_generated(g)
    info = S.blocked_info()
    print(f"  layout {info}", flush=True)
    assert info["active"] == 1 and info["values_owned"] == 0

    # the iteration's one-pass product with plain vectors
    rng = np.random.default_rng(53)
    v, u0 = rng.standard_normal(d.n), rng.standard_normal(d.m)
    u = torch.from_numpy(u0).cuda()
    _, xg = S.aprod12(torch.from_numpy(v).cuda(), u, scale_u=-0.5)
    u_gpu, x_gpu = u.cpu().numpy(), xg.cpu().numpy()
    del u, xg
    oa = abs_system(oracle_lib, g)
    print("[full 3m] oracle products", flush=True)
    check_aprod1(oracle_lib, o, oa, v, u0, -0.5, u_gpu, "one pass")
    check_aprod2(oracle_lib, g, o, oa, u_gpu, np.zeros(d.n), 0.0, x_gpu, "one pass (on the GPU's u')")
    del oa, u_gpu, x_gpu, u0, v

    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    it = 5
    S.cov_request(sel, block=64)
    print(f"[full 3m] {it} column-scaled LSQR iterations on the GPU", flush=True)
    x, var, r = S.lsqr_solve(torch.from_numpy(b).cuda(), atol=0, btol=0, itmax=it, precond=True)
    C = S.cov_get().cpu().numpy()
    S.close()
    assert r["itn"] == it
    print(f"[full 3m] {it} oracle LSQR iterations, and three with last-bit perturbations", flush=True)
    ref, sens = sensitivity(oracle_lib, g, o, b, atol=0, btol=0, itmax=it, precond=True, sel=sel)
    x, var = x.cpu().numpy(), var.cpu().numpy()
    for name, sl in blocks(d).items():
        ex, ev = rel(x[sl], ref["x"][sl]), rel(var[sl], ref["var"][sl])
        bx, bv = max(1e-13, 10 * sens[("x", name)]), max(1e-13, 10 * sens[("var", name)])
        print(f"  {name}: x {ex:.2e} (bar {bx:.1e}) var {ev:.2e} (bar {bv:.1e})", flush=True)
        assert ex <= bx and ev <= bv, name
    ec = rel(C, ref["cov"])
    bc = max(1e-13, 10 * sens["cov"])
    print(f"  covariances {ec:.2e} (bar {bc:.1e})", flush=True)
    assert ec <= bc
