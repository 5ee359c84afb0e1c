"""Parity at the full one-GPU share (10^6 stars x U[50,90] observations, m ~ 7.0e7,
n = 5,120,201), in the launch configuration bench.py times: rows placed by the
caller in the regrouped order (no library copy of A), one-pass iteration, graph
replay.

The oracle runs the whole share on the host CPU (a few seconds per product), so
every output is compared, not a sample:
  * the standalone products on rows in star order and on the packed rows, and
    the iteration's one-pass product (gsr_aprod12), at the 1e-13 normwise bar
    per block and element by element at 64 eps of the absolute-value sums
    (tests/_checks.py);
  * five column-scaled LSQR iterations and two unscaled ones, x and the
    variances per block at max(1e-13, 10 s), s the oracle's own response to
    last-bit perturbations;
  * the FP32 forms bench.py times, on FP32 values placed by the caller: the
    one-pass product with FP32 products against the oracle's FP32-product
    emulation and with FP64 products (exact upcasts) against the plain oracle,
    at the same bars, and five column-scaled LSQR iterations with FP32
    products against the oracle's one-pass FP32-product LSQR (the same
    operand rounded: fl32 of the unnormalised u')."""
import numpy as np
import pytest
import torch

import gsr_synth
from _checks import abs_system, blocks, check_aprod1, check_aprod2, rel, sensitivity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def share(oracle_lib):
    import paper_2503_22863_amd as gsr

    print("[full] generating the 10^6-star share", flush=True)
    g = gsr_synth.share_1m()
    o = oracle_lib.OSystem(g)
    oa = abs_system(oracle_lib, g)
    print("[full] packing the rows in the regrouped order", flush=True)
    S = gsr.System.packed_from_generated(g)
    yield g, o, oa, S
    S.close()


@pytest.mark.timeout(600)
def test_full_share_star_order_products(oracle_lib, share):
    """gsr_aprod1 / gsr_aprod2 on the caller's rows in star order (gsr_create)."""
    import paper_2503_22863_amd as gsr

    g, o, oa, _ = share
    d = g.dims
    rng = np.random.default_rng(41)
    x, y = rng.standard_normal(d.n), rng.standard_normal(d.m)
    S = gsr.System.from_generated(g)
    print("[full] star-order aprod 1 / aprod 2 on the GPU", flush=True)
    y_gpu = S.aprod1(torch.from_numpy(x).cuda()).cpu().numpy()
    x_gpu = S.aprod2(torch.from_numpy(y).cuda()).cpu().numpy()
    S.close()
    check_aprod1(oracle_lib, o, oa, x, np.zeros(d.m), 0.0, y_gpu, "star order")
    check_aprod2(oracle_lib, g, o, oa, y, np.zeros(d.n), 0.0, x_gpu, "star order")


@pytest.mark.timeout(600)
def test_full_share_one_pass_product(oracle_lib, share):
    """The iteration's row pass (k_fblk + segment reduction + tail) with plain
    vectors: u' = s_u u + A v, x' = s_x x + A^T u'."""
    g, o, oa, S = share
    d = g.dims
    rng = np.random.default_rng(43)
    v, u0, x0 = rng.standard_normal(d.n), rng.standard_normal(d.m), rng.standard_normal(d.n)
    su, sx = -0.7, -1.1
    u = torch.from_numpy(u0).cuda()
    xg = torch.from_numpy(x0).cuda()
    print("[full] one-pass product on the packed rows", flush=True)
    S.aprod12(torch.from_numpy(v).cuda(), u, xg, scale_u=su, scale_x=sx)
    u_gpu, x_gpu = u.cpu().numpy(), xg.cpu().numpy()
    del u, xg
    u_ref = check_aprod1(oracle_lib, o, oa, v, u0, su, u_gpu, "one pass")
    check_aprod2(oracle_lib, g, o, oa, u_gpu, x0, sx, x_gpu, "one pass (on the GPU's u')")
    x_ref = oracle_lib.aprod2(o, u_ref, x=x0, scale=sx)
    for name, sl in blocks(d).items():
        e = rel(x_gpu[sl], x_ref[sl])
        print(f"  chain {name} {e:.2e}", flush=True)
        assert e <= 1e-13, name


@pytest.mark.timeout(600)
def test_full_share_packed_products(oracle_lib, share):
    """gsr_aprod1 / gsr_aprod2 on the packed rows (the regrouped pass)."""
    g, o, oa, S = share
    d = g.dims
    rng = np.random.default_rng(47)
    x, y0 = rng.standard_normal(d.n), rng.standard_normal(d.m)
    y = torch.from_numpy(y0).cuda()
    S.aprod1(torch.from_numpy(x).cuda(), y, scale=0.5)
    check_aprod1(oracle_lib, o, oa, x, y0, 0.5, y.cpu().numpy(), "packed")
    x_gpu = S.aprod2(torch.from_numpy(y0).cuda()).cpu().numpy()
    check_aprod2(oracle_lib, g, o, oa, y0, np.zeros(d.n), 0.0, x_gpu, "packed")


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precond,it", [(True, 5), (False, 2)])
def test_full_share_lsqr_iterations(oracle_lib, share, precond, it):
    """LSQR iterates at the full share.  Column-scaled for 5 iterations; unscaled
    only for 2: unscaled, the long instrumental and global column sums (2e6 and
    7e7 terms) make the iterates past the second depend on the summation order
    of FP64 sums themselves, which the compensated oracle does not share (every
    GPU form, the paper's separate products included, sits 2e-10 from it in the
    global unknown at the third iteration, 6e-7 at the fifth), while perturbing
    the data leaves the oracle within 1e-13."""
    g, o, oa, S = share
    d = g.dims
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    print(f"[full] {it} LSQR iterations on the GPU (packed rows, graphs), precond={precond}", flush=True)
    x, var, r = S.lsqr_solve(torch.from_numpy(b).cuda(), atol=0, btol=0, itmax=it, precond=precond)
    assert r["itn"] == it
    print(f"[full] {it} oracle LSQR iterations, and three with last-bit perturbations", flush=True)
    ref, sens = sensitivity(oracle_lib, g, o, b, atol=0, btol=0, itmax=it, precond=precond)
    x, var = x.cpu().numpy(), var.cpu().numpy()
    for name, sl in blocks(d).items():
        ex, ev = rel(x[sl], ref["x"][sl]), rel(var[sl], ref["var"][sl])
        bx, bv = max(1e-13, 10 * sens[("x", name)]), max(1e-13, 10 * sens[("var", name)])
        print(f"  {name}: x {ex:.2e} (bar {bx:.1e}) var {ev:.2e} (bar {bv:.1e})", flush=True)
        assert ex <= bx and ev <= bv, name
    for k in ("rnorm", "anorm", "xnorm"):
        assert abs(r[k] - ref[k]) <= max(1e-13, 10 * sens[k]) * abs(ref[k]), k
    info = S.blocked_info()
    assert info["active"] == 1 and info["values_owned"] == 0  # the configuration bench.py times


@pytest.fixture(scope="module")
def share32(oracle_lib, share):
    import paper_2503_22863_amd as gsr

    g = share[0].as_f32()
    print("[full fp32] packing the FP32 rows in the regrouped order", flush=True)
    S = gsr.System.packed_from_generated(g)
    yield g, oracle_lib.OSystem(g), abs_system(oracle_lib, g), S
    S.close()


@pytest.mark.timeout(600)
def test_full_share_fp32_one_pass_product(oracle_lib, share32):
    """FP32 values: u' = s_u u + A v and x' = A^T u' in one pass, with FP32 products
    (each formed in FP32 from fl32 operands, sums in FP64) and with FP64 products."""
    g, o, oa, S = share32
    d = g.dims
    rng = np.random.default_rng(59)
    v, u0 = rng.standard_normal(d.n), rng.standard_normal(d.m)
    for product, mode in (("f32", oracle_lib.P32), ("f64", oracle_lib.P64)):
        print(f"[full fp32] one-pass product, {product} products", flush=True)
        u = torch.from_numpy(u0).cuda()
        _, xg = S.aprod12(torch.from_numpy(v).cuda(), u, scale_u=-0.5, product=product)
        u_gpu, x_gpu = u.cpu().numpy(), xg.cpu().numpy()
        del u, xg
        check_aprod1(oracle_lib, o, oa, v, u0, -0.5, u_gpu, f"{product} products", mode=mode)
        check_aprod2(oracle_lib, g, o, oa, u_gpu, np.zeros(d.n), 0.0, x_gpu,
                     f"{product} products (on the GPU's u')", mode=mode)


@pytest.mark.timeout(900)
def test_full_share_fp32_lsqr_iterations(oracle_lib, share32):
    """Five column-scaled LSQR iterations with FP32 products (the inner solves of
    the refinement bench.py times) against the oracle's one-pass FP32-product LSQR."""
    g, o, _, S = share32
    d = g.dims
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    it = 5
    print(f"[full fp32] {it} LSQR iterations with FP32 products on the GPU", flush=True)
    x, var, r = S.lsqr_solve(torch.from_numpy(b).cuda(), atol=0, btol=0, itmax=it, precond=True, product="f32")
    assert r["itn"] == it
    print(f"[full fp32] {it} oracle LSQR iterations (one-pass FP32 products), and six with b perturbed",
          flush=True)
    ref, sens = sensitivity(oracle_lib, g, o, b, nruns_b=6, atol=0, btol=0, itmax=it, precond=True,
                            mode=oracle_lib.P32_1P)
    x, var = x.cpu().numpy(), var.cpu().numpy()
    for name, sl in blocks(d).items():
        ex, ev = rel(x[sl], ref["x"][sl]), rel(var[sl], ref["var"][sl])
        bx, bv = max(1e-13, 10 * sens[("x", name)]), max(1e-13, 10 * sens[("var", name)])
        print(f"  {name}: x {ex:.2e} (bar {bx:.1e}) var {ev:.2e} (bar {bv:.1e})", flush=True)
        assert ex <= bx and ev <= bv, name
