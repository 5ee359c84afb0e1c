"""Parity of the HIP products (Eq. 2 and Eq. 3) with the CPU oracle.

Bar: relative 1e-13, normwise per block (astrometric, attitude,
instrumental, global) and overall, for FP64; FP32-product mode against the
oracle's FP32-product emulation at the same bar (the products are identical
bit for bit, only the FP64 summation order differs)."""
import numpy as np
import pytest
import torch

import gsr_synth

pytestmark = pytest.mark.gpu

CASES = {
    "small": dict(n_stars=40, obs=12, n_att=16, n_instr=8, n_glob=1, seed=7),
    "ragged_noglob": dict(n_stars=57, obs=(1, 150), n_att=9, n_instr=6, n_glob=0, seed=8),
    "empty_stars": dict(n_stars=300, obs=(0, 4), n_att=40, n_instr=12, n_glob=1, seed=9),
    "tiny_1000x20": dict(n_stars=1000, obs=20, n_att=64, n_instr=32, n_glob=1, seed=2503),
    "wide_attitude": dict(n_stars=3000, obs=(50, 90), n_att=2500, n_instr=200, n_glob=1, seed=10),
    "one_star": dict(n_stars=1, obs=300, n_att=4, n_instr=6, n_glob=1, seed=11),
    "att_buckets_small": dict(n_stars=20, obs=(0, 50), n_att=1000, n_instr=6, n_glob=0, seed=12),
    "att_buckets_many_chunks": dict(n_stars=700, obs=(40, 100), n_att=800, n_instr=40, n_glob=1, seed=13),
}


def _blocks(d):
    na = d.n_astro
    nt = na + 3 * d.n_att
    ni = nt + d.n_instr
    out = {"astro": slice(0, na), "att": slice(na, nt), "instr": slice(nt, ni), "all": slice(0, d.n)}
    if d.n_glob:
        out["glob"] = slice(ni, ni + 1)
    return out


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _assert_blocks(got, ref, d, tol):
    for name, sl in _blocks(d).items():
        if ref[sl].size == 0:
            continue
        e = _rel(got[sl], ref[sl])
        assert e <= tol, f"{name}: {e:.3e} > {tol:.0e}"


@pytest.fixture(scope="module")
def dev():
    import paper_2503_22863_amd as gsr

    assert torch.cuda.is_available()
    gsr.lib()
    return gsr


@pytest.mark.parametrize("tuning", [(32, 0), (8, 0), (32, 1)])
@pytest.mark.parametrize("case", list(CASES))
def test_aprod_fp64(dev, oracle_lib, case, tuning):
    print(f"[aprod fp64] case={case} tuning={tuning}", flush=True)
    g = gsr_synth.make_system(**CASES[case])
    o = oracle_lib.OSystem(g)
    S = dev.System.from_generated(g)
    S.set_tuning(*tuning)
    d = g.dims
    rng = np.random.default_rng(1)
    x = rng.standard_normal(d.n)
    y0 = rng.standard_normal(d.m)
    xt = torch.from_numpy(x).cuda()
    # y <- A x ; y <- -0.5 y + A x
    y = S.aprod1(xt).cpu().numpy()
    ref = oracle_lib.aprod1(o, x)
    if d.m:
        assert _rel(y, ref) <= 1e-13
    yt = torch.from_numpy(y0).cuda()
    S.aprod1(xt, yt, scale=-0.5)
    if d.m:
        assert _rel(yt.cpu().numpy(), oracle_lib.aprod1(o, x, y=y0, scale=-0.5)) <= 1e-13
    # x <- A^T y ; x <- 2 x + A^T y
    u = rng.standard_normal(d.m)
    ut = torch.from_numpy(u).cuda()
    _assert_blocks(S.aprod2(ut).cpu().numpy(), oracle_lib.aprod2(o, u), d, 1e-13)
    x2 = torch.from_numpy(x).cuda()
    S.aprod2(ut, x2, scale=2.0)
    _assert_blocks(x2.cpu().numpy(), oracle_lib.aprod2(o, u, x=x, scale=2.0), d, 1e-13)
    torch.cuda.synchronize()
    S.close()


def test_scale_zero_ignores_output_contents(dev):
    print("[aprod] scale=0 with NaN outputs", flush=True)
    g = gsr_synth.make_system(**CASES["small"])
    S = dev.System.from_generated(g)
    x = torch.ones(g.dims.n, dtype=torch.float64, device="cuda")
    y = torch.full((g.dims.m,), float("nan"), dtype=torch.float64, device="cuda")
    S.aprod1(x, y, scale=0.0)
    assert torch.isfinite(y).all()
    z = torch.full((g.dims.n,), float("nan"), dtype=torch.float64, device="cuda")
    S.aprod2(torch.ones(g.dims.m, dtype=torch.float64, device="cuda"), z, scale=0.0)
    assert torch.isfinite(z).all()
    S.close()


@pytest.mark.parametrize("case", ["small", "tiny_1000x20", "wide_attitude"])
def test_aprod_fp32_storage(dev, oracle_lib, case):
    print(f"[aprod fp32] case={case}", flush=True)
    g = gsr_synth.make_system(**CASES[case]).as_f32()
    o = oracle_lib.OSystem(g)
    S = dev.System.from_generated(g)
    d = g.dims
    rng = np.random.default_rng(2)
    x = rng.standard_normal(d.n)
    u = rng.standard_normal(d.m)
    xt, ut = torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda()
    for prod, mode in (("f32", oracle_lib.P32), ("f64", oracle_lib.P64)):
        assert _rel(S.aprod1(xt, product=prod).cpu().numpy(), oracle_lib.aprod1(o, x, mode=mode)) <= 1e-13
        _assert_blocks(S.aprod2(ut, product=prod).cpu().numpy(), oracle_lib.aprod2(o, u, mode=mode), d, 1e-13)
    S.close()


def test_fp32_products_refused_on_fp64_system(dev):
    g = gsr_synth.make_system(**CASES["small"])
    S = dev.System.from_generated(g)
    with pytest.raises(dev.GsrError):
        S.aprod1(torch.ones(g.dims.n, dtype=torch.float64, device="cuda"), product="f32")
    S.close()


def test_column_scale(dev, oracle_lib):
    print("[column scale]", flush=True)
    g = gsr_synth.make_system(**CASES["empty_stars"])
    o = oracle_lib.OSystem(g)
    S = dev.System.from_generated(g)
    got = S.column_scale().cpu().numpy()
    nrm = oracle_lib.colnorms(o)
    ref = np.where(nrm > 0, 1.0 / np.where(nrm > 0, nrm, 1.0), 1.0)
    assert _rel(got, ref) <= 1e-14
    assert np.all(got[nrm == 0] == 1.0)
    S.close()


def test_atomic_order_spread(dev, oracle_lib):
    """Attitude / instrumental / global sums use atomics: repeated runs agree to the bar."""
    print("[aprod2 repeat spread]", flush=True)
    g = gsr_synth.make_system(**CASES["wide_attitude"])
    o = oracle_lib.OSystem(g)
    S = dev.System.from_generated(g)
    u = np.random.default_rng(3).standard_normal(g.dims.m)
    ut = torch.from_numpy(u).cuda()
    ref = oracle_lib.aprod2(o, u)
    outs = [S.aprod2(ut).cpu().numpy() for _ in range(10)]
    for z in outs:
        _assert_blocks(z, ref, g.dims, 1e-13)
    spread = max(_rel(z, outs[0]) for z in outs)
    print(f"  run-to-run spread {spread:.2e}", flush=True)
    assert spread <= 1e-14
    S.close()


def test_invalid_index_data_is_rejected(dev):
    g = gsr_synth.make_system(**CASES["small"])
    bad_att = g.att_start.copy()
    bad_att[17] = g.dims.n_att - 3  # start + 3 would leave the axis
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    with pytest.raises(dev.GsrError, match="row 17"):
        dev.System(t(g.vals), t(g.star_row_ptr), t(bad_att), t(g.instr_col), g.dims.n_att, g.dims.n_instr, 1)
    bad_ic = g.instr_col.copy()
    bad_ic[5, 2] = g.dims.n_instr
    with pytest.raises(dev.GsrError, match="row 5"):
        dev.System(t(g.vals), t(g.star_row_ptr), t(g.att_start), t(bad_ic), g.dims.n_att, g.dims.n_instr, 1)
    bad_rp = g.star_row_ptr.copy()
    bad_rp[3], bad_rp[4] = bad_rp[4], bad_rp[3]
    with pytest.raises(dev.GsrError, match="star"):
        dev.System(t(g.vals), t(bad_rp), t(g.att_start), t(g.instr_col), g.dims.n_att, g.dims.n_instr, 1)
    with pytest.raises(dev.GsrError, match="device pointer"):
        dev.System(torch.from_numpy(g.vals), t(g.star_row_ptr), t(g.att_start), t(g.instr_col), g.dims.n_att,
                   g.dims.n_instr, 1)
