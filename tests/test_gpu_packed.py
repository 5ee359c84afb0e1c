"""Handles over rows the caller placed in the regrouped order (gsr_layout_plan /
gsr_layout_pack / gsr_create_packed: no library copy of A) against the oracle.

Products (Eq. 2 and Eq. 3) are held to the 1e-13 normwise bar per block and,
element by element, to 64 eps times the same sum over absolute values
(|A| |v| + |s| |u| for aprod 1, |A|^T |u| + |s| |x| for aprod 2, computed by
the oracle on |coefficients|): a wrong index at one window, segment or tile
boundary moves single elements far beyond that, whatever the norms do.  The
one-pass product gsr_aprod12 -- the LSQR iteration's own row pass with plain
vectors -- is checked the same way, its A^T part against the oracle's A^T
applied to the GPU's u' (which isolates that half) and the chain as a whole
against the oracle's two products.  LSQR solves on packed rows meet the bars
of the regrouped copy (the oracle's own response to last-bit perturbations)."""
import copy

import numpy as np
import pytest
import torch

import gsr_synth
from _checks import abs_system, blocks, check_aprod1 as _check_aprod1, check_aprod2, rel

pytestmark = pytest.mark.gpu

_rel, _blocks, _abs_system = rel, blocks, abs_system


def check_aprod1(oracle_lib, g, o, oa, x, y0, scale, y_gpu, tag):
    return _check_aprod1(oracle_lib, o, oa, x, y0, scale, y_gpu, tag)


@pytest.fixture(scope="module")
def dev():
    import paper_2503_22863_amd as gsr

    gsr.lib()
    return gsr


CASES = {
    # 25 windows of 40 starts, ragged tail (m not a multiple of 64)
    "many_windows": dict(n_stars=300, obs=(20, 40), n_att=1000, n_instr=16, seed=61, maxw=40),
    # one window; attitude block small enough for LDS too
    "one_window": dict(n_stars=200, obs=(10, 30), n_att=300, n_instr=10, seed=62, maxw=0),
    # stars of 0 to 6 rows: empty stars, tiles spanning many stars
    "short_stars": dict(n_stars=3000, obs=(0, 6), n_att=800, n_instr=12, seed=63, maxw=100),
    # stars of 300 to 600 rows: segments over many tiles and wave ranges
    "long_stars": dict(n_stars=20, obs=(300, 600), n_att=700, n_instr=16, seed=64, maxw=0),
}


def _make(dev, c, value_dtype=None, chunk_rows=1 << 22):
    g = gsr_synth.make_system(c["n_stars"], c["obs"], c["n_att"], c["n_instr"], 1, seed=c["seed"])
    if value_dtype is not None:
        g = copy.copy(g)
        g.vals = g.vals.astype(value_dtype)
    S = dev.System.packed_from_generated(g, device="cuda:0", max_window=c["maxw"], chunk_rows=chunk_rows)
    return g, S


@pytest.mark.parametrize("case", list(CASES))
def test_packed_products_match_oracle(dev, oracle_lib, case):
    c = CASES[case]
    print(f"[packed] products {case}", flush=True)
    g, S = _make(dev, c, chunk_rows=1000)  # several pack calls
    info = S.blocked_info()
    print(f"  layout {info}", flush=True)
    assert info["active"] == 1 and info["values_owned"] == 0
    assert info["value_bytes"] == info["padded_rows"] * 24 * 8
    if c["maxw"]:
        assert info["blocks"] >= 2
    o, oa = oracle_lib.OSystem(g), _abs_system(oracle_lib, g)
    rng = np.random.default_rng(c["seed"] + 100)
    d = g.dims
    x = rng.standard_normal(d.n)
    y0 = rng.standard_normal(d.m)
    x0 = rng.standard_normal(d.n)
    # aprod 1 with and without the scaled old vector
    for scale in (0.0, -0.75):
        y = torch.from_numpy(y0).cuda()
        S.aprod1(torch.from_numpy(x).cuda(), y, scale=scale)
        check_aprod1(oracle_lib, g, o, oa, x, y0, scale, y.cpu().numpy(), f"scale={scale}")
    for scale in (0.0, 1.5):
        xg = torch.from_numpy(x0).cuda()
        S.aprod2(torch.from_numpy(y0).cuda(), xg, scale=scale)
        check_aprod2(oracle_lib, g, o, oa, y0, x0, scale, xg.cpu().numpy(), f"scale={scale}")
    # column scaling from the square mode of the pass
    sc = S.column_scale().cpu().numpy()
    ref = oracle_lib.colnorms(o)
    want = np.where(ref > 0, 1.0 / np.where(ref > 0, ref, 1.0), 1.0)
    e = _rel(sc, want)
    print(f"  column scale {e:.2e}", flush=True)
    assert e <= 1e-14
    S.close()


@pytest.mark.parametrize("case", list(CASES))
def test_one_pass_product_matches_oracle(dev, oracle_lib, case):
    """gsr_aprod12: u' = s_u u + A v, then x' = s_x x + A^T u'."""
    c = CASES[case]
    print(f"[packed] one-pass product {case}", flush=True)
    g, S = _make(dev, c)
    o, oa = oracle_lib.OSystem(g), _abs_system(oracle_lib, g)
    d = g.dims
    rng = np.random.default_rng(c["seed"] + 200)
    v, u0, x0 = rng.standard_normal(d.n), rng.standard_normal(d.m), rng.standard_normal(d.n)
    su, sx = -0.6, -1.3
    u = torch.from_numpy(u0).cuda()
    xg = torch.from_numpy(x0).cuda()
    S.aprod12(torch.from_numpy(v).cuda(), u, xg, scale_u=su, scale_x=sx)
    u_gpu, x_gpu = u.cpu().numpy(), xg.cpu().numpy()
    u_ref = check_aprod1(oracle_lib, g, o, oa, v, u0, su, u_gpu, "aprod12")
    # the A^T half on the GPU's own u'
    check_aprod2(oracle_lib, g, o, oa, u_gpu, x0, sx, x_gpu, "aprod12 (on the GPU's u')")
    # the whole chain against the oracle's two products
    x_ref = oracle_lib.aprod2(o, u_ref, x=x0, scale=sx)
    for name, sl in _blocks(d).items():
        assert _rel(x_gpu[sl], x_ref[sl]) <= 1e-13, name
    S.close()


def test_one_pass_product_on_a_star_order_handle(dev, oracle_lib):
    """gsr_aprod12 on a handle from gsr_create runs the same pass on the library's copy."""
    c = CASES["many_windows"]
    g = gsr_synth.make_system(c["n_stars"], c["obs"], c["n_att"], c["n_instr"], 1, seed=c["seed"])
    S = dev.System.from_generated(g, device="cuda:0")
    S.set_blocked(True, c["maxw"])
    o, oa = oracle_lib.OSystem(g), _abs_system(oracle_lib, g)
    rng = np.random.default_rng(7)
    v, u0 = rng.standard_normal(g.dims.n), rng.standard_normal(g.dims.m)
    u = torch.from_numpy(u0).cuda()
    _, xg = S.aprod12(torch.from_numpy(v).cuda(), u, scale_u=1.0)
    check_aprod1(oracle_lib, g, o, oa, v, u0, 1.0, u.cpu().numpy(), "star-order handle")
    check_aprod2(oracle_lib, g, o, oa, u.cpu().numpy(), np.zeros(g.dims.n), 0.0, xg.cpu().numpy(),
                 "star-order handle")
    assert S.blocked_info()["values_owned"] == 1
    S.close()


def test_fp32_packed_products(dev, oracle_lib):
    """FP32 coefficients: FP64 products are exact upcasts (the FP64 bars hold); FP32
    products match the oracle's FP32-product emulation."""
    c = CASES["many_windows"]
    g, S = _make(dev, c, value_dtype=np.float32)
    assert S.blocked_info()["value_bytes"] == S.blocked_info()["padded_rows"] * 24 * 4
    o, oa = oracle_lib.OSystem(g), _abs_system(oracle_lib, g)
    rng = np.random.default_rng(9)
    x, y0 = rng.standard_normal(g.dims.n), rng.standard_normal(g.dims.m)
    y = torch.from_numpy(y0).cuda()
    S.aprod1(torch.from_numpy(x).cuda(), y, scale=0.0)
    check_aprod1(oracle_lib, g, o, oa, x, y0, 0.0, y.cpu().numpy(), "fp32 values")
    xg = S.aprod2(torch.from_numpy(y0).cuda())
    check_aprod2(oracle_lib, g, o, oa, y0, np.zeros(g.dims.n), 0.0, xg.cpu().numpy(), "fp32 values")
    y32 = S.aprod1(torch.from_numpy(x).cuda(), product="f32").cpu().numpy()
    assert _rel(y32, oracle_lib.aprod1(o, x, mode=oracle_lib.P32)) <= 1e-13
    x32 = S.aprod2(torch.from_numpy(y0).cuda(), product="f32").cpu().numpy()
    ref32 = oracle_lib.aprod2(o, y0, mode=oracle_lib.P32)
    for name, sl in _blocks(g.dims).items():
        assert _rel(x32[sl], ref32[sl]) <= 1e-13, name
    S.close()


def _sensitivity(oracle_lib, g, o, b, **kw):
    r1 = oracle_lib.lsqr(o, b, **kw)
    runs = []
    for seed in (5, 6):
        bp = b * (1 + 2e-16 * np.random.default_rng(seed).standard_normal(b.size))
        runs.append(oracle_lib.lsqr(o, bp, **kw))
    gp = copy.copy(g)
    gp.vals = g.vals * (1 + 2.2e-16 * np.random.default_rng(7).standard_normal(g.vals.shape))
    runs.append(oracle_lib.lsqr(oracle_lib.OSystem(gp), b, **kw))
    sx = max(_rel(r["x"], r1["x"]) for r in runs)
    sv = max(_rel(r["var"], r1["var"]) for r in runs)
    return r1, sx, sv


@pytest.mark.parametrize("precond", [True, False])
@pytest.mark.parametrize("case", ["many_windows", "short_stars"])
def test_packed_lsqr_matches_oracle(dev, oracle_lib, case, precond):
    c = CASES[case]
    print(f"[packed] lsqr {case} precond={precond}", flush=True)
    g, S = _make(dev, c)
    o = oracle_lib.OSystem(g)
    bn = oracle_lib.known_terms(o, g.x_true, g.noise)
    itmax = 25 if precond else 6
    ref, sx, sv = _sensitivity(oracle_lib, g, o, bn, atol=0, btol=0, itmax=itmax, precond=precond)
    tol_x, tol_v = max(1e-12, 10 * sx), max(1e-10, 10 * sv)
    x, var, r = S.lsqr_solve(torch.from_numpy(bn).cuda(), atol=0, btol=0, itmax=itmax, precond=precond)
    assert r["itn"] == itmax
    ex, ev = _rel(x.cpu().numpy(), ref["x"]), _rel(var.cpu().numpy(), ref["var"])
    print(f"  x {ex:.2e} (bar {tol_x:.1e}) var {ev:.2e} (bar {tol_v:.1e})", flush=True)
    assert ex <= tol_x and ev <= tol_v
    S.close()


def test_packed_covariances(dev, oracle_lib):
    """Covariances of selected unknowns (Eq. 4) from a solve on packed rows."""
    c = CASES["many_windows"]
    g, S = _make(dev, c)
    o = oracle_lib.OSystem(g)
    bn = oracle_lib.known_terms(o, g.x_true, g.noise)
    sel = gsr_synth.covariance_selection(g.dims, 30, 10, 8, seed=3)
    itmax = 25
    _, _, sv = _sensitivity(oracle_lib, g, o, bn, atol=0, btol=0, itmax=itmax, precond=True)
    refc = oracle_lib.lsqr(o, bn, atol=0, btol=0, itmax=itmax, precond=True, sel=sel)
    S.cov_request(sel, block=16)
    x, var, r = S.lsqr_solve(torch.from_numpy(bn).cuda(), atol=0, btol=0, itmax=itmax, precond=True)
    Cg = S.cov_get().cpu().numpy()
    ec = _rel(Cg, refc["cov"])
    print(f"  cov {ec:.2e} (bar {max(1e-10, 10 * sv):.1e})", flush=True)
    assert ec <= max(1e-10, 10 * sv)
    np.testing.assert_array_equal(Cg, Cg.T)
    S.close()


def test_packed_converged_solve_and_warm_start(dev, oracle_lib):
    """A converged preconditioned solve from zero and from an x0 (r0 = b - A x0
    formed inside the first pass) reach the oracle's solution."""
    c = CASES["many_windows"]
    g, S = _make(dev, c)
    o = oracle_lib.OSystem(g)
    bn = oracle_lib.known_terms(o, g.x_true, g.noise)
    ref = oracle_lib.lsqr(o, bn, atol=1e-13, btol=1e-13, itmax=400, precond=True)
    x, var, r = S.lsqr_solve(torch.from_numpy(bn).cuda(), atol=1e-13, btol=1e-13, itmax=400, precond=True)
    print(f"  istop {r['istop']} itn {r['itn']} (oracle {ref['istop']}/{ref['itn']})", flush=True)
    assert r["istop"] == ref["istop"] and abs(r["itn"] - ref["itn"]) <= 1
    assert _rel(x.cpu().numpy(), ref["x"]) <= 1e-10
    x0 = ref["x"] + 0.05 * np.random.default_rng(3).standard_normal(g.dims.n)
    xw, _, rw = S.lsqr_solve(torch.from_numpy(bn).cuda(), x0=torch.from_numpy(x0).cuda(), atol=1e-13, btol=1e-13,
                             itmax=400, precond=True)
    assert _rel(xw.cpu().numpy(), ref["x"]) <= 1e-10
    S.close()


def test_packed_fp32_refinement(dev, oracle_lib):
    c = CASES["many_windows"]
    g, S = _make(dev, c, value_dtype=np.float32)
    o = oracle_lib.OSystem(g)
    bn = oracle_lib.known_terms(o, g.x_true, g.noise)
    ref = oracle_lib.lsqr(o, bn, atol=1e-14, btol=1e-14, itmax=600, precond=True)
    x, r = S.lsqr_refine(torch.from_numpy(bn).cuda(), atol=1e-6, btol=1e-6, itmax=600, precond=True,
                         product="f32", outer_max=10, outer_tol=1e-11)
    e = _rel(x.cpu().numpy(), ref["x"])
    print(f"  refined {e:.2e} after {r['outer_steps']} outer steps", flush=True)
    assert e <= 1e-10
    S.close()


def test_packed_constraints(dev, oracle_lib):
    """Constraint rows under packed A (Sec. 2): the solve meets the oracle over [A; C]."""
    c = CASES["many_windows"]
    g, S = _make(dev, c)
    d = g.dims
    ptr = np.array([0, 3, 5], np.int64)
    col = np.array([0, 5, 10, d.n_astro, d.n - 1], np.int64)
    val = np.array([1.0, -2.0, 0.5, 1.0, 1.0])
    o = oracle_lib.OSystem(g, constraints=(ptr, col, val))
    bn = oracle_lib.known_terms(o, g.x_true, g.noise)
    ref = oracle_lib.lsqr(o, bn, atol=1e-13, btol=1e-13, itmax=400, precond=True)
    rhs = bn[d.m:]
    S.set_constraints(ptr, col, val, rhs)
    x, var, r = S.lsqr_solve(torch.from_numpy(bn[:d.m]).cuda(), atol=1e-13, btol=1e-13, itmax=400, precond=True)
    assert _rel(x.cpu().numpy(), ref["x"]) <= 1e-10
    S.close()


def test_packed_handle_refusals_and_layout_reuse(dev):
    """What a packed handle refuses (star-order passes), and that a consumed layout
    cannot be used again while an unconsumed one is destroyed cleanly."""
    c = CASES["one_window"]
    g = gsr_synth.make_system(c["n_stars"], c["obs"], c["n_att"], c["n_instr"], 1, seed=c["seed"])
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    L = dev.Layout(t(g.star_row_ptr), t(g.att_start), t(g.instr_col), g.dims.n_att, g.dims.n_instr, 1)
    packed = L.new_buffer()
    L.pack(t(g.vals), 0, packed)
    with pytest.raises(dev.GsrError):
        L.pack(t(g.vals[:10]), g.dims.m - 5, packed)  # past the last row
    h = L._h
    S = dev.System.from_packed(L, packed)
    assert L._h is None
    import ctypes as C

    assert dev.lib().gsr_layout_pack(h, C.c_void_p(packed.data_ptr()), 0, 1, C.c_void_p(packed.data_ptr()),
                                     None) != 0  # consumed
    with pytest.raises(dev.GsrError):
        S.set_fused(False)
    with pytest.raises(dev.GsrError):
        S.set_blocked(True, 40)
    x = torch.zeros(S.n, dtype=torch.float64, device="cuda:0")
    y = torch.zeros(S.m, dtype=torch.float64, device="cuda:0")
    with pytest.raises(dev.GsrError):
        S.aprod1_noalloc(x, y)
    with pytest.raises(dev.GsrError):
        S.features(y, x[5 * S.n_stars:])
    S.close()
    L2 = dev.Layout(t(g.star_row_ptr), t(g.att_start), t(g.instr_col), g.dims.n_att, g.dims.n_instr, 1)
    L2.close()
    bad = g.att_start.copy()
    bad[17] = g.dims.n_att  # start past n_att - 4
    with pytest.raises(dev.GsrError, match="row 17"):
        dev.Layout(t(g.star_row_ptr), t(bad), t(g.instr_col), g.dims.n_att, g.dims.n_instr, 1)


def test_packed_rows_in_any_chunk_order_give_the_same_products(dev, oracle_lib):
    """gsr_layout_pack places rows wherever they come from: chunks of 777 rows in
    reverse order give the same buffer, bit for bit, as one call over all rows."""
    c = CASES["many_windows"]
    g = gsr_synth.make_system(c["n_stars"], c["obs"], c["n_att"], c["n_instr"], 1, seed=c["seed"])
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    bufs = []
    for order in ("whole", "reversed"):
        L = dev.Layout(t(g.star_row_ptr), t(g.att_start), t(g.instr_col), g.dims.n_att, g.dims.n_instr, 1,
                       max_window=c["maxw"])
        P = L.new_buffer()
        P.fill_(7.0)
        if order == "whole":
            L.pack(t(g.vals), 0, P)
        else:
            starts = list(range(0, g.dims.m, 777))[::-1]
            for r0 in starts:
                L.pack(t(g.vals[r0:r0 + 777]), r0, P)
        S = dev.System.from_packed(L, P)  # zeroes the padding rows
        bufs.append(P.cpu().numpy())
        S.close()
    assert np.array_equal(bufs[0], bufs[1])
    # every coefficient appears once, the padding rows are zero
    assert np.isclose(np.abs(bufs[0]).sum(), np.abs(g.vals).sum(), rtol=1e-12)
    assert np.count_nonzero(bufs[0]) == np.count_nonzero(g.vals)


def test_packed_covariance_export_and_pairs(dev, oracle_lib):
    """Covariance pipeline versions 1 (export of whole d_i blocks) and 2 (index pairs)
    on packed rows, against the oracle's stored direction vectors."""
    c = CASES["many_windows"]
    g, S = _make(dev, c)
    o = oracle_lib.OSystem(g)
    bn = oracle_lib.known_terms(o, g.x_true, g.noise)
    itmax, block = 20, 8
    d = g.dims
    rng = np.random.default_rng(17)
    pairs = np.stack([rng.integers(0, d.n, 40), rng.integers(0, d.n, 40)], axis=1)
    U, inv = np.unique(pairs.reshape(-1), return_inverse=True)
    inv = inv.reshape(-1, 2)
    ref = oracle_lib.lsqr(o, bn, atol=0, btol=0, itmax=itmax, precond=True, sel=U)
    host = torch.zeros((itmax // block + 2, block, d.n), dtype=torch.float64).pin_memory()
    S.cov_export(host, block)
    S.cov_request_pairs(pairs, block=block)
    x, var, r = S.lsqr_solve(torch.from_numpy(bn).cuda(), atol=0, btol=0, itmax=itmax, precond=True)
    nb, lc = S.cov_export_status()
    assert (nb - 1) * block + lc == itmax
    D = host.numpy()[:nb].reshape(-1, d.n)[:itmax]
    ed = _rel(D[:, U], ref["dsel"])
    Cref = oracle_lib.covariances(ref["dsel"], ref["scale"][U])[inv[:, 0], inv[:, 1]]
    ep = _rel(S.cov_get_pairs().cpu().numpy(), Cref)
    print(f"  exported d_i {ed:.2e}  pair covariances {ep:.2e}", flush=True)
    assert ed <= 1e-10 and ep <= 1e-10
    S.cov_export(None)
    S.cov_request_pairs([], block=64)
    S.close()


def _with_empty_stars(g, at, gap):
    """The same rows, with `gap` stars that have no rows inserted before star `at`."""
    rp = g.star_row_ptr
    rp2 = np.concatenate([rp[:at + 1], np.full(gap, rp[at], dtype=rp.dtype), rp[at + 1:]])
    xt = np.concatenate([g.x_true[:5 * at], np.zeros(5 * gap), g.x_true[5 * at:]])
    d = gsr_synth.Dims(g.dims.n_stars + gap, g.dims.m, g.dims.n_att, g.dims.n_instr, g.dims.n_glob)
    return gsr_synth.System(d, g.vals, rp2, g.att_start, g.instr_col, xt, g.noise, g.seed, dict(g.meta))


def test_packed_star_gap_beyond_record_span(dev, oracle_lib):
    """Rows of one window whose stars lie 150,000 apart (that many stars without
    rows between them): a row record holds its star as an offset below 65,536
    from its tile's first star, so the layout starts a new tile at the gap
    (padding rows).  Products and LSQR iterates against the oracle."""
    c = CASES["many_windows"]
    g0 = gsr_synth.make_system(c["n_stars"], c["obs"], c["n_att"], c["n_instr"], 1, seed=c["seed"])
    g = _with_empty_stars(g0, c["n_stars"] // 2, 150_000)
    d = g.dims
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    pad0 = dev.Layout(t(g0.star_row_ptr), t(g0.att_start), t(g0.instr_col), d.n_att, d.n_instr, 1,
                      max_window=c["maxw"]).info()["padded_rows"]
    S = dev.System.packed_from_generated(g, device="cuda:0", max_window=c["maxw"])
    info = S.blocked_info()
    print(f"[packed] star gap: padded rows {info['padded_rows']} (without the gap {pad0})", flush=True)
    assert info["padded_rows"] > pad0  # the gap closed tiles early in some windows
    o, oa = oracle_lib.OSystem(g), _abs_system(oracle_lib, g)
    rng = np.random.default_rng(67)
    x, y0 = rng.standard_normal(d.n), rng.standard_normal(d.m)
    y = t(y0)
    S.aprod1(t(x), y, scale=-0.75)
    check_aprod1(oracle_lib, g, o, oa, x, y0, -0.75, y.cpu().numpy(), "star gap")
    check_aprod2(oracle_lib, g, o, oa, y0, np.zeros(d.n), 0.0, S.aprod2(t(y0)).cpu().numpy(), "star gap")
    bn = oracle_lib.known_terms(o, g.x_true, g.noise)
    ref, sx, sv = _sensitivity(oracle_lib, g, o, bn, atol=0, btol=0, itmax=25, precond=True)
    tol_x, tol_v = max(1e-12, 10 * sx), max(1e-10, 10 * sv)
    xs, var, r = S.lsqr_solve(t(bn), atol=0, btol=0, itmax=25, precond=True)
    ex, ev = _rel(xs.cpu().numpy(), ref["x"]), _rel(var.cpu().numpy(), ref["var"])
    print(f"  x {ex:.2e} (bar {tol_x:.1e}) var {ev:.2e} (bar {tol_v:.1e})", flush=True)
    assert r["itn"] == 25 and ex <= tol_x and ev <= tol_v
    S.close()
