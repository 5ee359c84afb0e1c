"""The one-pass iteration on the copy regrouped by attitude window against the
oracle: fixed-count LSQR iterates, variances and scalar estimates with one
window and with many (a capped window width: many blocks, workgroups and star
segments), stars spanning many tiles, empty and very short stars, FP32 storage
and FP32 products, covariances, and agreement with the bucketed pass on the
same handle.  The atomic LDS sums make the summation order run-dependent, so
the bars are the oracle's own response to last-bit perturbations of its data."""
import copy

import numpy as np
import pytest
import torch

import gsr_synth

pytestmark = pytest.mark.gpu


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def dev():
    import paper_2503_22863_amd as gsr

    gsr.lib()
    return gsr


def _sensitivity(oracle_lib, g, o, b, nruns=2, **kw):
    """Reference run and the largest relative deviations of x, var and the scalar
    estimates over runs with b and with A perturbed at the last bit."""
    r1 = oracle_lib.lsqr(o, b, **kw)
    runs = []
    # nruns perturbations of b (more for FP32 products, whose response is dominated by
    # rare FP32 rounding flips: a few runs can miss them)
    for seed in range(5, 5 + nruns):
        bp = b * (1 + 2e-16 * np.random.default_rng(seed).standard_normal(b.size))
        runs.append(oracle_lib.lsqr(o, bp, **kw))
    gp = copy.copy(g)
    gp.vals = g.vals * (1 + 2.2e-16 * np.random.default_rng(7).standard_normal(g.vals.shape))
    runs.append(oracle_lib.lsqr(oracle_lib.OSystem(gp), b, **kw))
    sx = max(_rel(r["x"], r1["x"]) for r in runs)
    sv = max(_rel(r["var"], r1["var"]) for r in runs)
    r1["sens"] = {k: max(abs(r[k] - r1[k]) / max(abs(r1[k]), 1e-300) for r in runs)
                  for k in ("rnorm", "anorm", "xnorm")}
    return r1, sx, sv


# tail_len = 3 n_att + n_instr + 1 > 2048 in every case: the attitude block is too
# large for LDS, so fused solves run on the regrouped copy
CASES = {
    # one window (Wb = n_att - 3)
    "one_window": dict(n_stars=300, obs=(20, 40), n_att=1000, n_instr=16, seed=31, maxw=0),
    # 25 windows of 40 starts: many blocks, workgroups per block and star segments
    "many_windows": dict(n_stars=300, obs=(20, 40), n_att=1000, n_instr=16, seed=32, maxw=40),
    # stars of 0 to 6 rows: empty stars, tiles spanning more than 12 stars
    "short_stars": dict(n_stars=3000, obs=(0, 6), n_att=800, n_instr=12, seed=33, maxw=100),
    # stars of 300 to 600 rows in one window: segments over many tiles and wave boundaries
    "long_stars": dict(n_stars=20, obs=(300, 600), n_att=700, n_instr=16, seed=34, maxw=0),
}


def _system(c):
    return gsr_synth.make_system(c["n_stars"], c["obs"], c["n_att"], c["n_instr"], 1, seed=c["seed"])


@pytest.mark.parametrize("precond", [True, False])
@pytest.mark.parametrize("case", list(CASES))
def test_blocked_lsqr_matches_oracle(dev, oracle_lib, case, precond):
    c = CASES[case]
    print(f"[blocked] {case} precond={precond}", flush=True)
    g = _system(c)
    o = oracle_lib.OSystem(g)
    bn = oracle_lib.known_terms(o, g.x_true, g.noise)
    # unscaled, these systems' iterates past a few steps depend on the summation
    # order itself, so that case stops at 6
    itmax = 25 if precond else 6
    ref, sx, sv = _sensitivity(oracle_lib, g, o, bn, atol=0, btol=0, itmax=itmax, precond=precond)
    tol_x, tol_v = max(1e-12, 10 * sx), max(1e-10, 10 * sv)
    S = dev.System.from_generated(g)
    S.set_blocked(True, c["maxw"])
    b = torch.from_numpy(bn).cuda()
    x, var, r = S.lsqr_solve(b, atol=0, btol=0, itmax=itmax, precond=precond)
    info = S.blocked_info()
    print(f"  layout {info}", flush=True)
    assert info["active"] == 1 and info["padded_rows"] % 64 == 0 and info["padded_rows"] >= g.dims.m
    if c["maxw"]:
        assert info["window"] <= c["maxw"] and info["blocks"] >= 2
    assert r["itn"] == itmax
    ex, ev = _rel(x.cpu().numpy(), ref["x"]), _rel(var.cpu().numpy(), ref["var"])
    print(f"  x {ex:.2e} (bar {tol_x:.1e}) var {ev:.2e} (bar {tol_v:.1e})", flush=True)
    assert ex <= tol_x and ev <= tol_v
    for k in ("rnorm", "anorm", "xnorm"):
        assert abs(r[k] - ref[k]) <= max(1e-10, 10 * ref["sens"][k]) * abs(ref[k])
    # the bucketed pass on the same handle meets the same bar
    S.set_blocked(False, c["maxw"])
    x2, var2, r2 = S.lsqr_solve(b, atol=0, btol=0, itmax=itmax, precond=precond)
    assert _rel(x2.cpu().numpy(), ref["x"]) <= tol_x and _rel(var2.cpu().numpy(), ref["var"]) <= tol_v
    S.close()


@pytest.mark.parametrize("precond", [True, False])
def test_blocked_empty_windows(dev, oracle_lib, precond):
    """Attitude starts moved out of [200, 440): windows 5 to 10 of 40 starts hold no
    rows (no workgroups, no window sums) and their columns are empty; the iterates
    still meet the oracle's bar (its empty columns stay at zero)."""
    print(f"[blocked] empty windows precond={precond}", flush=True)
    c = dict(CASES["many_windows"], seed=35)
    g = copy.copy(_system(c))
    a = g.att_start.astype(np.int64)
    g.att_start = np.where((a >= 200) & (a < 440), a + 400, a).astype(np.int32)
    assert not np.any((g.att_start >= 200) & (g.att_start < 440))
    o = oracle_lib.OSystem(g)
    bn = oracle_lib.known_terms(o, g.x_true, g.noise)
    itmax = 25 if precond else 6
    ref, sx, sv = _sensitivity(oracle_lib, g, o, bn, atol=0, btol=0, itmax=itmax, precond=precond)
    S = dev.System.from_generated(g)
    S.set_blocked(True, c["maxw"])
    x, var, r = S.lsqr_solve(torch.from_numpy(bn).cuda(), atol=0, btol=0, itmax=itmax, precond=precond)
    info = S.blocked_info()
    assert info["active"] == 1 and info["blocks"] == 25
    ex, ev = _rel(x.cpu().numpy(), ref["x"]), _rel(var.cpu().numpy(), ref["var"])
    print(f"  x {ex:.2e} var {ev:.2e} (sensitivity {sx:.1e}, {sv:.1e})", flush=True)
    assert ex <= max(1e-12, 10 * sx) and ev <= max(1e-10, 10 * sv)
    na, nat = g.dims.n_stars * 5, g.dims.n_att
    empty = np.concatenate([na + axis * nat + np.arange(203, 440) for axis in range(3)])
    xh = x.cpu().numpy()
    assert np.all(xh[empty] == 0.0) and np.all(ref["x"][empty] == 0.0)
    S.close()


def test_blocked_converged_solution(dev, oracle_lib):
    """To tolerance: the solution within 1e-10 of the oracle's and the same stop."""
    print("[blocked] converged, many windows", flush=True)
    g = _system(CASES["many_windows"])
    o = oracle_lib.OSystem(g)
    bn = oracle_lib.known_terms(o, g.x_true, g.noise)
    ref = oracle_lib.lsqr(o, bn, atol=1e-12, btol=1e-12, itmax=300, precond=True)
    S = dev.System.from_generated(g)
    S.set_blocked(True, 40)
    x, _, r = S.lsqr_solve(torch.from_numpy(bn).cuda(), atol=1e-12, btol=1e-12, itmax=300, precond=True)
    e = _rel(x.cpu().numpy(), ref["x"])
    print(f"  itn {r['itn']} (oracle {ref['itn']}) istop {r['istop']} x {e:.2e}", flush=True)
    assert r["istop"] == ref["istop"] and abs(r["itn"] - ref["itn"]) <= 1
    assert e <= 1e-10
    S.close()


def test_blocked_fp32_forms(dev, oracle_lib):
    """FP32 storage with FP64 products against the FP64 oracle on the same values, and
    FP32 products against the oracle's FP32-product LSQR in the one-pass order (its
    FP32 operand of A^T u is the unnormalised u'), each at the oracle's last-bit bar."""
    print("[blocked] FP32 forms", flush=True)
    c = CASES["many_windows"]
    g32 = _system(c).as_f32()
    g64 = _system(c)
    g64.vals = g32.vals.astype(np.float64)
    o = oracle_lib.OSystem(g64)
    bn = oracle_lib.known_terms(o, g64.x_true, g64.noise)
    kw = dict(atol=0, btol=0, itmax=25, precond=True)
    ref, sx, sv = _sensitivity(oracle_lib, g64, o, bn, **kw)
    S = dev.System.from_generated(g32)
    S.set_blocked(True, 40)
    b = torch.from_numpy(bn).cuda()
    x, var, r = S.lsqr_solve(b, product="f64", **kw)
    assert S.blocked_info()["active"] == 1
    ex, ev = _rel(x.cpu().numpy(), ref["x"]), _rel(var.cpu().numpy(), ref["var"])
    print(f"  FP64 products: x {ex:.2e} var {ev:.2e}", flush=True)
    assert ex <= max(1e-12, 10 * sx) and ev <= max(1e-10, 10 * sv)
    o32 = oracle_lib.OSystem(g32)
    ref32, sx32, sv32 = _sensitivity(oracle_lib, g32, o32, bn, nruns=12, mode=oracle_lib.P32_1P, **kw)
    dx = _rel(ref32["x"], ref["x"])
    x, var, r = S.lsqr_solve(b, product="f32", **kw)
    ex, ev = _rel(x.cpu().numpy(), ref32["x"]), _rel(var.cpu().numpy(), ref32["var"])
    print(f"  FP32 products: x {ex:.2e} (bar {max(1e-12, 10 * sx32):.1e}; FP32 effect {dx:.2e}) var {ev:.2e}",
          flush=True)
    assert ex <= max(1e-12, 10 * sx32) and ev <= max(1e-10, 10 * sv32)
    # refinement on the regrouped copy reaches the FP64 solution
    ref_c = oracle_lib.lsqr(o, bn, atol=1e-13, btol=1e-13, itmax=500, precond=True)
    xr, rr = S.lsqr_refine(b, atol=1e-6, btol=1e-6, itmax=1000, precond=True, outer_max=10, outer_tol=1e-11)
    e = _rel(xr.cpu().numpy(), ref_c["x"])
    print(f"  refined {e:.2e} after {rr['outer_steps']} outer / {rr['inner_total']} inner", flush=True)
    assert e <= 1e-10
    # from a given x0 (its residual formed inside the first pass of each inner solve)
    x0 = torch.from_numpy(ref_c["x"] + 1e-3 * np.random.default_rng(44).standard_normal(g64.dims.n)).cuda()
    xr0, rr0 = S.lsqr_refine(b, x0=x0, atol=1e-6, btol=1e-6, itmax=1000, precond=True, outer_max=10, outer_tol=1e-11)
    e0 = _rel(xr0.cpu().numpy(), ref_c["x"])
    print(f"  refined from x0 {e0:.2e} after {rr0['outer_steps']} outer / {rr0['inner_total']} inner", flush=True)
    assert e0 <= 1e-10 and rr0["inner_total"] <= rr["inner_total"]
    S.close()


@pytest.mark.parametrize("case", list(CASES))
def test_blocked_fp32_storage_cases(dev, oracle_lib, case):
    """FP32 coefficients (6 chunks per row: other tile offsets and window loads than
    FP64) with FP64 products against the FP64 oracle on the same values, in every
    layout case; FP32 products against the oracle's FP32-product LSQR in the one-pass
    order at its last-bit bar."""
    print(f"[blocked] FP32 storage, {case}", flush=True)
    c = CASES[case]
    g32 = _system(c).as_f32()
    g64 = _system(c)
    g64.vals = g32.vals.astype(np.float64)
    o = oracle_lib.OSystem(g64)
    bn = oracle_lib.known_terms(o, g64.x_true, g64.noise)
    kw = dict(atol=0, btol=0, itmax=20, precond=True)
    ref, sx, sv = _sensitivity(oracle_lib, g64, o, bn, **kw)
    S = dev.System.from_generated(g32)
    S.set_blocked(True, c["maxw"])
    b = torch.from_numpy(bn).cuda()
    x, var, r = S.lsqr_solve(b, product="f64", **kw)
    info = S.blocked_info()
    assert info["active"] == 1
    ex, ev = _rel(x.cpu().numpy(), ref["x"]), _rel(var.cpu().numpy(), ref["var"])
    print(f"  FP64 products: x {ex:.2e} var {ev:.2e} (sensitivity {sx:.1e}, {sv:.1e})", flush=True)
    assert ex <= max(1e-12, 10 * sx) and ev <= max(1e-10, 10 * sv)
    for k in ("rnorm", "anorm", "xnorm"):
        assert abs(r[k] - ref[k]) <= max(1e-12, 10 * ref["sens"][k]) * abs(ref[k]), k
    ref32, sx32, _ = _sensitivity(oracle_lib, g32, oracle_lib.OSystem(g32), bn, nruns=12, mode=oracle_lib.P32_1P,
                                  **kw)
    dx = _rel(ref32["x"], ref["x"])
    x, var, r = S.lsqr_solve(b, product="f32", **kw)
    ex = _rel(x.cpu().numpy(), ref32["x"])
    print(f"  FP32 products: x {ex:.2e} (bar {max(1e-12, 10 * sx32):.1e}; FP32 effect {dx:.2e})", flush=True)
    assert ex <= max(1e-12, 10 * sx32)
    S.close()


def test_blocked_covariances(dev, oracle_lib):
    """Covariances of selected unknowns (astrometric, attitude, instrumental) from the
    direction vectors of a solve on the regrouped copy."""
    print("[blocked] covariances", flush=True)
    g = _system(CASES["many_windows"])
    o = oracle_lib.OSystem(g)
    bn = oracle_lib.known_terms(o, g.x_true, g.noise)
    sel = gsr_synth.covariance_selection(g.dims, 30, 10, 8, seed=3)
    itmax = 25
    ref, sx, sv = _sensitivity(oracle_lib, g, o, bn, atol=0, btol=0, itmax=itmax, precond=True)
    refc = oracle_lib.lsqr(o, bn, atol=0, btol=0, itmax=itmax, precond=True, sel=sel)
    S = dev.System.from_generated(g)
    S.set_blocked(True, 40)
    S.cov_request(sel, block=16)
    x, var, r = S.lsqr_solve(torch.from_numpy(bn).cuda(), atol=0, btol=0, itmax=itmax, precond=True)
    Cg = S.cov_get().cpu().numpy()
    ec = _rel(Cg, refc["cov"])
    print(f"  cov {ec:.2e} (var bar {max(1e-10, 10 * sv):.1e})", flush=True)
    assert ec <= max(1e-10, 10 * sv)
    np.testing.assert_array_equal(Cg, Cg.T)
    S.close()


def test_blocked_toggle_and_limits(dev):
    """max_window below 4 is refused; changing it during a solve is refused; a system
    whose attitude block fits in LDS never builds the copy."""
    print("[blocked] toggles", flush=True)
    g = gsr_synth.make_system(50, 10, 32, 8, 1, seed=35)
    S = dev.System.from_generated(g)
    with pytest.raises(dev.GsrError):
        S.set_blocked(True, 3)
    S.set_blocked(True, 0)
    b = torch.from_numpy(g.noise).cuda()
    S.lsqr_begin(b, atol=0, btol=0, itmax=5, precond=True)
    with pytest.raises(dev.GsrError):
        S.set_blocked(False, 0)
    S.lsqr_end(want_var=False)
    assert S.blocked_info()["active"] == 0
    S.close()


def test_blocked_graphs_export_and_pairs(dev, oracle_lib):
    """On the regrouped copy: blocks of iterations replayed from a captured graph and
    direct launches both meet the oracle's bar; the exported d_i (version 1 of the
    covariance pipeline) match the oracle's; covariances of an index-pair list
    (version 2) match the oracle's dense covariances of the pairs' unknowns."""
    print("[blocked] graphs, export, pairs", flush=True)
    g = _system(CASES["many_windows"])
    o = oracle_lib.OSystem(g)
    bn = oracle_lib.known_terms(o, g.x_true, g.noise)
    n, itmax, block = g.dims.n, 25, 8
    ref, sx, sv = _sensitivity(oracle_lib, g, o, bn, atol=0, btol=0, itmax=itmax, precond=True)
    tol_x, tol_v = max(1e-12, 10 * sx), max(1e-10, 10 * sv)
    S = dev.System.from_generated(g)
    S.set_blocked(True, 40)
    b = torch.from_numpy(bn).cuda()
    for graphs in (True, False, True):
        S.set_graphs(graphs)
        x, var, r = S.lsqr_solve(b, atol=0, btol=0, itmax=itmax, precond=True)
        ex, ev = _rel(x.cpu().numpy(), ref["x"]), _rel(var.cpu().numpy(), ref["var"])
        print(f"  graphs={graphs}: x {ex:.2e} var {ev:.2e}", flush=True)
        assert r["itn"] == itmax and ex <= tol_x and ev <= tol_v
    rng = np.random.default_rng(41)
    pairs = rng.integers(0, n, size=(300, 2))
    pairs[:10, 1] = pairs[:10, 0]
    U, inv = np.unique(pairs.reshape(-1), return_inverse=True)
    inv = inv.reshape(-1, 2)
    refp = oracle_lib.lsqr(o, bn, atol=0, btol=0, itmax=itmax, precond=True, sel=np.arange(n))
    host = torch.empty((8, block, n), dtype=torch.float64).pin_memory()
    S.cov_export(host, block)
    S.cov_request_pairs(pairs, block=block)
    try:
        x, var, r = S.lsqr_solve(b, atol=0, btol=0, itmax=itmax, precond=True)
        nb, lc = S.cov_export_status()
        assert (nb - 1) * block + lc == itmax
        D = host[:nb].reshape(-1, n)[:itmax].numpy()
        ed = _rel(D, refp["dsel"])
        Cref = oracle_lib.covariances(refp["dsel"][:, U], refp["scale"][U])[inv[:, 0], inv[:, 1]]
        ep = _rel(S.cov_get_pairs().cpu().numpy(), Cref)
        print(f"  exported d_i {ed:.2e}  pair covariances {ep:.2e}", flush=True)
        assert ed <= max(1e-10, 10 * sv) and ep <= max(1e-10, 10 * sv)
    finally:
        S.cov_export(None)
        S.cov_request_pairs([], block=64)
    S.close()


@pytest.mark.parametrize("damp", [0.0, 0.5])
def test_blocked_warm_start_and_damp(dev, oracle_lib, damp):
    """A solve from x0 (r0 = b - A x0 formed in the caller's row order, then permuted
    into the regrouped order) and a damped solve on the regrouped copy against the
    oracle."""
    print(f"[blocked] x0 and damp={damp}", flush=True)
    g = _system(CASES["many_windows"])
    o = oracle_lib.OSystem(g)
    bn = oracle_lib.known_terms(o, g.x_true, g.noise)
    x0 = g.x_true + 0.05 * np.random.default_rng(43).standard_normal(g.dims.n)
    kw = dict(damp=damp, atol=0, btol=0, itmax=20, precond=True)
    r1 = oracle_lib.lsqr(o, bn, x0=x0, **kw)
    sx = 0.0
    for seed in (5, 6):
        bp = bn * (1 + 2e-16 * np.random.default_rng(seed).standard_normal(bn.size))
        sx = max(sx, _rel(oracle_lib.lsqr(o, bp, x0=x0, **kw)["x"], r1["x"]))
    S = dev.System.from_generated(g)
    S.set_blocked(True, 40)
    x, var, r = S.lsqr_solve(torch.from_numpy(bn).cuda(), x0=torch.from_numpy(x0).cuda(), **kw)
    assert S.blocked_info()["active"] == 1 and r["itn"] == 20
    ex = _rel(x.cpu().numpy(), r1["x"])
    print(f"  x {ex:.2e} (sens {sx:.1e})", flush=True)
    assert ex <= max(1e-12, 10 * sx)
    assert abs(r["rnorm"] - r1["rnorm"]) <= 1e-10 * abs(r1["rnorm"])
    S.close()
