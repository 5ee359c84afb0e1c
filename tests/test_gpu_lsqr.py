"""Parity of the device-resident LSQR (variances, covariances, FP32 form with
refinement) with the CPU oracle.

LSQR iterates past the point where the Krylov basis loses orthogonality are
themselves sensitive to rounding (the oracle perturbed at the last bit of b
or of A moves them by up to ~1e-8 on the unscaled 1,000-star system, and
moves the variances of a converged run by ~1e-4, its anorm estimate by ~1e-5).
Converged solutions are
held to 1e-10; unconverged iterates and post-convergence variances are held
to 1e-12 or, when the oracle's own last-bit sensitivity is larger, to 10x
that sensitivity."""
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


@pytest.fixture(scope="module")
def tiny(dev, oracle_lib):
    g = gsr_synth.tiny()
    o = oracle_lib.OSystem(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    S = dev.System.from_generated(g)
    return g, o, b, S


def _sensitivity(oracle_lib, g, o, b, nruns=2, **kw):
    """The oracle's own response to last-bit perturbations: b and, separately, every
    coefficient of A scaled by (1 + 2.2e-16 N(0,1)) (the size of the rounding differences
    between two valid summation orders).  Returns the reference run and the largest
    relative deviations of x and var over three perturbed runs; the deviations of the
    scalar estimates (rnorm, anorm, ...) are kept in r1["sens"]."""
    import copy

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
                  for k in ("rnorm", "anorm", "acond", "xnorm", "bnorm")}
    return r1, sx, sv


def test_lsqr_converged_tiny_precond(dev, oracle_lib, tiny):
    """Converged solution to 1e-10.  The variances keep accumulating after convergence,
    where the search directions lose orthogonality; they are held to 10x the oracle's own
    last-bit sensitivity (about 1e-4 here)."""
    print("[lsqr] tiny, column-scaled, to tolerance", flush=True)
    g, o, b, S = tiny
    ref, _, sv = _sensitivity(oracle_lib, g, o, b, atol=1e-12, btol=1e-12, itmax=200, precond=True)
    x, var, r = S.lsqr_solve(torch.from_numpy(b).cuda(), atol=1e-12, btol=1e-12, itmax=200, precond=True)
    x, var = x.cpu().numpy(), var.cpu().numpy()
    print(f"  gpu istop={r['istop']} itn={r['itn']}  oracle istop={ref['istop']} itn={ref['itn']}", flush=True)
    assert r["istop"] == ref["istop"]
    assert abs(r["itn"] - ref["itn"]) <= 1
    assert _rel(x, ref["x"]) <= 1e-10
    assert _rel(var, ref["var"]) <= max(1e-10, 10 * sv)
    # anorm and acond keep accumulating alpha and beta after convergence, as var does
    for k in ("rnorm", "anorm", "acond", "xnorm", "bnorm"):
        assert abs(r[k] - ref[k]) <= max(1e-6, 10 * ref["sens"][k]) * abs(ref[k]) + 1e-300, k
    # ||A^T r|| at the solution is at rounding level: compare on the scale of the stop test
    assert abs(r["arnorm"] - ref["arnorm"]) <= 0.05 * ref["arnorm"] + 1e-16 * ref["anorm"] * ref["rnorm"]


@pytest.mark.parametrize("precond,itmax", [(True, 5), (True, 30), (False, 20)])
def test_lsqr_fixed_iterations(dev, oracle_lib, tiny, precond, itmax):
    print(f"[lsqr] tiny fixed count precond={precond} itmax={itmax}", flush=True)
    g, o, b, S = tiny
    ref, sx, sv = _sensitivity(oracle_lib, g, o, b, atol=0, btol=0, itmax=itmax, precond=precond)
    x, var, r = S.lsqr_solve(torch.from_numpy(b).cuda(), atol=0, btol=0, itmax=itmax, precond=precond)
    assert r["itn"] == itmax and r["istop"] == 7
    print(f"  oracle sensitivity x {sx:.2e} var {sv:.2e}", flush=True)
    assert _rel(x.cpu().numpy(), ref["x"]) <= max(1e-12, 10 * sx)
    assert _rel(var.cpu().numpy(), ref["var"]) <= max(1e-12, 10 * sv)


def test_lsqr_unscaled_as_written(dev, oracle_lib, tiny):
    """The 1,000-star system without scaling, damp 0, atol = btol = 1e-12, itmax 200."""
    print("[lsqr] tiny unscaled itmax=200", flush=True)
    g, o, b, S = tiny
    ref, sx, _ = _sensitivity(oracle_lib, g, o, b, atol=1e-12, btol=1e-12, itmax=200, precond=False)
    x, _, r = S.lsqr_solve(torch.from_numpy(b).cuda(), atol=1e-12, btol=1e-12, itmax=200, precond=False)
    print(f"  oracle self-sensitivity {sx:.2e}; gpu istop={r['istop']} itn={r['itn']}", flush=True)
    assert r["istop"] == ref["istop"] == 7
    assert _rel(x.cpu().numpy(), ref["x"]) <= max(1e-12, 10 * sx)


def test_lsqr_damped_and_warm_start(dev, oracle_lib):
    print("[lsqr] damp > 0, warm start", flush=True)
    g = gsr_synth.make_system(300, (10, 30), 20, 10, 1, seed=12)
    o = oracle_lib.OSystem(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    S = dev.System.from_generated(g)
    bt = torch.from_numpy(b).cuda()
    ref = oracle_lib.lsqr(o, b, damp=0.3, atol=1e-13, btol=1e-13, itmax=1000, precond=True)
    x, _, r = S.lsqr_solve(bt, damp=0.3, atol=1e-13, btol=1e-13, itmax=1000, precond=True)
    assert _rel(x.cpu().numpy(), ref["x"]) <= 1e-10
    x0 = ref["x"] + 1e-3 * np.random.default_rng(0).standard_normal(g.dims.n)
    ref0 = oracle_lib.lsqr(o, b, x0=x0, atol=1e-13, btol=1e-13, itmax=1000, precond=True)
    x, _, r = S.lsqr_solve(bt, x0=torch.from_numpy(x0).cuda(), atol=1e-13, btol=1e-13, itmax=1000, precond=True)
    assert _rel(x.cpu().numpy(), ref0["x"]) <= 1e-10
    assert abs(r["itn"] - ref0["itn"]) <= 1
    S.close()


def test_lsqr_edge_cases(dev, oracle_lib):
    print("[lsqr] b = 0, itmax = 0, exact x0", flush=True)
    g = gsr_synth.make_system(50, 8, 8, 6, 1, seed=13)
    o = oracle_lib.OSystem(g)
    S = dev.System.from_generated(g)
    z = torch.zeros(g.dims.m, dtype=torch.float64, device="cuda")
    x, var, r = S.lsqr_solve(z, itmax=50)
    assert r["istop"] == 0 and r["itn"] == 0 and torch.all(x == 0) and torch.all(var == 0)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    x, _, r = S.lsqr_solve(torch.from_numpy(b).cuda(), itmax=0)
    assert r["itn"] == 0 and torch.all(x == 0)
    # x0 solving the system exactly: b0 = A x0 formed by the same product, so b0 - A x0 = 0 bit for bit
    x0 = torch.from_numpy(g.x_true).cuda()
    b0 = S.aprod1(x0)
    x, _, r = S.lsqr_solve(b0, x0=x0, itmax=50)
    assert r["itn"] == 0 and r["istop"] == 0 and torch.equal(x, x0)
    S.close()


def test_identity_solution(dev, oracle_lib):
    """Sec. 3: x_true = 1 and noise-free known terms give the identity solution."""
    print("[lsqr] identity solution", flush=True)
    g = gsr_synth.tiny(x_kind="ones", noise_std=0.0)
    o = oracle_lib.OSystem(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    S = dev.System.from_generated(g)
    x, _, r = S.lsqr_solve(torch.from_numpy(b).cuda(), atol=1e-12, btol=1e-12, itmax=500, precond=True)
    assert r["istop"] == 1
    assert float((x - 1).abs().max()) < 1e-9
    S.close()


def test_session_api_matches_solve(dev, oracle_lib, tiny):
    print("[lsqr] begin / iterate / peek / end", flush=True)
    g, o, b, S = tiny
    bt = torch.from_numpy(b).cuda()
    S.lsqr_begin(bt, atol=0, btol=0, itmax=40, precond=True)
    S.lsqr_iterate(10)
    st = S.lsqr_status()
    assert st["itn"] == 10
    xp = S.lsqr_peek().cpu().numpy()
    ref10 = oracle_lib.lsqr(o, b, atol=0, btol=0, itmax=10, precond=True)
    assert _rel(xp, ref10["x"]) <= 1e-12
    S.lsqr_iterate(100)  # capped by itmax
    x, var, r = S.lsqr_end()
    assert r["itn"] == 40 and r["istop"] == 7
    with pytest.raises(dev.GsrError):
        S.lsqr_iterate(1)


@pytest.mark.parametrize("block", [64, 7])
def test_covariances(dev, oracle_lib, block):
    print(f"[cov] block={block}", flush=True)
    g = gsr_synth.make_system(400, 20, 32, 16, 1, seed=14)
    o = oracle_lib.OSystem(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    sel = gsr_synth.covariance_selection(g.dims, 30, 10, 8, seed=3)
    S = dev.System.from_generated(g)
    S.cov_request(sel, block=block)
    itmax = 45  # below convergence: a stable comparison, and not a multiple of the block
    ref = oracle_lib.lsqr(o, b, atol=0, btol=0, itmax=itmax, precond=True, sel=sel)
    x, var, r = S.lsqr_solve(torch.from_numpy(b).cuda(), atol=0, btol=0, itmax=itmax, precond=True)
    Cg = S.cov_get().cpu().numpy()
    assert _rel(Cg, ref["cov"]) <= 1e-12
    np.testing.assert_array_equal(Cg, Cg.T)
    assert _rel(np.diag(Cg), var.cpu().numpy()[sel]) <= 1e-13
    S.close()


def test_syrk_entry_point(dev):
    """C += D D^T on the upper tiles for ragged sizes and column counts."""
    print("[syrk]", flush=True)
    rng = np.random.default_rng(7)
    for k, cols, ldd in [(1, 1, 1), (37, 5, 9), (100, 64, 64), (130, 150, 160), (200, 70, 71)]:
        D = rng.standard_normal((k, ldd))
        C0 = rng.standard_normal((k, k))
        Ct = torch.from_numpy(C0.copy()).cuda()
        dev.syrk(torch.from_numpy(D).cuda(), k, cols, ldd, Ct)
        ref = C0 + D[:, :cols] @ D[:, :cols].T
        got = Ct.cpu().numpy()
        T = (k + 31) // 32
        for ti in range(T):
            for tj in range(T):
                blk = (slice(32 * ti, 32 * ti + 32), slice(32 * tj, 32 * tj + 32))
                if ti <= tj:
                    np.testing.assert_allclose(got[blk], ref[blk], rtol=1e-13, atol=1e-12)
                else:
                    np.testing.assert_array_equal(got[blk], C0[blk])


def test_fp32_refinement(dev, oracle_lib):
    print("[fp32 refine] tiny", flush=True)
    g = gsr_synth.tiny().as_f32()
    o = oracle_lib.OSystem(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    ref = oracle_lib.lsqr(o, b, atol=1e-14, btol=1e-14, itmax=1000, precond=True)
    S = dev.System.from_generated(g)
    bt = torch.from_numpy(b).cuda()
    # inner LSQR with FP32 products alone, separate aprod passes: parity with the
    # oracle's FP32-product LSQR (both round the same operands to FP32)
    ref32 = oracle_lib.lsqr(o, b, atol=1e-6, btol=1e-6, itmax=1000, precond=True, mode=oracle_lib.P32)
    S.set_fused(False)
    x32, _, r32 = S.lsqr_solve(bt, atol=1e-6, btol=1e-6, itmax=1000, precond=True, product="f32")
    assert abs(r32["itn"] - ref32["itn"]) <= 1
    assert _rel(x32.cpu().numpy(), ref32["x"]) <= 1e-10
    # the refined solution, with and without the fused pass, within 1e-10 of the FP64 oracle
    for fused in (True, False):
        S.set_fused(fused)
        xr, rr = S.lsqr_refine(bt, atol=1e-6, btol=1e-6, itmax=1000, precond=True, outer_max=10, outer_tol=1e-11)
        e = _rel(xr.cpu().numpy(), ref["x"])
        print(f"  fused={fused}: refined error {e:.2e} after {rr['outer_steps']} outer / {rr['inner_total']} inner",
              flush=True)
        assert e <= 1e-10
    S.close()


@pytest.mark.parametrize("precond,cov", [(True, False), (False, False), (True, True)])
def test_graph_replay_matches_direct_launches(dev, oracle_lib, precond, cov):
    """Blocks of iterations replayed from a captured graph, direct launches, and a second
    replay of the same graph all meet the oracle's bar.  The atomic additions in aprod2
    sum in a run-dependent order, so runs differ among themselves at the oracle's own
    last-bit sensitivity."""
    print(f"[lsqr] graphs precond={precond} cov={cov}", flush=True)
    g = gsr_synth.make_system(400, 20, 32, 16, 1, seed=15)
    o = oracle_lib.OSystem(g)
    bn = oracle_lib.known_terms(o, g.x_true, g.noise)
    b = torch.from_numpy(bn).cuda()
    S = dev.System.from_generated(g)
    if cov:
        S.cov_request(gsr_synth.covariance_selection(g.dims, 10, 5, 4, seed=1), block=16)
    # unscaled, this matrix is ill-conditioned enough that iterates past ~12 depend
    # on the last bit of the data (oracle self-sensitivity 2e-3 at 20 iterations)
    itmax = 30 if precond else 10
    ref, sx, sv = _sensitivity(oracle_lib, g, o, bn, atol=0, btol=0, itmax=itmax, precond=precond)
    tol_x, tol_v = max(1e-12, 10 * sx), max(1e-10, 10 * sv)
    print(f"  oracle sensitivity x {sx:.2e} var {sv:.2e}", flush=True)
    out = []
    for on in (True, False, True):  # the second graph run reuses the captured graph
        S.set_graphs(on)
        x, var, r = S.lsqr_solve(b, atol=0, btol=0, itmax=itmax, precond=precond)
        out.append((x.cpu().numpy(), var.cpu().numpy(), r, S.cov_get().cpu().numpy() if cov else None))
    for x, var, r, C_ in out:
        assert r["itn"] == itmax
        assert _rel(x, ref["x"]) <= tol_x and _rel(var, ref["var"]) <= tol_v
        if cov:  # sums of products of the same direction vectors as var
            assert _rel(C_, out[0][3]) <= tol_v
    S.close()


@pytest.mark.parametrize("n_att,n_instr,precond", [(32, 16, True), (1000, 16, True), (1000, 16, False),
                                                   (1000, 2000, True)])
def test_fused_iteration_matches_separate_products(dev, oracle_lib, n_att, n_instr, precond):
    """One pass over the rows per iteration (A v and the star part of A^T u on the
    unnormalised u) against the oracle and against separate aprod 1 / aprod 2 passes.
    n_att = 32 keeps the tail in LDS; 1000 uses the bucketed attitude pass; 2000
    instrumental columns is close to the largest supported (2047)."""
    print(f"[lsqr] fused vs separate n_att={n_att} n_instr={n_instr} precond={precond}", flush=True)
    g = gsr_synth.make_system(300, (20, 40), n_att, n_instr, 1, seed=17)
    o = oracle_lib.OSystem(g)
    bn = oracle_lib.known_terms(o, g.x_true, g.noise)
    b = torch.from_numpy(bn).cuda()
    # Unscaled, this system's iterates past ~8 steps depend on the summation order
    # itself (dense numpy LSQR and the oracle differ by 4e-9 at 10 steps, more than
    # the response to last-bit data perturbations shows), so that case stops at 6.
    itmax = 25 if precond else 6
    ref, sx, sv = _sensitivity(oracle_lib, g, o, bn, atol=0, btol=0, itmax=itmax, precond=precond)
    tol_x, tol_v = max(1e-12, 10 * sx), max(1e-10, 10 * sv)
    S = dev.System.from_generated(g)
    out = {}
    for fused in (True, False):
        S.set_fused(fused)
        x, var, r = S.lsqr_solve(b, atol=0, btol=0, itmax=itmax, precond=precond)
        assert r["itn"] == itmax
        out[fused] = (x.cpu().numpy(), var.cpu().numpy(), r)
        print(f"  fused={fused}: x {_rel(out[fused][0], ref['x']):.2e} var {_rel(out[fused][1], ref['var']):.2e}",
              flush=True)
        assert _rel(out[fused][0], ref["x"]) <= tol_x
        assert _rel(out[fused][1], ref["var"]) <= tol_v
    for k in ("rnorm", "anorm", "xnorm"):
        assert abs(out[True][2][k] - ref[k]) <= max(1e-10, 10 * ref["sens"][k]) * abs(ref[k])
    S.close()


def test_fused_fp32_storage_fp64_products(dev, oracle_lib):
    """FP32-stored coefficients with FP64 products (the bytes-only form): the fused
    pass on float rows matches the FP64 oracle on the same FP32-representable matrix."""
    print("[lsqr] fused, FP32 storage, FP64 products", flush=True)
    g = gsr_synth.make_system(300, (20, 40), 1000, 16, 1, seed=18).as_f32()
    g64 = gsr_synth.make_system(300, (20, 40), 1000, 16, 1, seed=18)
    g64.vals = g.vals.astype(np.float64)  # the same values, exactly
    o = oracle_lib.OSystem(g64)
    bn = oracle_lib.known_terms(o, g64.x_true, g64.noise)
    ref, sx, sv = _sensitivity(oracle_lib, g64, o, bn, atol=0, btol=0, itmax=25, precond=True)
    S = dev.System.from_generated(g)
    x, var, r = S.lsqr_solve(torch.from_numpy(bn).cuda(), atol=0, btol=0, itmax=25, precond=True, product="f64")
    assert r["itn"] == 25
    ex, ev = _rel(x.cpu().numpy(), ref["x"]), _rel(var.cpu().numpy(), ref["var"])
    print(f"  x {ex:.2e} var {ev:.2e}", flush=True)
    assert ex <= max(1e-12, 10 * sx) and ev <= max(1e-10, 10 * sv)
    S.close()


@pytest.mark.parametrize("n_att", [32, 1000])
def test_fused_fp32_products(dev, oracle_lib, n_att):
    """FP32 products summed in FP64 (the inner solves of the FP32 form) against the
    oracle's FP32-product LSQR, with the attitude tail in LDS (32) and bucketed (1000).
    Separate aprod 1 / aprod 2 passes round the same operands as the oracle's textbook
    order (P32).  The one-pass iteration forms A^T u' on the unnormalised u' and scales
    by 1/beta afterwards, so its FP32 operands are fl32(u'_r), not fl32(u'_r / beta);
    the oracle's one-pass order (P32_1P) rounds the same operands.  Each form meets
    its oracle at the oracle's own last-bit bar, taken over twelve perturbations of b
    (the response of FP32-product iterates comes from rare FP32 rounding flips)."""
    print(f"[lsqr] fused FP32 products n_att={n_att}", flush=True)
    g = gsr_synth.make_system(300, (20, 40), n_att, 16, 1, seed=19).as_f32()
    o = oracle_lib.OSystem(g)
    bn = oracle_lib.known_terms(o, g.x_true, g.noise)
    kw = dict(atol=0, btol=0, itmax=25, precond=True)
    refs = {False: _sensitivity(oracle_lib, g, o, bn, nruns=12, mode=oracle_lib.P32, **kw),
            True: _sensitivity(oracle_lib, g, o, bn, nruns=12, mode=oracle_lib.P32_1P, **kw)}
    ref64 = oracle_lib.lsqr(o, bn, **kw)
    dx = _rel(refs[False][0]["x"], ref64["x"])
    d1p = _rel(refs[True][0]["x"], refs[False][0]["x"])
    print(f"  FP32 vs FP64 products x {dx:.2e}; one-pass vs textbook order {d1p:.2e}", flush=True)
    assert dx > 10 * refs[False][1]  # the FP32 products are visible above the last-bit noise
    S = dev.System.from_generated(g)
    for fused in (False, True):
        ref, sx, sv = refs[fused]
        S.set_fused(fused)
        x, var, r = S.lsqr_solve(torch.from_numpy(bn).cuda(), product="f32", **kw)
        assert r["itn"] == 25
        ex, ev = _rel(x.cpu().numpy(), ref["x"]), _rel(var.cpu().numpy(), ref["var"])
        print(f"  fused={fused}: x {ex:.2e} (bar {max(1e-12, 10 * sx):.1e}) var {ev:.2e}", flush=True)
        assert ex <= max(1e-12, 10 * sx) and ev <= max(1e-10, 10 * sv)
    S.close()


def test_cov_export_version1(dev, oracle_lib, tiny):
    """Whole d_i vectors exported every `block` iterations (version 1 of the covariance
    pipeline) against the oracle's d_i; covariances formed afterwards from the export
    against the in-run covariances and the oracle's.  Two solves: a fixed count
    ending in a partial block, and a converged solve stopping mid-block."""
    print("[lsqr] covariance export (version 1)", flush=True)
    g, o, b, S = tiny
    n, block = g.dims.n, 16
    sel = gsr_synth.covariance_selection(g.dims, 10, 5, 4, seed=1)
    Sc = S.column_scale()
    host = torch.empty((16, block, n), dtype=torch.float64).pin_memory()
    S.cov_export(host, block)
    S.cov_request(sel, block=block)
    try:
        for itmax, tol in ((40, 0.0), (200, 1e-12)):
            x, var, r = S.lsqr_solve(torch.from_numpy(b).cuda(), atol=tol, btol=tol, itmax=itmax, precond=True)
            nb, lc = S.cov_export_status()
            itn = r["itn"]
            print(f"  itmax={itmax}: itn={itn} blocks={nb} last={lc}", flush=True)
            assert (nb - 1) * block + lc == itn and 1 <= lc <= block
            ref = oracle_lib.lsqr(o, b, atol=tol, btol=tol, itmax=itmax, precond=True, sel=np.arange(n))
            assert abs(ref["itn"] - itn) <= 1
            k = min(itn, ref["itn"])
            D = host[:nb].reshape(-1, n)[:k].numpy()
            # the first 40 iterates are insensitive (1e-15); past convergence d_i shrinks
            # like the residual and keeps a last-bit relative error of its own size
            e = _rel(D[:40], ref["dsel"][:40])
            print(f"    exported d_i vs oracle (first 40): {e:.2e}", flush=True)
            assert e <= 1e-10
            C_post = dev.cov_from_export(host, n, block, nb, lc, sel, S=Sc).cpu().numpy()
            C_run = S.cov_get().cpu().numpy()
            C_ref = oracle_lib.covariances(ref["dsel"][:, sel], ref["scale"][sel])
            e_run, e_ref = _rel(C_post, C_run), _rel(C_post, C_ref)
            print(f"    post-hoc C vs in-run {e_run:.2e}, vs oracle {e_ref:.2e}", flush=True)
            assert e_run <= 1e-13
            # C sums d_i d_i^T over every iterate.  At 40 fixed iterations the oracle's own
            # last-bit response is 3e-14; the converged solve (77 steps) adds iterates past
            # convergence whose d_i are rounding-dominated, so there the bar is 10x the
            # oracle's measured response to last-bit perturbations (of b twice, of every
            # coefficient once), as for the variances
            if tol == 0.0:
                assert e_ref <= 1e-10
            else:
                import copy

                runs = []
                for seed in (5, 6):
                    bp = b * (1 + 2e-16 * np.random.default_rng(seed).standard_normal(b.size))
                    runs.append(oracle_lib.lsqr(o, bp, atol=tol, btol=tol, itmax=itmax, precond=True, sel=sel))
                gp = copy.copy(g)
                gp.vals = g.vals * (1 + 2.2e-16 * np.random.default_rng(7).standard_normal(g.vals.shape))
                runs.append(oracle_lib.lsqr(oracle_lib.OSystem(gp), b, atol=tol, btol=tol, itmax=itmax,
                                            precond=True, sel=sel))
                sens = max(_rel(rp["cov"], C_ref) for rp in runs)
                print(f"    oracle covariance sensitivity {sens:.2e}", flush=True)
                assert e_ref <= max(1e-10, 10 * sens)
    finally:
        S.cov_export(None)
        S.cov_request([], block=64)


def test_cov_pairs(dev, oracle_lib, tiny):
    """Covariances of a pair list (version 2 of the covariance pipeline), in-run and from
    an export, against the oracle's dense covariances of the pairs' indexes; (j, j)
    pairs give the variances."""
    print("[lsqr] covariance pair list", flush=True)
    g, o, b, S = tiny
    n, block, itmax = g.dims.n, 16, 40
    rng = np.random.default_rng(23)
    pairs = rng.integers(0, n, size=(500, 2))
    pairs[:20, 1] = pairs[:20, 0]  # variances
    pairs[20:30] = pairs[30:40]    # repeated pairs
    U, inv = np.unique(pairs.reshape(-1), return_inverse=True)
    inv = inv.reshape(-1, 2)
    ref = oracle_lib.lsqr(o, b, atol=0, btol=0, itmax=itmax, precond=True, sel=U)
    Cref = ref["cov"][inv[:, 0], inv[:, 1]]
    host = torch.empty((4, block, n), dtype=torch.float64).pin_memory()
    S.cov_export(host, block)
    S.cov_request_pairs(pairs, block=block)
    try:
        x, var, r = S.lsqr_solve(torch.from_numpy(b).cuda(), atol=0, btol=0, itmax=itmax, precond=True)
        assert r["itn"] == itmax
        cp = S.cov_get_pairs().cpu().numpy()
        nb, lc = S.cov_export_status()
        cx = dev.cov_pairs_from_export(host, n, block, nb, lc, pairs, S=S.column_scale()).cpu().numpy()
        v = var.cpu().numpy()
        print(f"  in-run {_rel(cp, Cref):.2e}  from export {_rel(cx, Cref):.2e}", flush=True)
        assert _rel(cp, Cref) <= 1e-10 and _rel(cx, Cref) <= 1e-10
        assert _rel(cp[:20], v[pairs[:20, 0]]) <= 1e-12
        np.testing.assert_array_equal(cp[20:30], cp[30:40])
        with pytest.raises(dev.GsrError):
            S.cov_get()  # a pair request has no dense block
    finally:
        S.cov_export(None)
        S.cov_request_pairs([], block=64)


@pytest.mark.parametrize("precond,conlim", [(False, 30.0), (True, 50.0)])
def test_conlim_stop(dev, oracle_lib, precond, conlim):
    """conlim > 0: the solve stops with istop 3 at the first iteration whose condition
    estimate acond reaches conlim, at the oracle's iteration (the estimate grows by
    ~3 per iteration on this system, far from the limit's rounding), with the oracle's
    iterate and estimates."""
    print(f"[lsqr] conlim {conlim} precond={precond}", flush=True)
    g = gsr_synth.make_system(n_stars=40, obs=12, n_att=16, n_instr=8, n_glob=1, seed=61)
    o = oracle_lib.OSystem(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    kw = dict(atol=1e-14, btol=1e-14, conlim=conlim, itmax=3000, precond=precond)
    ref, sx, _ = _sensitivity(oracle_lib, g, o, b, **kw)
    assert ref["istop"] == 3
    S = dev.System.from_generated(g)
    x, _, r = S.lsqr_solve(torch.from_numpy(b).cuda(), **kw)
    print(f"  gpu istop={r['istop']} itn={r['itn']} acond={r['acond']:.6f}  oracle itn={ref['itn']} "
          f"acond={ref['acond']:.6f}", flush=True)
    assert r["istop"] == 3 and r["itn"] == ref["itn"]
    assert r["acond"] >= conlim
    assert _rel(x.cpu().numpy(), ref["x"]) <= max(1e-12, 10 * sx)
    for k in ("acond", "anorm", "rnorm", "xnorm"):
        assert abs(r[k] - ref[k]) <= max(1e-12, 10 * ref["sens"][k]) * abs(ref[k]), k
    S.close()


def test_refine_rejects_damp(dev):
    """The refinement solves the undamped problem: damp > 0 is refused."""
    g = gsr_synth.make_system(50, 8, 8, 6, 1, seed=13).as_f32()
    S = dev.System.from_generated(g)
    b = torch.zeros(g.dims.m, dtype=torch.float64, device="cuda")
    with pytest.raises(dev.GsrError):
        S.lsqr_refine(b, damp=0.1)
    S.close()
