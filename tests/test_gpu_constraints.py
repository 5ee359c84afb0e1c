"""Constraint equations on the GPU (rows C under A, right-hand sides c) against the
oracle: fixed-count LSQR iterates and variances, the column scaling of [A; C], long
rows cut into several tiles, and the null space that a constraint removes."""
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


def _csr(rows):
    ptr = np.cumsum([0] + [len(c) for c, _ in rows]).astype(np.int64)
    col = np.concatenate([np.asarray(c, dtype=np.int64) for c, _ in rows])
    val = np.concatenate([np.asarray(v, dtype=np.float64) for _, v in rows])
    return ptr, col, val


def _constraints(d, seed):
    """A row over every star's first astrometric unknown (long: several tiles when
    there are more than 8192 stars... here the whole astrometric block), a sum of the
    attitude unknowns of axis 1, and short random rows."""
    rng = np.random.default_rng(seed)
    rows = [(np.arange(0, d.n_astro, dtype=np.int64), rng.standard_normal(d.n_astro)),
            (d.n_astro + d.n_att + np.arange(d.n_att), np.ones(d.n_att))]
    for _ in range(4):
        c = np.sort(rng.choice(d.n, size=25, replace=False))
        rows.append((c, rng.standard_normal(25)))
    # each row scaled to the norm of an observation row (~sqrt(24)), as weighted
    # constraint equations would be
    rows = [(c, v * (np.sqrt(24.0) / np.linalg.norm(v))) for c, v in rows]
    return _csr(rows)


def _sens(oracle_lib, g, o, b, **kw):
    r1 = oracle_lib.lsqr(o, b, **kw)
    sx = sv = 0.0
    for seed in (5, 6):
        bp = b * (1 + 2e-16 * np.random.default_rng(seed).standard_normal(b.size))
        r2 = oracle_lib.lsqr(o, bp, **kw)
        sx, sv = max(sx, _rel(r2["x"], r1["x"])), max(sv, _rel(r2["var"], r1["var"]))
    return r1, sx, sv


# maxw: None runs the star-order passes (bucketed attitude sums when n_att is large);
# 0 / 64 the copy regrouped by attitude window at full / capped window width
@pytest.mark.parametrize("n_stars,n_att,precond,itmax,maxw", [
    (300, 32, True, 15, None), (300, 1000, True, 25, None), (3000, 1000, True, 20, None),
    (300, 1000, False, 6, None), (300, 1000, True, 25, 64), (3000, 1000, True, 20, 0), (300, 1000, False, 6, 64)])
def test_constrained_lsqr_matches_oracle(dev, oracle_lib, n_stars, n_att, precond, itmax, maxw):
    print(f"[con] stars={n_stars} n_att={n_att} precond={precond} itmax={itmax} maxw={maxw}", flush=True)
    g = gsr_synth.make_system(n_stars, (10, 20), n_att, 16, 1, seed=61)
    con = _constraints(g.dims, seed=62)
    o = oracle_lib.OSystem(g, constraints=con)
    bfull = oracle_lib.known_terms(o, g.x_true, g.noise)
    ref, sx, sv = _sens(oracle_lib, g, o, bfull, atol=0, btol=0, itmax=itmax, precond=precond)
    S = dev.System.from_generated(g)
    S.set_blocked(maxw is not None, maxw or 0)
    S.set_constraints(*con, rhs=bfull[g.dims.m:])
    if precond:
        sc = S.column_scale().cpu().numpy()
        cn = oracle_lib.colnorms(o)
        assert _rel(sc, np.where(cn > 0, 1.0 / np.where(cn > 0, cn, 1.0), 1.0)) <= 1e-14
    x, var, r = S.lsqr_solve(torch.from_numpy(bfull[: g.dims.m]).cuda(), atol=0, btol=0, itmax=itmax,
                             precond=precond)
    ex, ev = _rel(x.cpu().numpy(), ref["x"]), _rel(var.cpu().numpy(), ref["var"])
    print(f"  x {ex:.2e} (sens {sx:.1e})  var {ev:.2e} (sens {sv:.1e})", flush=True)
    assert r["itn"] == itmax
    assert S.blocked_info()["active"] == (maxw is not None)
    assert ex <= max(1e-12, 10 * sx) and ev <= max(1e-10, 10 * sv)
    for k in ("rnorm", "anorm", "xnorm", "bnorm"):
        assert abs(r[k] - ref[k]) <= 1e-10 * abs(ref[k]), k
    S.close()


def test_constraint_removes_null_space_on_gpu(dev, oracle_lib):
    """Global coefficients equal to astrometric slot 0: without constraints the solve
    returns the minimum-norm solution, with x_glob fixed it returns x_true."""
    print("[con] null space", flush=True)
    g = gsr_synth.make_system(50, (8, 16), 16, 6, 1, seed=56, noise_std=0.0)
    g.vals = np.ascontiguousarray(g.vals.copy())
    g.vals[:, 23] = g.vals[:, 0]
    d = g.dims
    jg = d.n - 1
    z = np.zeros(d.n)
    z[jg] = 1.0
    z[0: 5 * d.n_stars: 5] = -1.0
    o = oracle_lib.OSystem(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    S = dev.System.from_generated(g)
    x, _, _ = S.lsqr_solve(torch.from_numpy(b).cuda(), atol=1e-15, btol=1e-15, itmax=5000, precond=False)
    x = x.cpu().numpy()
    assert abs(z @ x) <= 1e-9 * np.linalg.norm(x) * np.linalg.norm(z)
    assert _rel(x, g.x_true) > 1e-3
    S.set_constraints(np.array([0, 1]), np.array([jg]), np.array([1.0]), rhs=np.array([g.x_true[jg]]))
    xc, _, rc = S.lsqr_solve(torch.from_numpy(b).cuda(), atol=1e-15, btol=1e-15, itmax=5000, precond=False)
    e = _rel(xc.cpu().numpy(), g.x_true)
    print(f"  constrained: {e:.2e} after {rc['itn']} iterations", flush=True)
    assert e <= 1e-9
    S.close()


def test_constraints_need_the_fused_iteration(dev):
    g = gsr_synth.make_system(30, 10, 16, 6, 1, seed=63)
    S = dev.System.from_generated(g)
    S.set_constraints(np.array([0, 2]), np.array([0, 3]), np.array([1.0, -1.0]), rhs=np.array([0.0]))
    b = torch.zeros(g.dims.m, dtype=torch.float64, device="cuda")
    S.set_fused(False)
    with pytest.raises(dev.GsrError):
        S.lsqr_solve(b, itmax=3)
    S.set_fused(True)
    S.lsqr_solve(b, itmax=3)
    with pytest.raises(dev.GsrError):  # columns must be strictly increasing
        S.set_constraints(np.array([0, 2]), np.array([3, 3]), np.array([1.0, 1.0]), rhs=np.array([0.0]))
    S.close()


def test_constrained_fp32_storage_on_regrouped_copy(dev, oracle_lib):
    """FP32-stored coefficients with FP64 products and constraint equations, on the
    copy regrouped by attitude window, against the FP64 oracle on the same values."""
    print("[con] FP32 storage, regrouped copy", flush=True)
    g32 = gsr_synth.make_system(300, (10, 20), 1000, 16, 1, seed=64).as_f32()
    g64 = gsr_synth.make_system(300, (10, 20), 1000, 16, 1, seed=64)
    g64.vals = g32.vals.astype(np.float64)
    con = _constraints(g64.dims, seed=65)
    o = oracle_lib.OSystem(g64, constraints=con)
    bfull = oracle_lib.known_terms(o, g64.x_true, g64.noise)
    ref, sx, sv = _sens(oracle_lib, g64, o, bfull, atol=0, btol=0, itmax=25, precond=True)
    S = dev.System.from_generated(g32)
    S.set_blocked(True, 64)
    S.set_constraints(*con, rhs=bfull[g64.dims.m:])
    x, var, r = S.lsqr_solve(torch.from_numpy(bfull[: g64.dims.m]).cuda(), atol=0, btol=0, itmax=25, precond=True,
                             product="f64")
    assert S.blocked_info()["active"] == 1 and r["itn"] == 25
    ex, ev = _rel(x.cpu().numpy(), ref["x"]), _rel(var.cpu().numpy(), ref["var"])
    print(f"  x {ex:.2e} (sens {sx:.1e})  var {ev:.2e} (sens {sv:.1e})", flush=True)
    assert ex <= max(1e-12, 10 * sx) and ev <= max(1e-10, 10 * sv)
    with pytest.raises(dev.GsrError):  # FP32 products with constraint equations are refused
        S.lsqr_solve(torch.from_numpy(bfull[: g64.dims.m]).cuda(), itmax=3, product="f32")
    S.close()
