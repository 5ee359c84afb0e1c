"""Pins of the oracle with constraint equations (extra sparse rows C appended to A,
right-hand sides c appended to b): dense brute force for both products, dense least
squares of the stacked system, and a rank-deficient system whose null space the
constraints remove."""
import numpy as np

import gsr_synth
from _dense import dense_A


def _csr(rows):
    """rows: list of (cols, vals) -> (ptr, col, val)."""
    ptr = np.cumsum([0] + [len(c) for c, _ in rows]).astype(np.int64)
    col = np.concatenate([np.asarray(c, dtype=np.int64) for c, _ in rows])
    val = np.concatenate([np.asarray(v, dtype=np.float64) for _, v in rows])
    return ptr, col, val


def _dense_C(con, n):
    ptr, col, val = con
    Cm = np.zeros((ptr.size - 1, n))
    for i in range(ptr.size - 1):
        for e in range(ptr[i], ptr[i + 1]):
            Cm[i, col[e]] += val[e]
    return Cm


def _random_constraints(n, ncon, width, seed):
    rng = np.random.default_rng(seed)
    return _csr([(rng.choice(n, size=width, replace=False), rng.standard_normal(width)) for _ in range(ncon)])


def test_products_with_constraints_match_dense(oracle_lib):
    g = gsr_synth.make_system(60, (5, 15), 20, 8, 1, seed=51)
    con = _random_constraints(g.dims.n, 7, 30, seed=52)
    o = oracle_lib.OSystem(g, constraints=con)
    M = np.vstack([dense_A(g), _dense_C(con, g.dims.n)])
    assert o.m == g.dims.m + 7
    rng = np.random.default_rng(53)
    x = rng.standard_normal(g.dims.n)
    y = rng.standard_normal(o.m)
    np.testing.assert_allclose(oracle_lib.aprod1(o, x), M @ x, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(oracle_lib.aprod2(o, y), M.T @ y, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(oracle_lib.colnorms(o), np.linalg.norm(M, axis=0), rtol=1e-14)


def test_constrained_lsqr_matches_dense_least_squares(oracle_lib):
    g = gsr_synth.make_system(80, (10, 20), 24, 8, 1, seed=54)
    con = _random_constraints(g.dims.n, 5, 40, seed=55)
    o = oracle_lib.OSystem(g, constraints=con)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    M = np.vstack([dense_A(g), _dense_C(con, g.dims.n)])
    x_ls = np.linalg.lstsq(M, b, rcond=None)[0]
    r = oracle_lib.lsqr(o, b, atol=1e-14, btol=1e-14, itmax=5000, precond=True)
    assert np.linalg.norm(r["x"] - x_ls) <= 1e-10 * np.linalg.norm(x_ls)


def test_constraint_removes_null_space(oracle_lib):
    """Global coefficients equal to astrometric slot 0 make the global column the sum
    of every star's first astrometric column: z = e_glob - sum_s e_{5s} spans the null
    space.  Without constraints LSQR from 0 returns the minimum-norm solution (z . x = 0);
    the constraint x_glob = x_true_glob selects x_true."""
    g = gsr_synth.make_system(50, (8, 16), 16, 6, 1, seed=56, noise_std=0.0)
    g.vals = np.ascontiguousarray(g.vals.copy())
    g.vals[:, 23] = g.vals[:, 0]
    d = g.dims
    jg = d.n - 1
    z = np.zeros(d.n)
    z[jg] = 1.0
    z[0: 5 * d.n_stars: 5] = -1.0
    A = dense_A(g)
    assert np.linalg.norm(A @ z) <= 1e-12 * np.linalg.norm(A)
    o = oracle_lib.OSystem(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    r = oracle_lib.lsqr(o, b, atol=1e-15, btol=1e-15, itmax=5000, precond=False)
    assert abs(z @ r["x"]) <= 1e-9 * np.linalg.norm(r["x"]) * np.linalg.norm(z)
    assert np.linalg.norm(A @ r["x"] - b) <= 1e-9 * np.linalg.norm(b)
    assert np.linalg.norm(r["x"] - g.x_true) > 1e-3 * np.linalg.norm(g.x_true)  # not x_true
    con = _csr([([jg], [1.0])])
    oc = oracle_lib.OSystem(g, constraints=con)
    bc = oracle_lib.known_terms(oc, g.x_true, g.noise)
    assert bc[-1] == g.x_true[jg]
    rc = oracle_lib.lsqr(oc, bc, atol=1e-15, btol=1e-15, itmax=5000, precond=False)
    assert np.linalg.norm(rc["x"] - g.x_true) <= 1e-9 * np.linalg.norm(g.x_true)
