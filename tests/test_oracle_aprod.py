"""Pins of the oracle's products, Eq. (2) and Eq. (3), against facts that do
not depend on the oracle: a dense brute-force matrix, the adjoint identity,
row sums, unit vectors and exactly rounded sums."""
import math

import numpy as np
import pytest

import gsr_synth
from tests._dense import dense_A

SMALL_CASES = [
    dict(n_stars=40, obs=12, n_att=16, n_instr=8, n_glob=1, seed=7),
    dict(n_stars=25, obs=(3, 9), n_att=5, n_instr=6, n_glob=0, seed=8),
    dict(n_stars=1, obs=30, n_att=4, n_instr=12, n_glob=1, seed=9),
]


@pytest.fixture(params=range(len(SMALL_CASES)))
def small_sys(request, oracle_lib):
    g = gsr_synth.make_system(**SMALL_CASES[request.param])
    return g, oracle_lib.OSystem(g), dense_A(g)


def test_row_structure_matches_paper(small_sys):
    """Sec. 2: at most 24 nonzeros per row: 5 astro, 12 attitude, 6 instr, 1 global."""
    g, _, A = small_sys
    d = g.dims
    nz = (A != 0).sum(axis=1)
    assert np.all(nz == 23 + d.n_glob)
    assert np.all((A[:, : d.n_astro] != 0).sum(axis=1) == 5)
    assert np.all((A[:, d.n_astro: d.n_astro + 3 * d.n_att] != 0).sum(axis=1) == 12)
    NI = d.n_astro + 3 * d.n_att
    assert np.all((A[:, NI: NI + d.n_instr] != 0).sum(axis=1) == 6)


def test_aprod1_vs_dense(small_sys, oracle_lib):
    g, o, A = small_sys
    rng = np.random.default_rng(1)
    x = rng.standard_normal(g.dims.n)
    y0 = rng.standard_normal(g.dims.m)
    y = oracle_lib.aprod1(o, x)
    np.testing.assert_allclose(y, A @ x, rtol=0, atol=1e-13 * np.abs(A).sum(1).max() * np.abs(x).max())
    y2 = oracle_lib.aprod1(o, x, y=y0, scale=-0.75)
    np.testing.assert_allclose(y2, -0.75 * y0 + A @ x, rtol=1e-13, atol=1e-12)


def test_aprod2_vs_dense(small_sys, oracle_lib):
    g, o, A = small_sys
    rng = np.random.default_rng(2)
    y = rng.standard_normal(g.dims.m)
    x0 = rng.standard_normal(g.dims.n)
    x = oracle_lib.aprod2(o, y)
    np.testing.assert_allclose(x, A.T @ y, rtol=1e-13, atol=1e-12)
    x2 = oracle_lib.aprod2(o, y, x=x0, scale=2.5)
    np.testing.assert_allclose(x2, 2.5 * x0 + A.T @ y, rtol=1e-13, atol=1e-12)


def test_scale_zero_does_not_read_output(small_sys, oracle_lib):
    g, o, A = small_sys
    x = np.ones(g.dims.n)
    y = oracle_lib.aprod1(o, x, y=np.full(g.dims.m, np.nan), scale=0.0)
    assert np.all(np.isfinite(y))
    z = oracle_lib.aprod2(o, np.ones(g.dims.m), x=np.full(g.dims.n, np.nan), scale=0.0)
    assert np.all(np.isfinite(z))


def test_adjoint_identity(oracle_lib):
    """<A x, y> = <x, A^T y> on the 1,000-star system."""
    g = gsr_synth.tiny()
    o = oracle_lib.OSystem(g)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(g.dims.n)
    y = rng.standard_normal(g.dims.m)
    lhs = math.fsum(oracle_lib.aprod1(o, x) * y)
    rhs = math.fsum(x * oracle_lib.aprod2(o, y))
    assert abs(lhs - rhs) <= 1e-13 * math.sqrt(math.fsum((oracle_lib.aprod1(o, x) * y) ** 2)) * 30


def test_row_sums_independent_of_column_map(oracle_lib):
    """A 1 is the row sum of the coefficients, whatever the column of each slot."""
    g = gsr_synth.tiny()
    o = oracle_lib.OSystem(g)
    y = oracle_lib.aprod1(o, np.ones(g.dims.n))
    ref = np.array([math.fsum(r) for r in g.vals])
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13)


def test_unit_vectors(small_sys, oracle_lib):
    """A e_j is column j of the dense matrix; A^T e_r is row r."""
    g, o, A = small_sys
    for j in [0, 4, g.dims.n_astro, g.dims.n_astro + g.dims.n_att + 1, g.dims.n - 1]:
        e = np.zeros(g.dims.n)
        e[j] = 1.0
        np.testing.assert_array_equal(oracle_lib.aprod1(o, e), A[:, j])
    for r in [0, g.dims.m // 2, g.dims.m - 1]:
        e = np.zeros(g.dims.m)
        e[r] = 1.0
        np.testing.assert_array_equal(oracle_lib.aprod2(o, e), A[r, :])


def test_aprod2_compensated_sum_is_accurate(oracle_lib):
    """Columns with many cancelling terms are summed to (nearly) correct rounding:
    compare with math.fsum of the exact products."""
    g = gsr_synth.make_system(200, 50, 8, 6, 1, seed=5)
    o = oracle_lib.OSystem(g)
    rng = np.random.default_rng(4)
    y = rng.standard_normal(g.dims.m) * np.exp(rng.uniform(-10, 10, g.dims.m))
    x = oracle_lib.aprod2(o, y)
    glob = g.dims.n - 1
    exact = math.fsum(g.vals[:, 23] * y)  # each product is exact-rounded in both
    assert abs(x[glob] - exact) <= 2 * np.spacing(abs(exact)) + 1e-300


def test_colnorms_vs_dense(small_sys, oracle_lib):
    g, o, A = small_sys
    np.testing.assert_allclose(oracle_lib.colnorms(o), np.sqrt((A * A).sum(0)), rtol=1e-14)


def test_fp32_products(small_sys, oracle_lib):
    """FP32 form: each product fl32(fl32(a) * fl32(x)) is formed in FP32 and summed in FP64."""
    g, _, A = small_sys
    g32 = g.as_f32()
    o = oracle_lib.OSystem(g32)
    A32 = dense_A(g32).astype(np.float32)
    rng = np.random.default_rng(6)
    x = rng.standard_normal(g.dims.n)
    P = (A32 * x.astype(np.float32)[None, :]).astype(np.float64)  # FP32 products, exact upcast
    ref = np.array([math.fsum(r) for r in P])
    np.testing.assert_allclose(oracle_lib.aprod1(o, x, mode=oracle_lib.P32), ref, rtol=0, atol=1e-13)
    y = rng.standard_normal(g.dims.m)
    Q = (A32 * y.astype(np.float32)[:, None]).astype(np.float64)
    ref2 = np.array([math.fsum(c) for c in Q.T])
    np.testing.assert_allclose(oracle_lib.aprod2(o, y, mode=oracle_lib.P32), ref2, rtol=0, atol=1e-12)
    # FP64 products on FP32 storage are the exact upcast
    np.testing.assert_allclose(oracle_lib.aprod1(o, x), A32.astype(np.float64) @ x, rtol=1e-13, atol=1e-12)


def test_threads_do_not_change_results(oracle_lib):
    """The threaded oracle splits aprod 1 by stars and the column sums by fixed
    chunks of stars, so its results are bit for bit the same for any thread count;
    with more stars than chunks every column sum still lands within two units in
    the last place of the exactly rounded sum (math.fsum of the exact products)."""
    g = gsr_synth.make_system(500, (5, 30), 40, 12, 1, seed=12)
    o = oracle_lib.OSystem(g)
    rng = np.random.default_rng(13)
    x = rng.standard_normal(g.dims.n)
    y = rng.standard_normal(g.dims.m) * np.exp(rng.uniform(-8, 8, g.dims.m))
    out = {}
    try:
        for t in (1, 3, 8):
            oracle_lib.set_threads(t)
            out[t] = (oracle_lib.aprod1(o, x), oracle_lib.aprod2(o, y), oracle_lib.colnorms(o))
    finally:
        oracle_lib.set_threads(0)
    for t in (3, 8):
        for a, b in zip(out[t], out[1]):
            assert np.array_equal(a, b), t
    A = dense_A(g)
    exact = np.array([math.fsum(c) for c in (A * y[:, None]).T])
    got = out[8][1]
    assert np.all(np.abs(got - exact) <= 2 * np.spacing(np.abs(exact)) + 1e-300)
