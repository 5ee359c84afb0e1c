"""Pins of the oracle's LSQR, variances and covariances against dense least
squares, the damped augmented system, scipy's independent LSQR, the
identity-solution property of the paper's synthetic data (Sec. 3) and the
invariants of the covariance accumulation (Eq. 4)."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.linalg import lsqr as scipy_lsqr

import gsr_synth
from tests._dense import dense_A


def _small(seed=7, **kw):
    args = dict(n_stars=40, obs=12, n_att=16, n_instr=8, n_glob=1, seed=seed)
    args.update(kw)
    return gsr_synth.make_system(**args)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("precond", [False, True])
def test_lsqr_matches_dense_least_squares(oracle_lib, precond):
    g = _small()
    o = oracle_lib.OSystem(g)
    A = dense_A(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    x_ls = np.linalg.lstsq(A, b, rcond=None)[0]
    r = oracle_lib.lsqr(o, b, atol=1e-14, btol=1e-14, itmax=2000, precond=precond)
    assert r["istop"] in (1, 2)
    assert _rel(r["x"], x_ls) < 1e-10


@pytest.mark.parametrize("precond", [False, True])
def test_damped_lsqr_matches_augmented_system(oracle_lib, precond):
    g = _small(seed=17)
    o = oracle_lib.OSystem(g)
    A = dense_A(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    damp = 0.7
    S = 1.0 / np.sqrt((A * A).sum(0)) if precond else np.ones(g.dims.n)
    Aug = np.vstack([A * S[None, :], damp * np.eye(g.dims.n)])
    y_ls = np.linalg.lstsq(Aug, np.concatenate([b, np.zeros(g.dims.n)]), rcond=None)[0]
    r = oracle_lib.lsqr(o, b, damp=damp, atol=1e-14, btol=1e-14, itmax=2000, precond=precond)
    assert _rel(r["x"], S * y_ls) < 1e-10


def test_identity_solution(oracle_lib):
    """Sec. 3: with x_true = 1 and noise-free known terms the solver finds the identity solution."""
    g = gsr_synth.tiny(x_kind="ones", noise_std=0.0)
    o = oracle_lib.OSystem(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    r = oracle_lib.lsqr(o, b, atol=1e-12, btol=1e-12, itmax=500, precond=True)
    assert r["istop"] == 1
    assert np.max(np.abs(r["x"] - 1.0)) < 1e-9


def test_istop2_means_small_normal_residual(oracle_lib):
    g = _small(seed=21)
    o = oracle_lib.OSystem(g)
    A = dense_A(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise * 1e4)  # clearly inconsistent
    atol = 1e-10
    r = oracle_lib.lsqr(o, b, atol=atol, btol=1e-14, itmax=2000, precond=False)
    assert r["istop"] == 2
    res = b - A @ r["x"]
    arnorm_true = np.linalg.norm(A.T @ res)
    assert arnorm_true / (r["anorm"] * np.linalg.norm(res)) <= 2 * atol
    assert abs(np.linalg.norm(res) - r["rnorm"]) <= 1e-6 * r["rnorm"]


@pytest.mark.parametrize("damp", [0.0, 0.3])
@pytest.mark.parametrize("k", [1, 7, 15])
def test_iterates_match_scipy_lsqr(oracle_lib, damp, k):
    """scipy's LSQR is an independent implementation of the same method.  Iterate counts
    stay below the point where loss of orthogonality makes the iterates themselves
    sensitive to rounding (about 1e-8 at 25 iterations on this system)."""
    g = _small(seed=31)
    o = oracle_lib.OSystem(g)
    A = dense_A(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    xs = scipy_lsqr(sp.csr_matrix(A), b, damp=damp, atol=0.0, btol=0.0, conlim=0.0, iter_lim=k)[0]
    r = oracle_lib.lsqr(o, b, damp=damp, atol=0.0, btol=0.0, itmax=k, precond=False)
    assert r["itn"] == k and r["istop"] == 7
    assert _rel(r["x"], xs) < 1e-11


def test_preconditioned_iterates_match_scipy_on_scaled_matrix(oracle_lib):
    g = _small(seed=33)
    o = oracle_lib.OSystem(g)
    A = dense_A(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    S = 1.0 / np.sqrt((A * A).sum(0))
    ys = scipy_lsqr(sp.csr_matrix(A * S[None, :]), b, atol=0.0, btol=0.0, conlim=0.0, iter_lim=12)[0]
    r = oracle_lib.lsqr(o, b, atol=0.0, btol=0.0, itmax=12, precond=True)
    assert _rel(r["x"], S * ys) < 1e-11
    np.testing.assert_allclose(r["scale"], S, rtol=1e-14)


def test_stopping_iteration_matches_scipy(oracle_lib):
    g = _small(seed=35)
    o = oracle_lib.OSystem(g)
    A = dense_A(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise * 1e3)
    out = scipy_lsqr(sp.csr_matrix(A), b, atol=1e-8, btol=1e-8, iter_lim=5000)
    r = oracle_lib.lsqr(o, b, atol=1e-8, btol=1e-8, itmax=5000, precond=False)
    assert r["istop"] == out[1] == 2
    assert abs(r["itn"] - out[2]) <= 1


def test_tiny_system_converges_to_qr_solution(oracle_lib):
    """The 1,000-star system (20,000 x 5,225), column-scaled, to 1e-10 of dense QR."""
    g = gsr_synth.tiny()
    o = oracle_lib.OSystem(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    A = dense_A(g)
    Q, R = np.linalg.qr(A)
    x_qr = np.linalg.solve(R, Q.T @ b)
    del Q
    r = oracle_lib.lsqr(o, b, atol=1e-12, btol=1e-12, itmax=400, precond=True)
    assert r["istop"] in (1, 2)
    assert _rel(r["x"], x_qr) < 1e-10
    # noise-limited distance to the true solution
    assert _rel(r["x"], g.x_true) < 1e-5


def test_edge_cases(oracle_lib):
    g = _small(seed=41)
    o = oracle_lib.OSystem(g)
    r = oracle_lib.lsqr(o, np.zeros(g.dims.m), itmax=50)
    assert r["istop"] == 0 and r["itn"] == 0 and np.all(r["x"] == 0)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    r = oracle_lib.lsqr(o, b, atol=0, btol=0, itmax=3)
    assert r["istop"] == 7 and r["itn"] == 3
    # x0 equal to the solution of an exact system: nothing left to do
    x0 = g.x_true.copy()
    b0 = oracle_lib.known_terms(o, x0, np.zeros(g.dims.m))
    r = oracle_lib.lsqr(o, b0, x0=x0, itmax=50)
    assert r["itn"] == 0 and np.array_equal(r["x"], x0)


def test_warm_start_converges_to_same_solution_faster(oracle_lib):
    g = _small(seed=43)
    o = oracle_lib.OSystem(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    cold = oracle_lib.lsqr(o, b, atol=1e-13, btol=1e-13, itmax=3000)
    x0 = cold["x"] + 1e-4 * np.random.default_rng(0).standard_normal(g.dims.n)
    warm = oracle_lib.lsqr(o, b, x0=x0, atol=1e-13, btol=1e-13, itmax=3000)
    assert _rel(warm["x"], cold["x"]) < 1e-10
    assert warm["itn"] < cold["itn"]


def _golub_kahan_cov(As, b, k):
    """V_k (B_k^T B_k)^{-1} V_k^T from a Golub-Kahan bidiagonalisation with full
    reorthogonalisation (dense, independent of the oracle).  In exact arithmetic
    this is sum_{i<=k} d_i d_i^T for the LSQR search directions d_i = w_i / rho_i."""
    m, n = As.shape
    U = [b / np.linalg.norm(b)]
    v = As.T @ U[0]
    alphas = [np.linalg.norm(v)]
    V = [v / alphas[0]]
    betas = []
    for i in range(k):
        u = As @ V[-1] - alphas[-1] * U[-1]
        for q in U:
            u -= (q @ u) * q
        betas.append(np.linalg.norm(u))
        U.append(u / betas[-1])
        v = As.T @ U[-1] - betas[-1] * V[-1]
        for q in V:
            v -= (q @ v) * q
        alphas.append(np.linalg.norm(v))
        V.append(v / alphas[-1])
    B = np.zeros((k + 1, k))
    for i in range(k):
        B[i, i] = alphas[i]
        B[i + 1, i] = betas[i]
    Vk = np.array(V[:k]).T
    return Vk @ np.linalg.inv(B.T @ B) @ Vk.T


@pytest.mark.parametrize("precond", [False, True])
def test_variances_and_covariances_match_bidiagonalisation(oracle_lib, precond):
    """var and C after k iterations equal S V_k (B_k^T B_k)^{-1} V_k^T S (diagonal / selected block)."""
    g = _small(seed=51, n_stars=20, obs=30)
    o = oracle_lib.OSystem(g)
    A = dense_A(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    S = 1.0 / np.sqrt((A * A).sum(0)) if precond else np.ones(g.dims.n)
    sel = np.array([0, 3, 7, 50, g.dims.n_astro + 2, g.dims.n_astro + 20, g.dims.n - 2, g.dims.n - 1])
    k = 10
    r = oracle_lib.lsqr(o, b, atol=0, btol=0, itmax=k, precond=precond, sel=sel)
    assert r["itn"] == k
    M = S[:, None] * _golub_kahan_cov(A * S[None, :], b, k) * S[None, :]
    assert _rel(r["var"], np.diag(M)) < 1e-10
    assert _rel(r["cov"], M[np.ix_(sel, sel)]) < 1e-10


def test_variances_match_scipy(oracle_lib):
    g = _small(seed=52, n_stars=20, obs=30)
    o = oracle_lib.OSystem(g)
    A = dense_A(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    out = scipy_lsqr(sp.csr_matrix(A), b, atol=0, btol=0, conlim=0, iter_lim=12, calc_var=True)
    r = oracle_lib.lsqr(o, b, atol=0, btol=0, itmax=12, precond=False)
    assert _rel(r["var"], out[-1]) < 1e-11


def test_variances_monotone_and_covariance_invariants(oracle_lib):
    g = _small(seed=53, n_stars=20, obs=30)
    o = oracle_lib.OSystem(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    r5 = oracle_lib.lsqr(o, b, atol=0, btol=0, itmax=5, precond=True)
    r9 = oracle_lib.lsqr(o, b, atol=0, btol=0, itmax=9, precond=True)
    assert np.all(r9["var"] >= r5["var"])
    sel = np.arange(0, g.dims.n, 7)
    r = oracle_lib.lsqr(o, b, atol=1e-12, btol=1e-12, itmax=500, precond=True, sel=sel)
    Cv = r["cov"]
    np.testing.assert_array_equal(Cv, Cv.T)
    np.testing.assert_allclose(np.diag(Cv), r["var"][sel], rtol=1e-14)
    assert np.linalg.eigvalsh(Cv).min() >= -1e-14 * np.abs(Cv).max()


def test_fp32_refinement_reaches_fp64_solution(oracle_lib):
    g = gsr_synth.tiny().as_f32()
    o = oracle_lib.OSystem(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    ref = oracle_lib.lsqr(o, b, atol=1e-13, btol=1e-13, itmax=500, precond=True)
    plain32 = oracle_lib.lsqr(o, b, atol=1e-13, btol=1e-13, itmax=500, precond=True, mode=oracle_lib.P32)
    e32 = _rel(plain32["x"], ref["x"])
    assert 1e-9 < e32 < 1e-4  # FP32 products alone stall well above 1e-10
    ref_out = oracle_lib.lsqr_refine(o, b, inner_atol=1e-6, inner_btol=1e-6, outer_max=10, outer_tol=1e-11)
    assert ref_out["outer_steps"] >= 2
    assert _rel(ref_out["x"], ref["x"]) < 1e-10


@pytest.mark.parametrize("inner_tol", [1e-5, 1e-6, 1e-7])
def test_refinement_stop_rule_predicts_the_next_correction(oracle_lib, inner_tol):
    """The refinement stops when the correction, or the next one predicted from the
    contraction between the last two, is at most outer_tol ||x||.  Pin of that rule:
    one more outer step taken by hand (residual with FP64 products, inner FP32-product
    LSQR, as the loop does) gives a correction within 10 outer_tol ||x||."""
    g = gsr_synth.tiny().as_f32()
    o = oracle_lib.OSystem(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    tol = 1e-11
    out = oracle_lib.lsqr_refine(o, b, inner_atol=inner_tol, inner_btol=inner_tol, outer_max=10, outer_tol=tol)
    x = out["x"]
    r = b - oracle_lib.aprod1(o, x)
    dx = oracle_lib.lsqr(o, r, atol=inner_tol, btol=inner_tol, itmax=1000, precond=True, mode=oracle_lib.P32)["x"]
    nxt = np.linalg.norm(dx) / np.linalg.norm(x)
    assert out["outer_steps"] < 10  # stopped by the rule, not by outer_max
    assert nxt <= 10 * tol, nxt


def _scipy_out(A, b, **kw):
    out = scipy_lsqr(sp.csr_matrix(A), b, **kw)
    keys = ("x", "istop", "itn", "r1norm", "r2norm", "anorm", "acond", "arnorm", "xnorm", "var")
    return dict(zip(keys, out))


@pytest.mark.parametrize("damp", [0.0, 0.4])
@pytest.mark.parametrize("k", [3, 9, 15])
def test_estimates_match_scipy(oracle_lib, damp, k):
    """The Paige-Saunders estimates after k iterations -- the Frobenius estimate anorm,
    the condition estimate acond = anorm ||D_k||_F (D_k the search directions d_i =
    w_i / rho_i), rnorm of the damped problem and ||A^T r|| -- against scipy's
    independent LSQR, before loss of orthogonality makes the iterates (and with them
    alpha_i, beta_i and every estimate) depend on rounding."""
    g = _small(seed=71)
    o = oracle_lib.OSystem(g)
    A = dense_A(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    s = _scipy_out(A, b, damp=damp, atol=0.0, btol=0.0, conlim=0.0, iter_lim=k)
    r = oracle_lib.lsqr(o, b, damp=damp, atol=0.0, btol=0.0, itmax=k, precond=False)
    assert r["itn"] == s["itn"] == k and r["istop"] == s["istop"] == 7
    for ok, sk in (("anorm", "anorm"), ("acond", "acond"), ("rnorm", "r2norm"), ("arnorm", "arnorm")):
        assert abs(r[ok] - s[sk]) <= 1e-12 * abs(s[sk]), (ok, r[ok], s[sk])


def test_acond_is_frobenius_of_the_bidiagonal_inverse(oracle_lib):
    """acond = anorm * ||D_k||_F where D_k = V_k R_k^{-1} and the Golub-Kahan closed form
    gives ||D_k||_F^2 = trace(V_k (B_k^T B_k)^{-1} V_k^T) = trace((B_k^T B_k)^{-1}); anorm
    is the Frobenius norm of B_k (sum of alpha_i^2 + beta_{i+1}^2).  Checked against
    the dense bidiagonalisation with full reorthogonalisation."""
    g = _small(seed=72, n_stars=20, obs=30)
    o = oracle_lib.OSystem(g)
    A = dense_A(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    k = 10
    r = oracle_lib.lsqr(o, b, atol=0, btol=0, itmax=k, precond=False)
    M = _golub_kahan_cov(A, b, k)
    assert abs(r["acond"] / r["anorm"] - np.sqrt(np.trace(M))) <= 1e-10 * np.sqrt(np.trace(M))


def test_conlim_stop_matches_scipy(oracle_lib):
    """conlim > 0 (ctol = 1/conlim): the solve stops with istop 3 at the first iteration
    whose condition estimate reaches conlim; the stop iteration, x and the estimates
    agree with scipy's LSQR (Paige-Saunders stop rules, lowest-numbered test first)."""
    g = _small(seed=61)
    o = oracle_lib.OSystem(g)
    A = dense_A(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    s = _scipy_out(A, b, atol=1e-14, btol=1e-14, conlim=30.0, iter_lim=3000)
    r = oracle_lib.lsqr(o, b, atol=1e-14, btol=1e-14, conlim=30.0, itmax=3000, precond=False)
    assert r["istop"] == s["istop"] == 3
    assert r["itn"] == s["itn"]
    assert r["acond"] >= 30.0 and s["acond"] >= 30.0
    assert abs(r["acond"] - s["acond"]) <= 1e-12 * s["acond"]
    assert _rel(r["x"], s["x"]) < 1e-11
    # without the limit the same system runs on (and its estimate passes conlim)
    r2 = oracle_lib.lsqr(o, b, atol=1e-14, btol=1e-14, conlim=0.0, itmax=3000, precond=False)
    assert r2["istop"] != 3 and r2["itn"] > r["itn"]


@pytest.mark.parametrize("case,expect", [("consistent", 4), ("inconsistent", 5)])
def test_machine_precision_stops_match_scipy(oracle_lib, case, expect):
    """atol = btol = 0: a consistent system stops on the machine-precision form of test 1
    (istop 4), a clearly inconsistent one on that of test 2 (istop 5), as in scipy.  The
    stop iterations lie far past the loss of orthogonality, so they agree to a few
    iterations only."""
    if case == "consistent":
        g = _small(seed=62)
        nf = 0.0
    else:
        g = _small(seed=63)
        nf = 1e4
    o = oracle_lib.OSystem(g)
    A = dense_A(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise * nf)
    s = _scipy_out(A, b, atol=0.0, btol=0.0, conlim=0.0, iter_lim=3000)
    r = oracle_lib.lsqr(o, b, atol=0.0, btol=0.0, conlim=0.0, itmax=3000, precond=False)
    assert r["istop"] == s["istop"] == expect
    assert abs(r["itn"] - s["itn"]) <= 0.05 * s["itn"]
    x_ls = np.linalg.lstsq(A, b, rcond=None)[0]
    assert _rel(r["x"], x_ls) < 1e-12


@pytest.mark.parametrize("damp", [0.0, 0.3])
@pytest.mark.parametrize("k", [1, 7, 15])
def test_one_pass_order_matches_scipy_lsqr(oracle_lib, damp, k):
    """The one-pass order (A^T applied to the unnormalised u', divided by beta
    afterwards; mode P64_1P) is the same LSQR: its iterates meet scipy's independent
    LSQR at the bar of the textbook order."""
    g = _small(seed=31)
    o = oracle_lib.OSystem(g)
    A = dense_A(g)
    b = oracle_lib.known_terms(o, g.x_true, g.noise)
    xs = scipy_lsqr(sp.csr_matrix(A), b, damp=damp, atol=0.0, btol=0.0, conlim=0.0, iter_lim=k)[0]
    r = oracle_lib.lsqr(o, b, damp=damp, atol=0.0, btol=0.0, itmax=k, precond=False, mode=oracle_lib.P64_1P)
    assert r["itn"] == k and r["istop"] == 7
    assert _rel(r["x"], xs) < 1e-11


def test_one_pass_fp32_products_round_the_unnormalised_operand(oracle_lib):
    """FP32 products in the one-pass order (mode P32_1P) round u'_r where the textbook
    order (P32) rounds u'_r / beta.  With b = 1 on 1,024 rows, beta_1 = 32 and
    u_1 = b / 32 are exact, so both orders round exactly the same operands in the
    first step and agree bit for bit after one iteration; from the second on the
    operands differ and so do the iterates, both by the size of the FP32 product
    effect (their distance from FP64 products)."""
    g = _small(seed=33, n_stars=64, obs=16).as_f32()
    assert g.dims.m == 1024
    o = oracle_lib.OSystem(g)
    b = np.ones(g.dims.m)
    kw = dict(atol=0.0, btol=0.0, precond=False)
    r1 = oracle_lib.lsqr(o, b, itmax=1, mode=oracle_lib.P32, **kw)
    q1 = oracle_lib.lsqr(o, b, itmax=1, mode=oracle_lib.P32_1P, **kw)
    assert np.array_equal(r1["x"], q1["x"]) and np.array_equal(r1["var"], q1["var"])
    r = oracle_lib.lsqr(o, b, itmax=6, mode=oracle_lib.P32, **kw)
    q = oracle_lib.lsqr(o, b, itmax=6, mode=oracle_lib.P32_1P, **kw)
    f = oracle_lib.lsqr(o, b, itmax=6, mode=oracle_lib.P64, **kw)
    d = _rel(q["x"], r["x"])
    e32, e1p = _rel(r["x"], f["x"]), _rel(q["x"], f["x"])
    assert d > 0
    assert 0.1 * e32 < e1p < 10 * e32 and d < 10 * e32
