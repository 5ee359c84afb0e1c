"""Pins of the FP64 warm-start network reference: gradients against central
finite differences, the closed form of Adam's first step, and the per-star
features against dense brute force."""
import numpy as np
import pytest

import gsr_synth
from oracle import mlp as omlp
from tests._dense import dense_A


def _net(seed=11, n_in=28, h=16, n_out=5):
    return gsr_synth.mlp_init(n_in, h, n_out, seed=seed)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    P = _net()
    P = [p + 0.1 * rng.standard_normal(p.shape) for p in P]  # non-zero biases too
    X = rng.standard_normal((37, 28))
    T = rng.standard_normal((37, 5))
    L, G = omlp.grads(P, X, T)
    assert abs(L - omlp.loss(P, X, T)) < 1e-15
    h = 1e-6
    for pi, p in enumerate(P):
        flat = p.reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = omlp.loss(P, X, T)
            flat[idx] = old - h
            lm = omlp.loss(P, X, T)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            g = G[pi].reshape(-1)[idx]
            assert abs(fd - g) <= 1e-7 * max(1.0, abs(g)), (pi, idx, fd, g)


def test_adam_first_step_closed_form():
    """After one step from zero moments the bias-corrected update is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    P = _net()
    G = [rng.standard_normal(p.shape) for p in P]
    opt = omlp.Adam(P, lr=1e-3)
    P1 = opt.step(P, G)
    for p, p1, g in zip(P, P1, G):
        np.testing.assert_allclose(p - p1, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)


def test_training_reduces_loss():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((256, 28))
    W = rng.standard_normal((28, 5))
    T = np.tanh(X @ W / 5)
    P = _net(h=32)
    opt = omlp.Adam(P, lr=3e-3)
    l0 = omlp.loss(P, X, T)
    for _ in range(300):
        _, G = omlp.grads(P, X, T)
        P = opt.step(P, G)
    assert omlp.loss(P, X, T) < 0.1 * l0


def test_standardize_stats():
    X = np.array([[1.0, 5.0], [3.0, 5.0]])
    mu, sd = omlp.standardize_stats(X)
    np.testing.assert_array_equal(mu, [2.0, 5.0])
    np.testing.assert_array_equal(sd, [1.0, 1.0])


@pytest.mark.parametrize("n_glob", [1, 0])
def test_features_vs_dense(oracle_lib, n_glob):
    g = gsr_synth.make_system(30, (4, 15), 8, 7, n_glob, seed=12)
    o = oracle_lib.OSystem(g)
    A = dense_A(g)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(g.dims.m)
    NA = g.dims.n_astro
    xo = rng.standard_normal(g.dims.n - NA)
    F = oracle_lib.features(o, b, xo)
    bt = b - A[:, NA:] @ xo
    iu = np.triu_indices(5)
    for s in range(g.dims.n_stars):
        r0, r1 = g.star_row_ptr[s], g.star_row_ptr[s + 1]
        As = A[r0:r1, 5 * s: 5 * s + 5]
        np.testing.assert_allclose(F[s, :15], (As.T @ As)[iu], rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(F[s, 15:20], As.T @ bt[r0:r1], rtol=1e-12, atol=1e-12)
        rows = r1 - r0
        at = g.att_start[r0:r1] / g.dims.n_att
        assert F[s, 20] == rows
        np.testing.assert_allclose(F[s, 21:23], [at.mean(), at.std()], rtol=1e-13, atol=1e-15)
        V = g.vals[r0:r1]
        np.testing.assert_allclose(F[s, 23], np.sqrt((V[:, 5:17] ** 2).mean()), rtol=1e-13)
        np.testing.assert_allclose(F[s, 24], np.sqrt((V[:, 17:23] ** 2).mean()), rtol=1e-13)
        np.testing.assert_allclose(F[s, 25], np.sqrt((V[:, 23] ** 2).mean()) if n_glob else 0.0, rtol=1e-13)
        np.testing.assert_allclose(F[s, 26], np.linalg.norm(bt[r0:r1]) / np.sqrt(rows), rtol=1e-12)
        ref27 = (V[:, 23] * bt[r0:r1]).sum() / rows if n_glob else 0.0
        np.testing.assert_allclose(F[s, 27], ref27, rtol=1e-11, atol=1e-13)
