"""Learned warm start: features, network gradients and Adam against the CPU
oracle, and the gain of the trained network over zero-start LSQR on a family
of related systems (same matrix, x_true perturbed by 0.05 N(0,1), fresh noise)."""
import numpy as np
import pytest
import torch

import gsr_synth
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def dev():
    import paper_2503_22863_amd as gsr

    gsr.lib()
    return gsr


@pytest.mark.parametrize("f32", [False, True])
def test_features_match_oracle(dev, oracle_lib, f32):
    print(f"[features] f32={f32}", flush=True)
    g = gsr_synth.make_system(300, (1, 40), 24, 10, 1, seed=21)
    if f32:
        g = g.as_f32()
    o = oracle_lib.OSystem(g)
    rng = np.random.default_rng(0)
    b = rng.standard_normal(g.dims.m)
    xo = rng.standard_normal(g.dims.n - g.dims.n_astro)
    S = dev.System.from_generated(g)
    F = S.features(torch.from_numpy(b).cuda(), torch.from_numpy(xo).cuda()).cpu().numpy()
    ref = oracle_lib.features(o, b, xo)
    for c in range(28):
        assert _rel(F[:, c], ref[:, c]) <= 1e-12, c
    S.close()


def _std(X):
    mu, sd = omlp.standardize_stats(X)
    return (X - mu) / sd


def test_gradients_match_oracle(dev):
    print("[mlp] gradients", flush=True)
    rng = np.random.default_rng(1)
    N, I, H, O = 3000, 28, 128, 5
    X = rng.standard_normal((N, I)) * rng.uniform(0.5, 20, I) + rng.uniform(-5, 5, I)
    T = np.tanh(X[:, :O] / 10) + 0.1 * rng.standard_normal((N, O))
    P = gsr_synth.mlp_init(I, H, O, seed=5)
    P = [p + 0.05 * rng.standard_normal(p.shape) for p in P]
    P32 = [p.astype(np.float32).astype(np.float64) for p in P]  # the network runs on FP32-rounded weights
    net = dev.MLP(P)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    net.fit_norm(Xd, Td)
    loss, g = net.grad(Xd, Td)
    L_ref, G_ref = omlp.grads(P32, _std(X), _std(T))
    assert abs(loss - L_ref) <= 1e-5 * L_ref
    g = g.cpu().numpy().astype(np.float64)
    o = 0
    for gi in G_ref:
        k = gi.size
        e = _rel(g[o:o + k], gi.reshape(-1))
        assert e <= 1e-4, (o, e)
        o += k
    net.close()


def test_adam_steps_match_oracle(dev):
    print("[mlp] Adam", flush=True)
    rng = np.random.default_rng(2)
    N, I, H, O = 1000, 28, 64, 5
    X = rng.standard_normal((N, I))
    T = rng.standard_normal((N, O))
    P = [p.astype(np.float32).astype(np.float64) for p in gsr_synth.mlp_init(I, H, O, seed=6)]
    net = dev.MLP(P)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    net.fit_norm(Xd, Td)
    net.train(Xd, Td, steps=3, lr=1e-3)
    opt = omlp.Adam(P, lr=1e-3)
    Xs, Ts = _std(X), _std(T)
    Q = P
    for _ in range(3):
        _, G = omlp.grads(Q, Xs, Ts)
        Q = opt.step(Q, G)
    got = net.params()
    for a, b, p0 in zip(got, Q, P):
        d = np.abs(a - b)
        # a step is about lr * sign(g); allow FP32 rounding, and sign flips only where g ~ 0
        assert np.mean(d > 1e-6) <= 2e-3
        assert _rel(a - p0, b - p0) <= 2e-2
    net.close()


def test_warm_start_gain(dev, oracle_lib):
    """Train on the LSQR solutions of systems 0-7 of a family built on the 1,000-star
    system; warm-start systems 8-15.  Iterations to reach the oracle's solution to
    1e-10 from the zero start, from the mean of the training solutions (the
    non-learned ablation) and from the network's x0.  The warm start must beat the
    zero start.  On this family the network ties the mean start: a member differs
    from the mean by a perturbation of every unknown, and a star's features see the
    attitude and instrumental part of it at the size of the star's own part, so they
    cannot resolve the star's unknowns better than the mean does.  The test asserts
    that the network loses nothing against the mean (at most one iteration per
    system) and reports the gain."""
    print("[warm start] family of the 1,000-star system", flush=True)
    base = gsr_synth.tiny()
    o = oracle_lib.OSystem(base)
    S = dev.System.from_generated(base)
    ns, n = base.dims.n_stars, base.dims.n
    opts = dict(atol=1e-12, btol=1e-12, itmax=300, precond=True)
    sols, bs = [], []
    for s in range(16):
        fm = gsr_synth.family_member(base, s)
        b = oracle_lib.known_terms(o, fm.x_true, fm.noise)
        bs.append(torch.from_numpy(b).cuda())
        if s < 8:
            x, _, r = S.lsqr_solve(bs[-1], **opts)
            sols.append(x)
    Xs = torch.stack(sols)
    x_mean = dev.mean_rows(Xs)
    xo = x_mean[5 * ns:].contiguous()
    F = torch.cat([S.features(bs[s], xo) for s in range(8)])
    T = torch.cat([sols[s][: 5 * ns].reshape(ns, 5) for s in range(8)])
    net = dev.MLP(gsr_synth.mlp_init(28, 128, 5, seed=11))
    net.fit_norm(F, T)
    loss = net.train(F, T, steps=1500, lr=1e-3)
    print(f"  training loss (standardised) {loss:.3e}", flush=True)
    assert loss < 0.5

    def iters_to(b, x0, x_ref, tol=1e-10, cap=300):
        S.lsqr_begin(b, x0=x0, atol=0, btol=0, itmax=cap, precond=True)
        for it in range(1, cap + 1):
            S.lsqr_iterate(1)
            if _rel(S.lsqr_peek().cpu().numpy(), x_ref) <= tol:
                S.lsqr_end()
                return it
        S.lsqr_end()
        return cap + 1

    ks = []
    for s in range(8, 16):
        ref = oracle_lib.lsqr(o, bs[s].cpu().numpy(), atol=1e-14, btol=1e-14, itmax=1000, precond=True)["x"]
        x0 = torch.empty(n, dtype=torch.float64, device="cuda")
        x0[: 5 * ns] = net.forward(S.features(bs[s], xo)).reshape(-1)
        x0[5 * ns:] = xo
        xw, _, rw = S.lsqr_solve(bs[s], x0=x0, **opts)
        assert _rel(xw.cpu().numpy(), ref) <= 1e-10
        k_zero = iters_to(bs[s], None, ref)
        k_mean = iters_to(bs[s], x_mean, ref)
        k_mlp = iters_to(bs[s], x0, ref)
        print(f"  system {s}: iterations to 1e-10  zero {k_zero}  mean-x0 {k_mean}  mlp-x0 {k_mlp}", flush=True)
        ks.append((k_zero, k_mean, k_mlp))
        assert k_mlp <= k_mean + 1
    kz, km, kn = (float(np.mean(c)) for c in zip(*ks))
    print(f"  mean over systems 8-15: zero {kz:.3f}  mean-x0 {km:.3f}  mlp-x0 {kn:.3f}  "
          f"(network vs mean start: {km - kn:+.3f} iterations)", flush=True)
    assert kn < kz
    net.close()
    S.close()
