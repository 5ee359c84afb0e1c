"""Comparison helpers shared by the GPU parity tests (test helper).

Products (Eq. 2 and Eq. 3) are held to the 1e-13 normwise bar per block
(astrometric, attitude, instrumental, global and overall) and, element by
element, to 64 eps times the same sum taken over absolute values, which the
oracle computes on |coefficients|:
    |y_gpu - y_ref| <= 64 eps (|A| |x| + |s| |y0|)          (aprod 1)
    |x_gpu - x_ref| <= 64 eps (|A|^T |y| + |s| |x0|)        (aprod 2)
With FP32 products the oracle forms each product in FP32 from the same FP32
operands as the kernel (exact in both), so only the FP64 sums differ and the
same bars apply.
A floating-point sum of K terms is within about K u of that bound in the
worst case and within sqrt(K) u typically (u = eps / 2); the oracle's own
sums are compensated (aprod 2) or of 25 terms (aprod 1), so a correct kernel
sits at a few eps while a wrong index at one window, segment or tile
boundary moves single elements far past the bar.

LSQR iterates are held to max(floor, 10 s) per block, where s is the
oracle's own response to last-bit perturbations of b and of every
coefficient (two runs with b perturbed and one with A; at the full shares
the coefficients' last mantissa bits are flipped at random rather than
scaled by 1 + 2.2e-16 N(0,1); FP32 coefficients are data, not rounding, so
for them only b is perturbed, in more runs): past the first iterations the
iterates depend on the summation order itself.
"""
import copy
import time

import numpy as np

EPS = np.finfo(np.float64).eps


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def blocks(d):
    na = d.n_astro
    nt = na + 3 * d.n_att
    ni = nt + d.n_instr
    out = {"astro": slice(0, na), "att": slice(na, nt), "instr": slice(nt, ni), "all": slice(0, d.n)}
    if d.n_glob:
        out["glob"] = slice(ni, ni + 1)
    return out


def abs_system(oracle_lib, g):
    ga = copy.copy(g)
    ga.vals = np.abs(g.vals)
    return oracle_lib.OSystem(ga)


def _both(f1, f2):
    """Two oracle calls, one after the other (each uses every core)."""
    return f1(), f2()


def check_aprod1(oracle_lib, o, oa, x, y0, scale, y_gpu, tag, bar=1e-13, c=64, mode=0):
    """aprod 1 at the product bar: normwise and per element (mode: the oracle's
    product mode, FP64 or FP32 products).  Returns the oracle's y."""
    ref, bnd = _both(lambda: oracle_lib.aprod1(o, x, y=y0, scale=scale, mode=mode),
                     lambda: oracle_lib.aprod1(oa, np.abs(x), y=np.abs(y0), scale=abs(scale)))
    e = rel(y_gpu, ref)
    d = np.abs(y_gpu - ref)
    worst = float(np.max(d / np.maximum(bnd, 1e-300)))
    print(f"  {tag} aprod1 {e:.2e}, worst element {worst / EPS:.2f} eps of |A||x|", flush=True)
    assert e <= bar
    assert np.all(d <= c * EPS * bnd), int(np.argmax(d / np.maximum(bnd, 1e-300)))
    return ref


def check_aprod2(oracle_lib, g, o, oa, y, x0, scale, x_gpu, tag, bar=1e-13, c=64, mode=0):
    """aprod 2 at the product bar: normwise per block and per element (mode as for
    check_aprod1).  Returns the oracle's x."""
    ref, bnd = _both(lambda: oracle_lib.aprod2(o, y, x=x0, scale=scale, mode=mode),
                     lambda: oracle_lib.aprod2(oa, np.abs(y), x=np.abs(x0), scale=abs(scale)))
    for name, sl in blocks(g.dims).items():
        e = rel(x_gpu[sl], ref[sl])
        print(f"  {tag} aprod2 {name} {e:.2e}", flush=True)
        assert e <= bar, name
    d = np.abs(x_gpu - ref)
    worst = float(np.max(d / np.maximum(bnd, 1e-300)))
    print(f"  {tag} aprod2 worst element {worst / EPS:.2f} eps of |A|^T|y|", flush=True)
    assert np.all(d <= c * EPS * bnd), int(np.argmax(d / np.maximum(bnd, 1e-300)))
    return ref


def sensitivity(oracle_lib, g, o, b, nruns_b=2, **kw):
    """Reference run and the oracle's largest relative deviations, per block of x and
    var, and of the scalar estimates, over nruns_b runs with b perturbed at the last
    bit and one with A perturbed at the last bit.  The runs go one after the other
    (each uses every core), each reporting when it is done.  FP32 coefficients are
    the data itself (kernel and oracle read the same FP32 numbers, and a last-bit
    change of one is a 6e-8 change of the system), so for them only b is
    perturbed; with FP32 products the response comes from rare FP32 roundings of
    u' that flip, so such runs take more b perturbations."""
    t = time.time()
    bps = [b * (1 + 2e-16 * np.random.default_rng(seed).standard_normal(b.size)) for seed in range(5, 5 + nruns_b)]
    jobs = [("reference", o, b)] + [(f"b perturbed ({i + 1})", o, bp) for i, bp in enumerate(bps)]
    if g.vals.dtype == np.float32:
        return _runs(oracle_lib, g, jobs, kw)
    gp = copy.copy(g)
    gp.vals = g.vals.copy()
    rng = np.random.default_rng(7)
    if gp.vals.size <= 1 << 26:
        gp.vals *= 1 + 2.2e-16 * rng.standard_normal(gp.vals.shape)
    else:
        # the full shares: the last mantissa bit of each coefficient flipped with
        # probability 1/2 (a relative change of one unit in the last place), in
        # place, chunk by chunk -- one extra copy of A and no large temporaries
        bits = gp.vals.reshape(-1).view(np.uint64 if gp.vals.dtype == np.float64 else np.uint32)
        step = 1 << 26
        for i in range(0, bits.size, step):
            n = min(step, bits.size - i)
            bits[i:i + n] ^= rng.integers(0, 2, n, dtype=np.uint8).astype(bits.dtype)
    op = oracle_lib.OSystem(gp)
    print(f"  A perturbed at the last bit in {time.time() - t:.1f} s", flush=True)
    out = _runs(oracle_lib, g, jobs + [("A perturbed", op, b)], kw)
    del op, gp
    return out


def _runs(oracle_lib, g, jobs, kw):
    done = []
    for name, osys, rhs in jobs:
        t = time.time()
        done.append(oracle_lib.lsqr(osys, rhs, **kw))
        print(f"  oracle run ({name}) in {time.time() - t:.1f} s", flush=True)
    r1, runs = done[0], done[1:]
    sens = {}
    for name, sl in blocks(g.dims).items():
        sens[("x", name)] = max(rel(r["x"][sl], r1["x"][sl]) for r in runs)
        sens[("var", name)] = max(rel(r["var"][sl], r1["var"][sl]) for r in runs)
    for k in ("rnorm", "anorm", "xnorm"):
        sens[k] = max(abs(r[k] - r1[k]) / max(abs(r1[k]), 1e-300) for r in runs)
    if "cov" in r1:
        sens["cov"] = max(rel(r["cov"], r1["cov"]) for r in runs)
    return r1, sens
