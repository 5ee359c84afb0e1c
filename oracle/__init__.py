"""CPU reference ("oracle") for the AVU-GSR solver hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  It shares no code with the HIP
library (``paper_2503_22863_amd``) and neither package imports the other; the
only module both sides use is the seeded input generator ``gsr_synth``.

The arithmetic lives in ``oracle.c`` (plain FP64 C, compiled with
-ffp-contract=off); this module marshals numpy arrays into it.  The
warm-start network reference (``oracle.mlp``) is plain numpy in FP64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

P64, P32 = 0, 1
# LSQR only: A^T on the unnormalised u', divided by beta afterwards (the order of one pass over
# the rows per iteration), with FP32 or FP64 products
P32_1P, P64_1P = 2, 3


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP64, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off",
                               "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Sys(C.Structure):
    _fields_ = [("n_stars", C.c_int64), ("m", C.c_int64), ("n_att", C.c_int64), ("n_instr", C.c_int64),
                ("n_glob", C.c_int32), ("f32", C.c_int32), ("vals", C.c_void_p),
                ("star_row_ptr", C.c_void_p), ("att_start", C.c_void_p), ("instr_col", C.c_void_p),
                ("ncon", C.c_int64), ("con_ptr", C.c_void_p), ("con_col", C.c_void_p), ("con_val", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("damp", C.c_double), ("atol", C.c_double), ("btol", C.c_double), ("conlim", C.c_double),
                ("itmax", C.c_int64), ("precond", C.c_int32), ("mode", C.c_int32)]


class _Res(C.Structure):
    _fields_ = [("istop", C.c_int32), ("itn", C.c_int64), ("rnorm", C.c_double), ("arnorm", C.c_double),
                ("anorm", C.c_double), ("acond", C.c_double), ("xnorm", C.c_double), ("bnorm", C.c_double)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = C.CDLL(_LIB)
        vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        lib.orc_n_unknowns.restype = i64
        lib.orc_n_unknowns.argtypes = [vp]
        lib.orc_rows.restype = i64
        lib.orc_rows.argtypes = [vp]
        lib.orc_col.restype = i64
        lib.orc_col.argtypes = [vp, i64, i64, C.c_int]
        lib.orc_aprod1.restype = None
        lib.orc_aprod1.argtypes = [vp, vp, vp, d, C.c_int]
        lib.orc_aprod2.restype = C.c_int
        lib.orc_aprod2.argtypes = [vp, vp, vp, d, C.c_int]
        lib.orc_colnorms.restype = C.c_int
        lib.orc_colnorms.argtypes = [vp, vp]
        lib.orc_lsqr.restype = C.c_int
        lib.orc_lsqr.argtypes = [vp, vp, vp, vp, vp, vp, i64, vp, vp, vp, vp]
        lib.orc_covariances.restype = None
        lib.orc_covariances.argtypes = [vp, i64, i64, vp, vp]
        lib.orc_lsqr_refine.restype = C.c_int
        lib.orc_lsqr_refine.argtypes = [vp, vp, vp, vp, vp, i32, d, vp, vp, vp]
        lib.orc_set_threads.restype = None
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_get_threads.restype = C.c_int
        lib.orc_get_threads.argtypes = []
        lib.orc_features.restype = None
        lib.orc_features.argtypes = [vp, vp, vp, vp]
        _lib = lib
    return _lib


def set_threads(n: int) -> None:
    """Threads of the oracle's products (0: all processors).  Results do not depend on it."""
    _L().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_L().orc_get_threads())


def _p(a):
    return None if a is None else a.ctypes.data


class OSystem:
    """Oracle view of a generated system (keeps the numpy arrays alive).
    constraints: optional (con_ptr [ncon+1], con_col, con_val) CSR rows appended to A."""

    def __init__(self, sysgen, constraints=None):
        d = sysgen.dims
        self.dims = d
        self.vals = np.ascontiguousarray(sysgen.vals)
        if self.vals.dtype not in (np.float64, np.float32):
            raise TypeError("vals must be float64 or float32")
        self.star_row_ptr = np.ascontiguousarray(sysgen.star_row_ptr, dtype=np.int64)
        self.att_start = np.ascontiguousarray(sysgen.att_start, dtype=np.int32)
        self.instr_col = np.ascontiguousarray(sysgen.instr_col, dtype=np.int32)
        self.n = d.n
        if constraints is None:
            self.con = (np.zeros(1, np.int64), np.zeros(0, np.int64), np.zeros(0, np.float64))
        else:
            self.con = (np.ascontiguousarray(constraints[0], dtype=np.int64),
                        np.ascontiguousarray(constraints[1], dtype=np.int64),
                        np.ascontiguousarray(constraints[2], dtype=np.float64))
        self.ncon = self.con[0].size - 1
        self.m = d.m + self.ncon  # rows of [A; C]
        self._s = _Sys(d.n_stars, d.m, d.n_att, d.n_instr, d.n_glob, int(self.vals.dtype == np.float32),
                       _p(self.vals), _p(self.star_row_ptr), _p(self.att_start), _p(self.instr_col),
                       self.ncon, _p(self.con[0]), _p(self.con[1]), _p(self.con[2]))
        assert _L().orc_n_unknowns(C.byref(self._s)) == d.n
        assert _L().orc_rows(C.byref(self._s)) == self.m

    @property
    def ref(self):
        return C.byref(self._s)


def col(osys: OSystem, s: int, r: int, k: int) -> int:
    return int(_L().orc_col(osys.ref, s, r, k))


def aprod1(osys: OSystem, x, y=None, scale: float = 0.0, mode: int = P64):
    """Eq. (2): y <- scale*y + A x."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    assert x.shape == (osys.n,)
    y = np.zeros(osys.m) if y is None else np.array(y, dtype=np.float64, copy=True)
    _L().orc_aprod1(osys.ref, _p(x), _p(y), float(scale), int(mode))
    return y


def aprod2(osys: OSystem, y, x=None, scale: float = 0.0, mode: int = P64):
    """Eq. (3): x <- scale*x + A^T y."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    assert y.shape == (osys.m,)
    x = np.zeros(osys.n) if x is None else np.array(x, dtype=np.float64, copy=True)
    if _L().orc_aprod2(osys.ref, _p(y), _p(x), float(scale), int(mode)):
        raise MemoryError
    return x


def colnorms(osys: OSystem):
    out = np.empty(osys.n)
    if _L().orc_colnorms(osys.ref, _p(out)):
        raise MemoryError
    return out


def known_terms(osys: OSystem, x_true, noise):
    """b = A x_true + noise (the synthetic known terms); with constraint rows the
    consistent right-hand sides c = C x_true follow."""
    y = np.concatenate([np.asarray(noise, dtype=np.float64), np.zeros(osys.ncon)])
    return aprod1(osys, x_true, y=y, scale=1.0)


def lsqr(osys: OSystem, b, x0=None, damp=0.0, atol=1e-12, btol=1e-12, conlim=0.0, itmax=200,
         precond=True, mode=P64, sel=None, want_var=True):
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty(osys.n)
    var = np.empty(osys.n) if want_var else None
    scale = np.empty(osys.n)
    x0c = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    if sel is not None:
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        dsel = np.zeros((int(itmax), len(sel)))
        k = len(sel)
    else:
        dsel, k = None, 0
    o = _Opts(float(damp), float(atol), float(btol), float(conlim), int(itmax), int(bool(precond)), int(mode))
    r = _Res()
    if _L().orc_lsqr(osys.ref, _p(b), _p(x0c), _p(x), _p(var), _p(sel), k, _p(dsel), _p(scale),
                     C.byref(o), C.byref(r)):
        raise MemoryError
    out = dict(x=x, var=var, istop=r.istop, itn=r.itn, rnorm=r.rnorm, arnorm=r.arnorm, anorm=r.anorm,
               acond=r.acond, xnorm=r.xnorm, bnorm=r.bnorm, scale=scale)
    if sel is not None:
        out["dsel"] = dsel[: r.itn].copy()
        out["cov"] = covariances(out["dsel"], scale[sel])
    return out


def covariances(dsel, ssel=None):
    """Eq. (4) over the stored per-iteration vectors: C = S_sel (sum_i d_i d_i^T) S_sel."""
    dsel = np.ascontiguousarray(dsel, dtype=np.float64)
    itn, k = dsel.shape
    C_ = np.empty((k, k))
    ss = None if ssel is None else np.ascontiguousarray(ssel, dtype=np.float64)
    _L().orc_covariances(_p(dsel), itn, k, _p(ss), _p(C_))
    return C_


def lsqr_refine(osys: OSystem, b, x0=None, inner_atol=1e-6, inner_btol=1e-6, inner_itmax=1000,
                precond=True, outer_max=10, outer_tol=1e-11, inner_mode=P32):
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty(osys.n)
    x0c = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    o = _Opts(0.0, float(inner_atol), float(inner_btol), 0.0, int(inner_itmax), int(bool(precond)), int(inner_mode))
    tot = C.c_int64(0)
    steps = C.c_int32(0)
    r = _Res()
    if _L().orc_lsqr_refine(osys.ref, _p(b), _p(x0c), _p(x), C.byref(o), int(outer_max), float(outer_tol),
                            C.byref(tot), C.byref(steps), C.byref(r)):
        raise MemoryError
    return dict(x=x, inner_total=tot.value, outer_steps=steps.value, last_istop=r.istop)


def features(osys: OSystem, b, xo):
    """Per-star warm-start features, [n_stars, 28] float64."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    xo = np.ascontiguousarray(xo, dtype=np.float64)
    assert xo.shape == (osys.n - 5 * osys.dims.n_stars,)
    F = np.empty((osys.dims.n_stars, 28))
    _L().orc_features(osys.ref, _p(b), _p(xo), _p(F))
    return F
