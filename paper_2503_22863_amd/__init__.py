"""MI355X (gfx950) hot path of the Gaia AVU-GSR solver: Python binding of libgsr.

Argument marshalling only.  Every step of the method runs in the HIP kernels
of ``libgsr.so`` (built in-tree by ``paper_2503_22863_amd.build``); this
module passes device pointers of PyTorch tensors and the current HIP stream
through the C interface declared in ``include/gsr.h``.  There is no CPU
fallback: if the library is missing, loading fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # loads the HIP runtime that libgsr shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsr.so")

GSR_F64, GSR_F32 = 0, 1
PROD_F64, PROD_F32 = 0, 1


class GsrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gsr error {code}: {msg}")
        self.code = code


class Dims(C.Structure):
    _fields_ = [("n_stars", C.c_int64), ("m", C.c_int64), ("n_att", C.c_int64), ("n_instr", C.c_int64),
                ("n_glob", C.c_int32), ("value_type", C.c_int32)]


class LsqrOpts(C.Structure):
    _fields_ = [("damp", C.c_double), ("atol", C.c_double), ("btol", C.c_double), ("conlim", C.c_double),
                ("itmax", C.c_int64), ("precond", C.c_int32), ("product", C.c_int32),
                ("outer_max", C.c_int32), ("outer_tol", C.c_double)]


class LsqrResult(C.Structure):
    _fields_ = [("istop", C.c_int32), ("outer_steps", C.c_int32), ("itn", C.c_int64),
                ("inner_total", C.c_int64), ("rnorm", C.c_double), ("arnorm", C.c_double),
                ("anorm", C.c_double), ("acond", C.c_double), ("xnorm", C.c_double), ("bnorm", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BlockedInfo(C.Structure):
    _fields_ = [("active", C.c_int32), ("workgroups", C.c_int32), ("window", C.c_int64), ("blocks", C.c_int64),
                ("padded_rows", C.c_int64), ("segments", C.c_int64), ("bytes", C.c_int64),
                ("value_bytes", C.c_int64), ("values_owned", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Timing(C.Structure):
    _fields_ = [("aprod1_ms", C.c_double), ("aprod2_ms", C.c_double), ("tail_ms", C.c_double),
                ("update_ms", C.c_double), ("syrk_ms", C.c_double), ("aprod1_n", C.c_int64),
                ("aprod2_n", C.c_int64), ("tail_n", C.c_int64), ("update_n", C.c_int64), ("syrk_n", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

_SIGS = {
    # name: (restype, argtypes)
    "gsr_num_unknowns": (C.c_int64, [C.c_void_p]),
    "gsr_last_error": (C.c_char_p, []),
    "gsr_version": (C.c_char_p, []),
    "gsr_create": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_destroy": (C.c_int, [C.c_void_p]),
    "gsr_aprod1": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_void_p]),
    "gsr_aprod2": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_void_p]),
    "gsr_aprod1_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_void_p]),
    "gsr_aprod12": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_double, C.c_int32,
                              C.c_void_p]),
    "gsr_layout_plan": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                  C.c_void_p]),
    "gsr_layout_info": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gsr_layout_pack": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p]),
    "gsr_create_packed": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_layout_destroy": (C.c_int, [C.c_void_p]),
    "gsr_column_scale": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_lsqr_solve": (C.c_int, [C.c_void_p] * 8),
    "gsr_lsqr_begin": (C.c_int, [C.c_void_p] * 5),
    "gsr_lsqr_iterate": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p]),
    "gsr_lsqr_status": (C.c_int, [C.c_void_p] * 3),
    "gsr_lsqr_peek": (C.c_int, [C.c_void_p] * 3),
    "gsr_lsqr_end": (C.c_int, [C.c_void_p] * 5),
    "gsr_lsqr_refine": (C.c_int, [C.c_void_p] * 7),
    "gsr_cov_request": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32]),
    "gsr_cov_get": (C.c_int, [C.c_void_p] * 3),
    "gsr_cov_bytes": (C.c_int64, [C.c_int32, C.c_int64, C.c_int64]),
    "gsr_syrk": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p]),
    "gsr_set_tuning": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "gsr_timing_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "gsr_set_graphs": (C.c_int, [C.c_void_p, C.c_int32]),
    "gsr_set_fused": (C.c_int, [C.c_void_p, C.c_int32]),
    "gsr_set_blocked": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "gsr_blocked_info": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gsr_set_constraints": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_cov_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32]),
    "gsr_cov_export_status": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_cov_from_export": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int64, C.c_int32, C.c_void_p,
                                      C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_cov_request_pairs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32]),
    "gsr_cov_get_pairs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_cov_pairs_from_export": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int64, C.c_int32, C.c_void_p,
                                            C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gsr_timing_get": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gsr_features": (C.c_int, [C.c_void_p] * 5),
    "gsr_mean_rows": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p]),
    "gsr_mlp_create": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p]),
    "gsr_mlp_destroy": (C.c_int, [C.c_void_p]),
    "gsr_mlp_get_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gsr_mlp_fit_norm": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "gsr_mlp_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "gsr_mlp_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                               C.c_void_p]),
    "gsr_mlp_train": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_double,
                                C.c_void_p, C.c_void_p]),
}


def lib():
    """The loaded libgsr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2503_22863_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name, None)
            if f is None:
                continue
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise GsrError(rc, lib().gsr_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _prod(product):
    if product in ("f64", PROD_F64, None):
        return PROD_F64
    if product in ("f32", PROD_F32):
        return PROD_F32
    raise ValueError(product)


def num_unknowns(n_stars, n_att, n_instr, n_glob, m=0):
    d = Dims(n_stars, m, n_att, n_instr, n_glob, 0)
    return int(lib().gsr_num_unknowns(C.byref(d)))


def cov_bytes(version, itn_cov_cp, count):
    return int(lib().gsr_cov_bytes(version, itn_cov_cp, count))


def syrk(D, k, cols, ldd, Cmat, stream=None):
    _check(lib().gsr_syrk(_ptr(D), k, cols, ldd, _ptr(Cmat), _stream(stream)))


def cov_from_export(blocks, n, block, nblocks, last_cols, sel, S=None, stream=None):
    """Covariances of the selected unknowns from exported d_i blocks (host tensor
    [>= nblocks][block][n]); S: the solve's column scaling (device) or None."""
    sel = np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    out = torch.empty((sel.size, sel.size), dtype=torch.float64, device="cuda")
    _check(lib().gsr_cov_from_export(C.c_void_p(blocks.data_ptr()), int(n), int(block), int(nblocks),
                                     int(last_cols), sel.ctypes.data if sel.size else None, sel.size,
                                     _ptr(S) if S is not None else None, _ptr(out), _stream(stream)))
    return out


def cov_pairs_from_export(blocks, n, block, nblocks, last_cols, pairs, S=None, stream=None):
    """Covariances of the index pairs [P][2] from exported d_i blocks; S as cov_from_export."""
    pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))
    out = torch.empty(pairs.shape[0], dtype=torch.float64, device="cuda")
    _check(lib().gsr_cov_pairs_from_export(C.c_void_p(blocks.data_ptr()), int(n), int(block), int(nblocks),
                                           int(last_cols), pairs.ctypes.data if pairs.size else None,
                                           pairs.shape[0], _ptr(S) if S is not None else None, _ptr(out),
                                           _stream(stream)))
    return out


def mean_rows(X, stream=None):
    """Mean of the k rows of a [k][len] device matrix (e.g. the mean of training solutions)."""
    k, ln = X.shape
    out = torch.empty(ln, dtype=torch.float64, device=X.device)
    _check(lib().gsr_mean_rows(_ptr(X), k, ln, _ptr(out), _stream(stream)))
    return out


class MLP:
    """FP32 network n_in -> hidden -> hidden -> n_out (ReLU), trained on the device with Adam.
    params: [W1 (H,I), b1, W2 (H,H), b2, W3 (O,H), b3] (host numpy, any float dtype)."""

    def __init__(self, params):
        W1, b1, W2, b2, W3, b3 = params
        self.n_in, self.n_hidden, self.n_out = W1.shape[1], W1.shape[0], W3.shape[0]
        flat = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1) for p in params]))
        self.size = flat.size
        h = C.c_void_p()
        _check(lib().gsr_mlp_create(C.byref(h), self.n_in, self.n_hidden, self.n_out, flat.ctypes.data))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().gsr_mlp_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        flat = np.empty(self.size)
        _check(lib().gsr_mlp_get_params(self._h, flat.ctypes.data))
        I, H, O = self.n_in, self.n_hidden, self.n_out
        out, o = [], 0
        for shp in ((H, I), (H,), (H, H), (H,), (O, H), (O,)):
            k = int(np.prod(shp))
            out.append(flat[o:o + k].reshape(shp))
            o += k
        return out

    def fit_norm(self, X, T, stream=None):
        _check(lib().gsr_mlp_fit_norm(self._h, _ptr(X), _ptr(T), X.shape[0], _stream(stream)))

    def forward(self, X, stream=None):
        Y = torch.empty((X.shape[0], self.n_out), dtype=torch.float64, device=X.device)
        _check(lib().gsr_mlp_forward(self._h, _ptr(X), X.shape[0], _ptr(Y), _stream(stream)))
        return Y

    def grad(self, X, T, stream=None):
        g = torch.empty(self.size, dtype=torch.float32, device=X.device)
        loss = C.c_double()
        _check(lib().gsr_mlp_grad(self._h, _ptr(X), _ptr(T), X.shape[0], C.byref(loss), _ptr(g), _stream(stream)))
        return loss.value, g

    def train(self, X, T, steps, lr=1e-3, stream=None):
        loss = C.c_double()
        _check(lib().gsr_mlp_train(self._h, _ptr(X), _ptr(T), X.shape[0], int(steps), float(lr), C.byref(loss),
                                   _stream(stream)))
        return loss.value


def _opts(damp=0.0, atol=1e-12, btol=1e-12, conlim=0.0, itmax=200, precond=True, product="f64",
          outer_max=10, outer_tol=1e-11):
    return LsqrOpts(float(damp), float(atol), float(btol), float(conlim), int(itmax), int(bool(precond)),
                    _prod(product), int(outer_max), float(outer_tol))


class Layout:
    """The regrouped row order of a system, computed from its index arrays
    (gsr_layout_plan).  The caller allocates ``info()["value_bytes"]`` of
    device memory, places its rows there with ``pack`` and hands the buffer
    to ``System.from_packed``, which consumes the layout."""

    def __init__(self, star_row_ptr, att_start, instr_col, n_att, n_instr, n_glob=1, value_type=GSR_F64,
                 max_window=0, stream=None):
        if star_row_ptr.dtype != torch.int64 or att_start.dtype != torch.int32 or instr_col.dtype != torch.int32:
            raise TypeError("star_row_ptr int64, att_start int32, instr_col int32")
        n_stars = star_row_ptr.numel() - 1
        m = att_start.numel()
        self.dims = Dims(n_stars, m, n_att, n_instr, n_glob, value_type)
        self.value_type = value_type
        self.device = att_start.device
        h = C.c_void_p()
        _check(lib().gsr_layout_plan(C.byref(h), C.byref(self.dims), _ptr(star_row_ptr), _ptr(att_start),
                                     _ptr(instr_col), int(max_window), _stream(stream)))
        self._h = h

    def info(self):
        i = BlockedInfo()
        _check(lib().gsr_layout_info(self._h, C.byref(i)))
        return i.as_dict()

    def new_buffer(self):
        """Device tensor of the packed rows' size ([padded_rows, 24] of the value type)."""
        dt = torch.float32 if self.value_type == GSR_F32 else torch.float64
        return torch.empty((self.info()["padded_rows"], 24), dtype=dt, device=self.device)

    def pack(self, rows, row0, packed, stream=None):
        """Place rows row0 .. row0+len(rows)-1 (device [count, 24]) into packed."""
        _check(lib().gsr_layout_pack(self._h, _ptr(rows), int(row0), int(rows.shape[0]), _ptr(packed),
                                     _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().gsr_layout_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class System:
    """A handle over a system held in device tensors (borrowed; kept alive here)."""

    def __init__(self, vals, star_row_ptr, att_start, instr_col, n_att, n_instr, n_glob=1, stream=None):
        if vals.dtype == torch.float64:
            vt = GSR_F64
        elif vals.dtype == torch.float32:
            vt = GSR_F32
        else:
            raise TypeError("vals must be float64 or float32")
        if star_row_ptr.dtype != torch.int64 or att_start.dtype != torch.int32 or instr_col.dtype != torch.int32:
            raise TypeError("star_row_ptr int64, att_start int32, instr_col int32")
        self.vals, self.star_row_ptr, self.att_start, self.instr_col = vals, star_row_ptr, att_start, instr_col
        n_stars = star_row_ptr.numel() - 1
        m = vals.shape[0] if vals.dim() else 0
        self.dims = Dims(n_stars, m, n_att, n_instr, n_glob, vt)
        self.n_stars, self.m, self.n_att, self.n_instr, self.n_glob = n_stars, m, n_att, n_instr, n_glob
        self.n = int(lib().gsr_num_unknowns(C.byref(self.dims)))
        self.value_type = vt
        self.device = vals.device
        h = C.c_void_p()
        _check(lib().gsr_create(C.byref(h), C.byref(self.dims), _ptr(vals), _ptr(star_row_ptr), _ptr(att_start),
                                _ptr(instr_col), _stream(stream)))
        self._h = h
        self.ncov = 0

    @classmethod
    def from_packed(cls, layout, packed, stream=None):
        """A handle over rows placed by ``layout.pack`` into ``packed`` (borrowed; the
        library holds no copy of the coefficients).  Consumes the layout."""
        self = cls.__new__(cls)
        self.vals, self.star_row_ptr, self.att_start, self.instr_col = None, None, None, None
        self.packed = packed
        d = layout.dims
        self.dims = Dims(d.n_stars, d.m, d.n_att, d.n_instr, d.n_glob, d.value_type)
        self.n_stars, self.m, self.n_att, self.n_instr, self.n_glob = d.n_stars, d.m, d.n_att, d.n_instr, d.n_glob
        self.n = int(lib().gsr_num_unknowns(C.byref(self.dims)))
        self.value_type = d.value_type
        self.device = packed.device
        h = C.c_void_p()
        _check(lib().gsr_create_packed(C.byref(h), layout._h, _ptr(packed), _stream(stream)))
        layout._h = None  # consumed
        self._h = h
        self.ncov = 0
        return self

    @classmethod
    def packed_from_generated(cls, g, device="cuda", value_dtype=None, max_window=0, chunk_rows=1 << 22):
        """Load a gsr_synth system the way a caller without room for two copies of A
        would: upload the index arrays, plan the layout, move the coefficients in
        chunks of ``chunk_rows`` rows through a staging buffer into their places,
        and free the index arrays.  The device then holds one copy of A."""
        vals = g.vals if value_dtype is None else g.vals.astype(value_dtype)
        vt = GSR_F32 if vals.dtype == np.float32 else GSR_F64
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        L = Layout(t(g.star_row_ptr), t(g.att_start), t(g.instr_col), g.dims.n_att, g.dims.n_instr, g.dims.n_glob,
                   value_type=vt, max_window=max_window)
        packed = L.new_buffer()
        m = vals.shape[0]
        for r0 in range(0, m, chunk_rows):
            L.pack(t(vals[r0:r0 + chunk_rows]), r0, packed)
            torch.cuda.synchronize(packed.device)  # the staging tensor may be freed
        return cls.from_packed(L, packed)

    @classmethod
    def from_generated(cls, g, device="cuda", value_dtype=None):
        """Upload a gsr_synth system (coefficients and index arrays) to the device."""
        vals = g.vals if value_dtype is None else g.vals.astype(value_dtype)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        return cls(t(vals), t(g.star_row_ptr), t(g.att_start), t(g.instr_col), g.dims.n_att, g.dims.n_instr,
                   g.dims.n_glob)

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().gsr_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self, size):
        return torch.empty(size, dtype=torch.float64, device=self.device)

    # ---- products
    def aprod1(self, x, y=None, scale=0.0, product="f64", stream=None):
        """Eq. (2): y <- scale*y + A x."""
        if y is None:
            y = self._new(self.m)
            scale = 0.0
        _check(lib().gsr_aprod1(self._h, _ptr(x), _ptr(y), float(scale), _prod(product), _stream(stream)))
        return y

    def aprod1_noalloc(self, x, y, scale=0.0, product="f64", stream=None):
        """gsr_aprod1 with its workspace in the library's static device scratch (no allocation)."""
        _check(lib().gsr_aprod1_noalloc(self._h, _ptr(x), _ptr(y), float(scale), _prod(product),
                                        _stream(stream)))
        return y

    def aprod12(self, v, u, x=None, scale_u=1.0, scale_x=0.0, product="f64", stream=None):
        """Both products in one pass: u <- scale_u*u + A v, then x <- scale_x*x + A^T u (new u)."""
        if x is None:
            x = self._new(self.n)
            scale_x = 0.0
        _check(lib().gsr_aprod12(self._h, _ptr(v), _ptr(u), float(scale_u), _ptr(x), float(scale_x),
                                 _prod(product), _stream(stream)))
        return u, x

    def aprod2(self, y, x=None, scale=0.0, product="f64", stream=None):
        """Eq. (3): x <- scale*x + A^T y."""
        if x is None:
            x = self._new(self.n)
            scale = 0.0
        _check(lib().gsr_aprod2(self._h, _ptr(y), _ptr(x), float(scale), _prod(product), _stream(stream)))
        return x

    def column_scale(self, stream=None):
        out = self._new(self.n)
        _check(lib().gsr_column_scale(self._h, _ptr(out), _stream(stream)))
        return out

    # ---- LSQR
    def lsqr_solve(self, b, x0=None, want_var=True, stream=None, **opts):
        x = self._new(self.n)
        var = self._new(self.n) if want_var else None
        r = LsqrResult()
        o = _opts(**opts)
        _check(lib().gsr_lsqr_solve(self._h, _ptr(b), _ptr(x0), _ptr(x), _ptr(var), C.byref(o), C.byref(r),
                                    _stream(stream)))
        return x, var, r.as_dict()

    def lsqr_begin(self, b, x0=None, stream=None, **opts):
        self._session = (b, x0)  # keep alive until end
        o = _opts(**opts)
        _check(lib().gsr_lsqr_begin(self._h, _ptr(b), _ptr(x0), C.byref(o), _stream(stream)))

    def lsqr_iterate(self, n, stream=None):
        _check(lib().gsr_lsqr_iterate(self._h, int(n), _stream(stream)))

    def lsqr_status(self, stream=None):
        r = LsqrResult()
        _check(lib().gsr_lsqr_status(self._h, C.byref(r), _stream(stream)))
        return r.as_dict()

    def lsqr_peek(self, x=None, stream=None):
        x = self._new(self.n) if x is None else x
        _check(lib().gsr_lsqr_peek(self._h, _ptr(x), _stream(stream)))
        return x

    def lsqr_end(self, want_var=True, stream=None):
        x = self._new(self.n)
        var = self._new(self.n) if want_var else None
        r = LsqrResult()
        _check(lib().gsr_lsqr_end(self._h, _ptr(x), _ptr(var), C.byref(r), _stream(stream)))
        self._session = None
        return x, var, r.as_dict()

    def lsqr_refine(self, b, x0=None, stream=None, **opts):
        opts.setdefault("product", "f32")
        opts.setdefault("atol", 1e-6)
        opts.setdefault("btol", 1e-6)
        opts.setdefault("itmax", 1000)
        x = self._new(self.n)
        r = LsqrResult()
        o = _opts(**opts)
        _check(lib().gsr_lsqr_refine(self._h, _ptr(b), _ptr(x0), _ptr(x), C.byref(o), C.byref(r),
                                     _stream(stream)))
        return x, r.as_dict()

    # ---- covariances
    def cov_request(self, sel, block=64):
        sel = np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
        _check(lib().gsr_cov_request(self._h, sel.ctypes.data if sel.size else None, sel.size, int(block)))
        self.ncov = sel.size

    def cov_export(self, host=None, block=64):
        """Attach a host buffer [max_blocks][block][n] (CPU float64 tensor, pinned for overlap)
        for the whole d_i of the next solves; host=None detaches."""
        if host is None:
            _check(lib().gsr_cov_export(self._h, None, 0, 0))
            self._export = None
            return
        assert host.device.type == "cpu" and host.dtype == torch.float64 and host.is_contiguous()
        assert host.shape[1] == block and host.shape[2] == self.n
        _check(lib().gsr_cov_export(self._h, C.c_void_p(host.data_ptr()), host.shape[0], int(block)))
        self._export = host  # keep alive

    def cov_export_status(self):
        nb, lc = C.c_int64(), C.c_int32()
        _check(lib().gsr_cov_export_status(self._h, C.byref(nb), C.byref(lc)))
        return nb.value, lc.value

    def cov_request_pairs(self, pairs, block=64):
        pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))
        _check(lib().gsr_cov_request_pairs(self._h, pairs.ctypes.data if pairs.size else None, pairs.shape[0],
                                           int(block)))
        self.npairs = pairs.shape[0]

    def cov_get_pairs(self, stream=None):
        out = torch.empty(self.npairs, dtype=torch.float64, device=self.device)
        _check(lib().gsr_cov_get_pairs(self._h, _ptr(out), _stream(stream)))
        return out

    def cov_get(self, stream=None):
        out = torch.empty((self.ncov, self.ncov), dtype=torch.float64, device=self.device)
        _check(lib().gsr_cov_get(self._h, _ptr(out), _stream(stream)))
        return out

    # ---- learned warm start
    def features(self, b, x_other, stream=None):
        """Per-star features [n_stars, 28] (FP64) with bt = b - A_other x_other."""
        F = torch.empty((self.n_stars, 28), dtype=torch.float64, device=self.device)
        _check(lib().gsr_features(self._h, _ptr(b), _ptr(x_other), _ptr(F), _stream(stream)))
        return F

    # ---- tuning and timing
    def set_tuning(self, waves_per_cu=32, att_atomics=0):
        _check(lib().gsr_set_tuning(self._h, int(waves_per_cu), int(att_atomics)))

    def set_graphs(self, on=True):
        _check(lib().gsr_set_graphs(self._h, int(bool(on))))

    def set_constraints(self, ptr=None, col=None, val=None, rhs=None):
        """Constraint rows (CSR, host arrays) under A with right-hand sides rhs; no arguments removes them."""
        if ptr is None:
            _check(lib().gsr_set_constraints(self._h, 0, None, None, None, None))
            return
        ptr = np.ascontiguousarray(ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int64)
        val = np.ascontiguousarray(val, dtype=np.float64)
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        _check(lib().gsr_set_constraints(self._h, ptr.size - 1, ptr.ctypes.data, col.ctypes.data if col.size else None,
                                         val.ctypes.data if val.size else None, rhs.ctypes.data))

    def set_fused(self, on=True):
        _check(lib().gsr_set_fused(self._h, int(bool(on))))

    def set_blocked(self, on=True, max_window=0):
        _check(lib().gsr_set_blocked(self._h, int(bool(on)), int(max_window)))

    def blocked_info(self):
        i = BlockedInfo()
        _check(lib().gsr_blocked_info(self._h, C.byref(i)))
        return i.as_dict()

    def timing_enable(self, on=True):
        _check(lib().gsr_timing_enable(self._h, int(bool(on))))

    def timing_get(self):
        t = Timing()
        _check(lib().gsr_timing_get(self._h, C.byref(t)))
        return t.as_dict()
