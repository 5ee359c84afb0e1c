"""Dense matrices for brute-force checks on small systems (test helper).

The dense A is assembled block by block from the structure of the
observation matrix (block-diagonal astrometric part, attitude windows of 4
consecutive spline coefficients per axis, instrumental one-hot columns, one
global column), independently of any per-slot column function.
"""
import numpy as np


def dense_A(sysgen):
    d = sysgen.dims
    V = np.asarray(sysgen.vals, dtype=np.float64)
    m, S = d.m, d.n_stars
    NA = 5 * S
    A = np.zeros((m, d.n))
    rows = np.arange(m)
    star_of_row = np.repeat(np.arange(S), np.diff(sysgen.star_row_ptr))
    # astrometric: a 5-wide block on the diagonal for every star
    for k in range(5):
        A[rows, 5 * star_of_row + k] += V[:, k]
    # attitude: axis a, spline coefficient att_start + j
    for a in range(3):
        base = NA + a * d.n_att
        for j in range(4):
            A[rows, base + sysgen.att_start + j] += V[:, 5 + 4 * a + j]
    # instrumental: one-hot per listed column
    base = NA + 3 * d.n_att
    for p in range(6):
        A[rows, base + sysgen.instr_col[:, p]] += V[:, 17 + p]
    if d.n_glob:
        A[:, base + d.n_instr] = V[:, 23]
    return A
