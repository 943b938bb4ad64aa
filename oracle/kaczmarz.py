"""Kaczmarz sweeps -- test infrastructure only ("parity" reference for the
GPU sweep kernel; never called by the product path).

The paper names the Kaczmarz method beside Gauss-Seidel among the solvers
whose row dependencies call for a coloring (Section 1, with a distance-1
or distance-2 coloring as the dependencies require).  A Kaczmarz sweep
projects x onto the hyperplane of one equation after another:

    x <- x + omega (b_i - a_i . x) / |a_i|^2  a_i,

a_i being row i of the full symmetric matrix (its diagonal included) and
omega the relaxation (1 = the plain projection).  Row i reads and writes x
at every column of a_i, so two rows conflict when they share a column: rows
that are at distance 3 or more (a distance-2 coloring, Section 4.2) can be
projected at the same time and give the same result as one after another.
A row with no stored value is skipped (there is nothing to project on).

* ``sweep`` runs the rule over a given row order on the symmetric matrix
  stored as its upper triangle (the lower part of row i is column i of the
  upper part, Section 3.2).  Plain loops in float64: the dot product and
  the squared norm are summed left to right in ascending column order.
* ``symmetric_sweep`` is a forward sweep followed by a backward sweep over
  the reversed order.
* ``sweep_c`` runs the same loop in plain C (``kaczmarz.c``) for the
  full-size cases.  The row order of a schedule is ``gauss_seidel.race_order``.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import build as _build
from .gauss_seidel import full_rows


def rows_with_diagonal(n, row_ptr, col, val):
    """Every row of the full symmetric matrix as (columns, values) lists in
    ascending column order, the diagonal in its place when it is stored."""
    cols, vals, diag = full_rows(n, row_ptr, col, val)
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    has = np.zeros(n, dtype=bool)
    for r in range(n):
        for k in range(row_ptr[r], row_ptr[r + 1]):
            if int(col[k]) == r:
                has[r] = True
    out_c, out_v = [], []
    for r in range(n):
        c, v = list(cols[r]), list(vals[r])
        if has[r]:
            p = int(np.searchsorted(np.asarray(c, dtype=np.int64), r))
            c.insert(p, r)
            v.insert(p, float(diag[r]))
        out_c.append(c)
        out_v.append(v)
    return out_c, out_v


def sweep(n, row_ptr, col, val, b, x, order, omega=1.0):
    """One Kaczmarz sweep over the rows in ``order``; returns the new x (the
    input is not modified)."""
    cols, vals = rows_with_diagonal(n, row_ptr, col, val)
    x = np.array(x, dtype=np.float64, copy=True)
    for i in order:
        i = int(i)
        dot = 0.0
        nrm = 0.0
        for c, a in zip(cols[i], vals[i]):
            dot += a * x[c]
            nrm += a * a
        if nrm == 0.0:
            continue
        coef = omega * (float(b[i]) - dot) / nrm
        for c, a in zip(cols[i], vals[i]):
            x[c] += coef * a
    return x


def symmetric_sweep(n, row_ptr, col, val, b, x, order, omega=1.0):
    """Forward sweep over ``order``, then backward over its reverse."""
    order = list(order)
    x1 = sweep(n, row_ptr, col, val, b, x, order, omega)
    return sweep(n, row_ptr, col, val, b, x1, order[::-1], omega)


def sweep_c(n, row_ptr, col, val, b, x, order, omega=1.0):
    """``sweep`` in plain C (same summation order); returns the new x."""
    lib = ctypes.CDLL(_build.build(force=False))
    f = lib.oracle_kacz_sweep
    f.restype = ctypes.c_int
    I32 = ctypes.POINTER(ctypes.c_int32)
    D = ctypes.POINTER(ctypes.c_double)
    f.argtypes = [ctypes.c_int32, I32, I32, D, D, D, I32, ctypes.c_int32, ctypes.c_double]
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    xx = np.array(x, dtype=np.float64, copy=True)
    od = np.ascontiguousarray(order, dtype=np.int32)
    rc = f(int(n), rp.ctypes.data_as(I32), c.ctypes.data_as(I32), v.ctypes.data_as(D), bb.ctypes.data_as(D),
           xx.ctypes.data_as(D), od.ctypes.data_as(I32), int(od.size), float(omega))
    if rc != 0:
        raise MemoryError("oracle_kacz_sweep: out of memory")
    return xx


def symmetric_sweep_c(n, row_ptr, col, val, b, x, order, omega=1.0):
    order = np.asarray(order, dtype=np.int32)
    x1 = sweep_c(n, row_ptr, col, val, b, x, order, omega)
    return sweep_c(n, row_ptr, col, val, b, x1, order[::-1].copy(), omega)
