"""Gauss-Seidel sweeps -- test infrastructure only ("parity" reference for the
GPU sweep kernel; never called by the product path).

The paper names Gauss-Seidel as a prime user of colorings (Section 1 and
Section 4.2; its row dependencies need distance 1): a sweep updates row i
with the newest values of all other unknowns,

    x_i <- (b_i - sum_{j != i} a_ij x_j) / a_ii,

in a fixed row order.  A coloring changes that order, not the rule: rows of
one color that share no edge (distance-1 independent) can be updated at the
same time and give the same result as updating them one after another.

* ``sweep`` runs the rule over a given row order on the symmetric matrix
  stored as its upper triangle (the lower part of row i is column i of the
  upper part, Section 3.2).  Plain loops in float64.
* ``symmetric_sweep`` is a forward sweep followed by a backward sweep over
  the reversed order (SymmGS).
* ``race_order`` is the order a RACE schedule runs its rows in: leaves by
  phase (colors, Section 4.4.3), then by first row, rows ascending inside a
  leaf; in the input numbering.
* ``sweep_c`` runs the same loop in plain C (``gauss_seidel.c``) for the
  full-size cases.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build


def full_rows(n, row_ptr, col, val):
    """Every row of the full symmetric matrix as (columns, values) lists,
    off-diagonal entries in ascending column order, and the diagonal."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    cols = [[] for _ in range(n)]
    vals = [[] for _ in range(n)]
    diag = np.zeros(n)
    for r in range(n):
        for k in range(row_ptr[r], row_ptr[r + 1]):
            c = int(col[k])
            if c == r:
                diag[r] = float(val[k])
            else:
                cols[r].append(c)
                vals[r].append(float(val[k]))
                cols[c].append(r)
                vals[c].append(float(val[k]))
    for r in range(n):
        if cols[r]:
            o = sorted(range(len(cols[r])), key=lambda t: cols[r][t])
            cols[r] = [cols[r][t] for t in o]
            vals[r] = [vals[r][t] for t in o]
    return cols, vals, diag


def sweep(n, row_ptr, col, val, b, x, order):
    """One Gauss-Seidel sweep over the rows in ``order``; returns the new x
    (the input is not modified).  Each row sums its off-diagonal products
    left to right in ascending column order, then divides by the diagonal."""
    cols, vals, diag = full_rows(n, row_ptr, col, val)
    x = np.array(x, dtype=np.float64, copy=True)
    for i in order:
        i = int(i)
        s = 0.0
        for c, a in zip(cols[i], vals[i]):
            s += a * x[c]
        x[i] = (float(b[i]) - s) / diag[i]
    return x


def symmetric_sweep(n, row_ptr, col, val, b, x, order):
    """Forward sweep over ``order``, then backward over its reverse."""
    order = list(order)
    x1 = sweep(n, row_ptr, col, val, b, x, order)
    return sweep(n, row_ptr, col, val, b, x1, order[::-1])


def race_order(perm, leaf_lo, leaf_hi, leaf_phase):
    """Rows (input numbering) in the order a schedule runs them: leaves
    sorted by (phase, first row), rows of a leaf ascending in the permuted
    numbering; perm maps permuted rows to input rows."""
    perm = np.asarray(perm, dtype=np.int64)
    leaves = sorted(zip(leaf_phase, leaf_lo, leaf_hi))
    out = []
    for _, lo, hi in leaves:
        out.extend(int(perm[r]) for r in range(lo, hi))
    return out


def sweep_c(n, row_ptr, col, val, b, x, order):
    """``sweep`` in plain C (same summation order); returns the new x."""
    lib = ctypes.CDLL(_build.build(force=False))
    f = lib.oracle_gs_sweep
    f.restype = ctypes.c_int
    I32 = ctypes.POINTER(ctypes.c_int32)
    D = ctypes.POINTER(ctypes.c_double)
    f.argtypes = [ctypes.c_int32, I32, I32, D, D, D, I32, ctypes.c_int32]
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    xx = np.array(x, dtype=np.float64, copy=True)
    od = np.ascontiguousarray(order, dtype=np.int32)
    rc = f(int(n), rp.ctypes.data_as(I32), c.ctypes.data_as(I32), v.ctypes.data_as(D), bb.ctypes.data_as(D),
           xx.ctypes.data_as(D), od.ctypes.data_as(I32), int(od.size))
    if rc != 0:
        raise MemoryError("oracle_gs_sweep: out of memory")
    return xx


def symmetric_sweep_c(n, row_ptr, col, val, b, x, order):
    order = np.asarray(order, dtype=np.int32)
    x1 = sweep_c(n, row_ptr, col, val, b, x, order)
    return sweep_c(n, row_ptr, col, val, b, x1, order[::-1].copy())
