"""Matrix powers and polynomials -- test infrastructure only.

Section 7 names in-place matrix powers and polynomials as the next kernels
that RACE schedules serve.  What they compute has a plain definition, which
this oracle writes out:

    y_0 = x,   y_p = A y_(p-1)   (p = 1, 2, ...),   so y_p = A^p x;
    p(A) x = sum_p c_p A^p x.

Each product is the product oracle (``symmspmv.symm_spmv_c``, the serial
Algorithm "SymmSpMV" in plain C, or ``symmspmv.symm_spmv`` on request), in
float64, one power after the other; the polynomial sums the powers with
their coefficients left to right.
"""
from __future__ import annotations

import numpy as np

from . import symmspmv as O


def powers(n, row_ptr, col, val, x, count, product="c"):
    """[A x, A^2 x, ..., A^count x] for the symmetric matrix stored as its
    upper triangle (CRS)."""
    out = []
    y = np.asarray(x, dtype=np.float64)
    for _ in range(count):
        y = O.symm_spmv_c(n, row_ptr, col, val, y) if product == "c" else O.symm_spmv(n, row_ptr, col, val, y)
        out.append(y)
    return out


def poly(n, row_ptr, col, val, coeffs, x, product="c"):
    """sum_{p=0..len(coeffs)-1} coeffs[p] A^p x."""
    x = np.asarray(x, dtype=np.float64)
    z = coeffs[0] * x
    for c, y in zip(coeffs[1:], powers(n, row_ptr, col, val, x, len(coeffs) - 1, product)):
        z = z + c * y
    return z
