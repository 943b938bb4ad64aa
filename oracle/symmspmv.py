"""Product oracle -- test infrastructure only.

y = A x for a real symmetric A that is stored as its upper triangle
(diagonal included) in CRS, as in the SymmSpMV kernel of Section 3.2
(Algorithm "SymmSpMV"): every stored off-diagonal A[r, c] contributes
A[r, c] * x[c] to y[r] (the gather) and A[r, c] * x[r] to y[c] (the
scatter); the diagonal contributes once.  The full-matrix CRS SpMV of
Section 3.1 (Algorithm "SpMV") is the yardstick.

Complex values (complex symmetric or Hermitian) follow the same
algorithm with a_ij or conj(a_ij) in the scatter: ``symm_spmv_complex_loop``
and ``symm_spmv_complex``.

Three independent renderings of the same definition:

* ``symm_spmv_loop``  -- the serial algorithm, pure Python (small inputs);
* ``symm_spmv``       -- y = (U + U^T - diag(U)) x with scipy's sparse matmul;
* ``symm_spmv_c``     -- the serial algorithm in plain C (``symmspmv.c``),
  used for the timed CPU baseline.

Rows without a stored diagonal are allowed and mean a zero diagonal.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")


def symm_spmv_loop(n, row_ptr, col, val, x):
    """Algorithm SymmSpMV (Section 3.2) as written: b starts at zero; the first
    stored entry of a row is its diagonal when its column equals the row."""
    b = [0.0] * n
    for row in range(n):
        start, end = int(row_ptr[row]), int(row_ptr[row + 1])
        xr = float(x[row])
        if start < end and int(col[start]) == row:
            b[row] += float(val[start]) * xr
            start += 1
        tmp = 0.0
        for idx in range(start, end):
            c = int(col[idx])
            tmp += float(val[idx]) * float(x[c])
            b[c] += float(val[idx]) * xr
        b[row] += tmp
    return np.array(b, dtype=np.float64)


def upper_matrix(n, row_ptr, col, val):
    return sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col), np.asarray(row_ptr)), shape=(n, n))


def symm_spmv(n, row_ptr, col, val, x):
    """y = (U + U^T - diag(U)) x; x may be (n,) or row-major (n, k)."""
    u = upper_matrix(n, row_ptr, col, val)
    d = u.diagonal()
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        return u @ x + u.T @ x - d * x
    return u @ x + u.T @ x - d[:, None] * x


def expand_full(n, row_ptr, col, val):
    """Full symmetric matrix in CRS (columns ascending): U + U^T - diag(U)."""
    u = upper_matrix(n, row_ptr, col, val)
    full = (u + u.T - sp.diags(u.diagonal())).tocsr()
    full.sort_indices()
    return (full.indptr.astype(np.int32), full.indices.astype(np.int32), full.data.astype(np.float64))


def spmv_full(n, row_ptr, col, val, x):
    """Algorithm SpMV (Section 3.1): b = A x from the full CRS matrix."""
    a = sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col), np.asarray(row_ptr)), shape=(n, n))
    return a @ np.asarray(x, dtype=np.float64)


def abs_product(n, row_ptr, col, val, x):
    """(|A| |x|), the scale of the rounding error of any summation order."""
    return symm_spmv(n, row_ptr, col, np.abs(val), np.abs(x))


def errors(y, y_ref, absprod=None):
    """Normwise ||y - y_ref||_inf / ||y_ref||_inf and, when |A||x| is given,
    componentwise max_i |y_i - y_ref_i| / (|A||x|)_i."""
    y = np.asarray(y, dtype=np.float64)
    y_ref = np.asarray(y_ref, dtype=np.float64)
    d = np.abs(y - y_ref)
    den = float(np.max(np.abs(y_ref))) if y_ref.size else 0.0
    err_norm = float(np.max(d)) / den if den > 0 else float(np.max(d, initial=0.0))
    err_comp = None
    if absprod is not None:
        a = np.asarray(absprod, dtype=np.float64)
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.where(a > 0, d / np.where(a > 0, a, 1.0), np.where(d > 0, np.inf, 0.0))
        err_comp = float(np.max(r, initial=0.0))
    return err_norm, err_comp


# --- complex values -----------------------------------------------------------
#
# The paper notes that the method carries over to complex matrices.  With
# only the upper triangle U stored, the full matrix is U + U^T - diag(U)
# when it is complex symmetric (a_ji = a_ij) and U + U^H - diag(U) when it is
# Hermitian (a_ji = conj(a_ij)); the scatter of the serial algorithm then
# uses a_ij or conj(a_ij).  The diagonal is used as stored.

def symm_spmv_complex_loop(n, row_ptr, col, val, x, hermitian):
    """The serial algorithm for complex values (pure Python, small inputs)."""
    b = [0j] * n
    for row in range(n):
        start, end = int(row_ptr[row]), int(row_ptr[row + 1])
        xr = complex(x[row])
        if start < end and int(col[start]) == row:
            b[row] += complex(val[start]) * xr
            start += 1
        tmp = 0j
        for idx in range(start, end):
            c = int(col[idx])
            a = complex(val[idx])
            tmp += a * complex(x[c])
            b[c] += (a.conjugate() if hermitian else a) * xr
        b[row] += tmp
    return np.array(b, dtype=np.complex128)


def symm_spmv_complex(n, row_ptr, col, val, x, hermitian):
    """y = (U + U^T - diag(U)) x, or (U + U^H - conj(diag(U))) x when hermitian
    (the stored diagonal either way)."""
    u = sp.csr_matrix((np.asarray(val, dtype=np.complex128), np.asarray(col), np.asarray(row_ptr)), shape=(n, n))
    d = u.diagonal()
    x = np.asarray(x, dtype=np.complex128)
    low = u.conj().T if hermitian else u.T
    # low repeats the diagonal (conjugated when hermitian): take that copy out
    return u @ x + low @ x - (np.conj(d) if hermitian else d) * x


def abs_product_complex(n, row_ptr, col, val, x):
    """(|A| |x|) for complex values: the rounding scale of any order."""
    return symm_spmv(n, row_ptr, col, np.abs(np.asarray(val)), np.abs(np.asarray(x)))


# --- the plain C serial algorithm ------------------------------------------

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle C library missing: {LIB_PATH} (run the build)")
        lib = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_symm_spmv.argtypes = [ctypes.c_int32, ip, ip, dp, dp, dp]
        lib.oracle_symm_spmv.restype = None
        lib.oracle_symm_spmv_f32.argtypes = [ctypes.c_int32, ip, ip, ctypes.POINTER(ctypes.c_float), dp, dp]
        lib.oracle_symm_spmv_f32.restype = None
        _lib = lib
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def symm_spmv_c(n, row_ptr, col, val, x, y=None):
    """Serial Algorithm SymmSpMV in C; ``val`` float64 or float32 (promoted)."""
    lib = _load()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if y is None:
        y = np.empty(n, dtype=np.float64)
    if val.dtype == np.float32:
        v = np.ascontiguousarray(val)
        lib.oracle_symm_spmv_f32(n, _ptr(row_ptr, ctypes.c_int32), _ptr(col, ctypes.c_int32), _ptr(v, ctypes.c_float),
                                 _ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double))
    else:
        v = np.ascontiguousarray(val, dtype=np.float64)
        lib.oracle_symm_spmv(n, _ptr(row_ptr, ctypes.c_int32), _ptr(col, ctypes.c_int32), _ptr(v, ctypes.c_double),
                             _ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double))
    return y
