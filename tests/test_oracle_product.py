"""Pins for the product oracle (CPU only).

The oracle's three renderings of y = A x are checked against things that do
not share their code: a dense matvec of the symmetric matrix built entry by
entry, exactly rounded row sums (math.fsum), the rounding-error bound of a
recursive sum, and symmetry identities.  A deliberately broken variant
(planted on the CPU) must fail the same checks, so the pins have teeth.
"""
import math

import numpy as np
import pytest

import matgen
from oracle import symmspmv as O


def dense_symmetric(m):
    """Dense A from the upper CRS, written out entry by entry."""
    a = np.zeros((m.n, m.n))
    for r in range(m.n):
        for idx in range(m.row_ptr[r], m.row_ptr[r + 1]):
            c = int(m.col[idx])
            a[r, c] = m.val[idx]
            a[c, r] = m.val[idx]
    return a


def fsum_rows(a, x):
    return np.array([math.fsum(a[i, j] * x[j] for j in range(a.shape[1])) for i in range(a.shape[0])])


SMALL = [
    matgen.stencil2d_5pt(7, seed=11),
    matgen.stencil3d_27pt(4, seed=12),
    matgen.stencil2d_7pt(5),
    matgen.random_symmetric(40, 0.2, seed=13),
    matgen.random_symmetric(37, 0.1, seed=14, with_diag=False),
    matgen.banded_irregular(200, seed=15, band=16),
]


def gamma(n):
    u = 2.0 ** -53
    return n * u / (1 - n * u)


@pytest.mark.parametrize("m", SMALL, ids=lambda m: m.name)
def test_loop_matches_dense_and_fsum(m):
    x = matgen.rhs(m.n, 5)
    a = dense_symmetric(m)
    y_exact = fsum_rows(a, x)
    y_loop = O.symm_spmv_loop(m.n, m.row_ptr, m.col, m.val, x)
    absax = np.abs(a) @ np.abs(x)
    # every row sums at most (row length) products in some order
    k = int(np.max(np.count_nonzero(a, axis=1))) + 1
    assert np.all(np.abs(y_loop - y_exact) <= gamma(k) * absax + 1e-300)
    assert np.allclose(a @ x, y_exact, rtol=0, atol=1e-13 * max(1.0, np.abs(y_exact).max()))


@pytest.mark.parametrize("m", SMALL, ids=lambda m: m.name)
def test_three_renderings_agree(m, oracle_lib):
    x = matgen.rhs(m.n, 6)
    y_loop = O.symm_spmv_loop(m.n, m.row_ptr, m.col, m.val, x)
    y_sp = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x)
    y_c = O.symm_spmv_c(m.n, m.row_ptr, m.col, m.val, x)
    # identical algorithm and order in Python and C (no contraction): bit equal
    assert np.array_equal(y_loop, y_c)
    absax = O.abs_product(m.n, m.row_ptr, m.col, m.val, x)
    assert np.all(np.abs(y_sp - y_loop) <= 2 * gamma(64) * absax + 1e-300)


def test_symmetry_identity():
    # x^T (A z) == z^T (A x) for symmetric A (to rounding)
    m = matgen.stencil3d_27pt(6, seed=21)
    x = matgen.rhs(m.n, 1)
    z = matgen.rhs(m.n, 2)
    ax = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x)
    az = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, z)
    assert abs(x @ az - z @ ax) <= 1e-12 * (np.abs(x) @ np.abs(az) + 1)


def test_full_expansion_and_spmv():
    m = matgen.random_symmetric(50, 0.15, seed=31)
    x = matgen.rhs(m.n, 3)
    rp, c, v = O.expand_full(m.n, m.row_ptr, m.col, m.val)
    a = dense_symmetric(m)
    assert rp[-1] == np.count_nonzero(a)
    y = O.spmv_full(m.n, rp, c, v, x)
    assert np.allclose(y, a @ x, rtol=0, atol=1e-13)


def test_special_cases(oracle_lib):
    # diagonal only
    n = 5
    rp = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    val = np.arange(1, n + 1, dtype=np.float64)
    x = np.ones(n)
    assert np.array_equal(O.symm_spmv_c(n, rp, col, val, x), val)
    # rows without diagonal and empty rows
    rp = np.array([0, 1, 1, 2, 2], dtype=np.int32)
    col = np.array([2, 3], dtype=np.int32)
    val = np.array([2.0, 3.0])
    x = np.array([1.0, 10.0, 100.0, 1000.0])
    y = O.symm_spmv_loop(4, rp, col, val, x)
    assert np.array_equal(y, np.array([200.0, 0.0, 2.0 + 3000.0, 300.0]))
    assert np.array_equal(O.symm_spmv_c(4, rp, col, val, x), y)
    # n = 1
    assert np.array_equal(O.symm_spmv_loop(1, [0, 1], [0], [3.0], [2.0]), np.array([6.0]))


def test_float32_values_promoted(oracle_lib):
    m = matgen.stencil2d_5pt(9, seed=41)
    x = matgen.rhs(m.n, 4)
    v32 = m.val.astype(np.float32)
    y32 = O.symm_spmv_c(m.n, m.row_ptr, m.col, v32, x)
    y64 = O.symm_spmv_c(m.n, m.row_ptr, m.col, v32.astype(np.float64), x)
    assert np.array_equal(y32, y64)


def _broken_no_scatter(n, row_ptr, col, val, x):
    b = np.zeros(n)
    for row in range(n):
        for idx in range(row_ptr[row], row_ptr[row + 1]):
            b[row] += val[idx] * x[col[idx]]
    return b


def _broken_transposed(n, row_ptr, col, val, x):
    b = np.zeros(n)
    for row in range(n):
        for idx in range(row_ptr[row], row_ptr[row + 1]):
            c = col[idx]
            b[row] += val[idx] * x[row]
            if c != row:
                b[c] += val[idx] * x[c]
    return b


@pytest.mark.parametrize("broken", [_broken_no_scatter, _broken_transposed])
def test_pins_catch_planted_mistakes(broken):
    m = matgen.random_symmetric(30, 0.2, seed=51)
    x = matgen.rhs(m.n, 7)
    y_exact = fsum_rows(dense_symmetric(m), x)
    assert not np.allclose(broken(m.n, m.row_ptr, m.col, m.val, x), y_exact, rtol=1e-12, atol=1e-12)


def test_error_metrics():
    y_ref = np.array([1.0, -2.0, 4.0])
    y = y_ref + np.array([0.0, 1e-13, -2e-13])
    en, ec = O.errors(y, y_ref, np.array([1.0, 1.0, 2.0]))
    assert en == pytest.approx(2e-13 / 4.0)
    assert ec == pytest.approx(1e-13)


# ---------------------------------------------------------------------------
# Complex values (complex symmetric and Hermitian)

def _dense_upper(m, vals):
    u = np.zeros((m.n, m.n), dtype=np.complex128)
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    u[rows, m.col] = vals
    return u


def _complex_case(seed, n=40):
    m = matgen.random_symmetric(n, 0.15, seed=seed)
    rng = np.random.default_rng(seed)
    vals = m.val + 1j * rng.standard_normal(m.nnz)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return m, vals, x


@pytest.mark.parametrize("hermitian", [False, True])
def test_complex_loop_and_sparse_match_dense(hermitian):
    """Both complex renderings equal the dense product of the assembled
    matrix: A = U + U^T - D (complex symmetric) or U + U^H - conj(D) with the
    stored diagonal D (Hermitian), numpy's matmul as the library routine."""
    for seed in range(5):
        m, vals, x = _complex_case(30 + seed)
        u = _dense_upper(m, vals)
        d = np.diag(np.diag(u))
        a = u + (u.conj().T - d.conj() if hermitian else u.T - d)
        ref = a @ x
        for y in (O.symm_spmv_complex_loop(m.n, m.row_ptr, m.col, vals, x, hermitian),
                  O.symm_spmv_complex(m.n, m.row_ptr, m.col, vals, x, hermitian)):
            assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


def test_complex_properties():
    m, vals, x = _complex_case(7)
    # real values: both complex forms reduce to the real product
    xr = np.real(x)
    for h in (False, True):
        y = O.symm_spmv_complex(m.n, m.row_ptr, m.col, m.val.astype(np.complex128), xr, h)
        assert np.abs(y - O.symm_spmv(m.n, m.row_ptr, m.col, m.val, xr)).max() <= 1e-13 * np.abs(y).max()
    # a Hermitian matrix with a real diagonal: x^H A x is real
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    herm_vals = np.where(rows == m.col, np.real(vals), vals)
    q = np.vdot(x, O.symm_spmv_complex(m.n, m.row_ptr, m.col, herm_vals, x, True))
    assert abs(q.imag) <= 1e-12 * abs(q)
    # the transpose identity of a complex symmetric matrix: y^T (A x) = x^T (A y)
    z = np.random.default_rng(8).standard_normal(m.n) + 1j
    ax = O.symm_spmv_complex(m.n, m.row_ptr, m.col, vals, x, False)
    az = O.symm_spmv_complex(m.n, m.row_ptr, m.col, vals, z, False)
    assert abs(z @ ax - x @ az) <= 1e-12 * abs(z @ ax)
    # the two kinds differ once off-diagonal values have imaginary parts
    assert np.abs(O.symm_spmv_complex(m.n, m.row_ptr, m.col, vals, x, True) - ax).max() > 1e-3
