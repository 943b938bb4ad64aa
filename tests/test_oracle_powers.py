"""Pins of the matrix-power and polynomial oracle (oracle/powers.py) against
what mathematics fixes: powers of a diagonal matrix, an eigenvector of the
path Laplacian (Dirichlet), numpy's dense matrix_power on small random
symmetric matrices, and the binomial identity (I + A)^2 = I + 2A + A^2.
Planted mistakes (an off-by-one power, a dropped constant term) fail."""
import math

import numpy as np
import pytest

import matgen
from oracle import powers as P
from oracle import symmspmv as O


def _diag(d):
    n = len(d)
    return matgen.UpperCSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.asarray(d, float))


def _path_laplacian(n):
    rp = [0]
    col, val = [], []
    for i in range(n):
        col.append(i)
        val.append(2.0)
        if i + 1 < n:
            col.append(i + 1)
            val.append(-1.0)
        rp.append(len(col))
    return matgen.UpperCSR(n, np.array(rp, np.int32), np.array(col, np.int32), np.array(val))


@pytest.mark.parametrize("product", ["c", "scipy"])
def test_powers_of_a_diagonal_matrix_are_elementwise(product):
    d = np.array([2.0, -3.0, 0.5, 1.0, 0.0])
    m = _diag(d)
    x = np.array([1.0, 2.0, -1.0, 4.0, 7.0])
    ys = P.powers(m.n, m.row_ptr, m.col, m.val, x, 6, product)
    for p, y in enumerate(ys, start=1):
        assert np.array_equal(y, d ** p * x)  # exact: small powers of these values are representable


def test_path_laplacian_eigenvector():
    """sin(k pi j / (n + 1)) is an eigenvector with eigenvalue
    2 - 2 cos(k pi / (n + 1)); the largest one (k = n) keeps the rounding
    of the other components from growing faster than lambda^p."""
    n = 40
    m = _path_laplacian(n)
    j = np.arange(1, n + 1)
    for k in (n, n - 1):
        v = np.sin(k * math.pi * j / (n + 1))
        lam = 2.0 - 2.0 * math.cos(k * math.pi / (n + 1))
        for p, y in enumerate(P.powers(m.n, m.row_ptr, m.col, m.val, v, 8), start=1):
            assert np.max(np.abs(y - lam ** p * v)) <= 1e-12 * lam ** p


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_powers_match_dense_matrix_power(seed):
    m = matgen.random_symmetric(60, 0.1, seed=seed)
    dense = O.upper_matrix(m.n, m.row_ptr, m.col, m.val).toarray()
    dense = dense + dense.T - np.diag(np.diag(dense))
    x = np.random.default_rng(seed).uniform(-1, 1, m.n)
    for p, y in enumerate(P.powers(m.n, m.row_ptr, m.col, m.val, x, 5), start=1):
        ref = np.linalg.matrix_power(dense, p) @ x
        assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_polynomial_binomial_identity():
    m = matgen.stencil2d_5pt(12, seed=4)
    x = np.random.default_rng(5).uniform(-1, 1, m.n)
    z = P.poly(m.n, m.row_ptr, m.col, m.val, [1.0, 2.0, 1.0], x)
    w = x + O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x)          # (I + A) x
    w = w + O.symm_spmv(m.n, m.row_ptr, m.col, m.val, w)          # (I + A)^2 x
    assert np.max(np.abs(z - w)) <= 1e-13 * np.max(np.abs(w))
    # degree 0 is the scaled vector
    assert np.array_equal(P.poly(m.n, m.row_ptr, m.col, m.val, [3.0], x), 3.0 * x)


def test_planted_mistakes_fail():
    d = np.array([2.0, 3.0])
    m = _diag(d)
    x = np.array([1.0, 1.0])
    off_by_one = [x] + P.powers(m.n, m.row_ptr, m.col, m.val, x, 2)[:-1]  # A^(p-1) x
    assert not np.array_equal(off_by_one[1], d ** 2 * x)
    z_no_c0 = 2.0 * P.powers(m.n, m.row_ptr, m.col, m.val, x, 1)[0]
    z = P.poly(m.n, m.row_ptr, m.col, m.val, [1.0, 2.0], x)
    assert np.array_equal(z, x + 2.0 * d * x) and not np.array_equal(z, z_no_c0)
