"""Pins for the Kaczmarz oracle (CPU only).

* A forward Kaczmarz sweep with relaxation omega from x0 is x0 + A^T u,
  where u is one SOR sweep from zero on the row-action system
  A A^T u = b - A x0 in the same row order (Bjorck and Elfving, 1979):
  u = omega (D + omega L)^{-1} (b - A x0), D and L the diagonal and strict
  lower part of A A^T with rows and columns in sweep order (dense, scipy's
  triangular solver).  This fixes the dot product, the squared row norm
  (the diagonal of A A^T), the relaxation and the direction of the update.
* With omega = 1 the projected row holds exactly afterwards; with
  omega = 2 every step is a reflection, which keeps |x - x*| for a
  consistent system, and 0 < omega < 2 shrinks it.
* A row with no stored value leaves x alone.
* The plain C sweep is bit-equal to the Python sweep.
* On a distance-2 schedule (Section 4.2) leaves of one phase share no
  column, so shuffling them leaves the sweep bit-equal; on a distance-1
  schedule they may share one, and the shuffled sweep differs.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import matgen
from oracle import gauss_seidel as G
from oracle import kaczmarz as K
from oracle import schedule as S
from oracle import symmspmv as O


def full_dense(m):
    u = O.upper_matrix(m.n, m.row_ptr, m.col, m.val).toarray()
    return u + u.T - np.diag(np.diag(u))


SMALL = [
    ("2d5pt_9", lambda: matgen.stencil2d_5pt(9, seed=1)),
    ("3d27pt_5", lambda: matgen.stencil3d_27pt(5, seed=2)),
    ("banded_150", lambda: matgen.banded_irregular(150, seed=3, band=12)),
    ("rand_120", lambda: matgen.random_symmetric(120, 0.05, seed=4)),
]


def row_action_sweep(a, b, x0, order, omega):
    """Kaczmarz through its SOR form on A A^T (dense)."""
    p = np.asarray(order)
    ap = a[p, :]
    m = ap @ ap.T
    r = (b - a @ x0)[p]
    u = omega * sla.solve_triangular(np.diag(np.diag(m)) + omega * np.tril(m, -1), r, lower=True)
    return x0 + ap.T @ u


@pytest.mark.parametrize("omega", [1.0, 0.6, 1.5])
@pytest.mark.parametrize("name,make", SMALL, ids=[c[0] for c in SMALL])
def test_sweep_is_sor_on_the_row_action_system(name, make, omega):
    m = make()
    a = full_dense(m)
    assert np.all(np.abs(a).sum(axis=1) > 0)
    rng = np.random.default_rng(7)
    b = rng.standard_normal(m.n)
    x0 = rng.standard_normal(m.n)
    for order in (np.arange(m.n), rng.permutation(m.n)):
        ref = row_action_sweep(a, b, x0, order, omega)
        got = K.sweep(m.n, m.row_ptr, m.col, m.val, b, x0, order, omega)
        assert np.max(np.abs(got - ref)) <= 1e-10 * max(1.0, np.max(np.abs(ref)))
        back = K.sweep(m.n, m.row_ptr, m.col, m.val, b, x0, order[::-1], omega)
        assert np.max(np.abs(back - row_action_sweep(a, b, x0, order[::-1], omega))) <= 1e-10 * max(
            1.0, np.max(np.abs(back)))


def test_planted_mistakes_fail_the_row_action_pin():
    """A norm without the diagonal, an update without it, and the old x in
    every dot product (a Jacobi-style Cimmino step) all differ from the SOR
    form: the pin above would catch each."""
    m = matgen.stencil2d_5pt(7, seed=2)
    a = full_dense(m)
    rng = np.random.default_rng(4)
    b = rng.standard_normal(m.n)
    x0 = rng.standard_normal(m.n)
    ref = row_action_sweep(a, b, x0, np.arange(m.n), 1.0)
    d = np.diag(a)
    off = a - np.diag(d)
    x = x0.copy()
    for i in range(m.n):  # norm of the off-diagonal part only
        x += (b[i] - a[i] @ x) / (off[i] @ off[i]) * a[i]
    assert not np.allclose(x, ref, rtol=1e-8, atol=1e-8)
    x = x0.copy()
    for i in range(m.n):  # the diagonal left out of the update
        x += (b[i] - a[i] @ x) / (a[i] @ a[i]) * off[i]
    assert not np.allclose(x, ref, rtol=1e-8, atol=1e-8)
    x = x0 + sum((b[i] - a[i] @ x0) / (a[i] @ a[i]) * a[i] for i in range(m.n))
    assert not np.allclose(x, ref, rtol=1e-8, atol=1e-8)


def test_projection_reflection_and_contraction():
    m = matgen.stencil3d_27pt(4, seed=9)
    a = full_dense(m)
    rng = np.random.default_rng(5)
    xs = rng.standard_normal(m.n)
    b = a @ xs
    x0 = rng.standard_normal(m.n)
    # omega = 1: the projected row holds
    for i in (0, m.n // 2, m.n - 1):
        x1 = K.sweep(m.n, m.row_ptr, m.col, m.val, b, x0, [i], 1.0)
        assert abs(a[i] @ x1 - b[i]) <= 1e-12 * max(1.0, abs(b[i]))
    # omega = 2: reflections keep the distance to the solution
    x2 = K.sweep(m.n, m.row_ptr, m.col, m.val, b, x0, range(m.n), 2.0)
    e0 = np.linalg.norm(x0 - xs)
    assert abs(np.linalg.norm(x2 - xs) - e0) <= 1e-10 * e0
    # 0 < omega < 2: every symmetric sweep shrinks it
    for omega in (0.5, 1.0, 1.7):
        x = x0
        e = e0
        for _ in range(4):
            x = K.symmetric_sweep(m.n, m.row_ptr, m.col, m.val, b, x, range(m.n), omega)
            e1 = np.linalg.norm(x - xs)
            assert e1 < e
            e = e1


def test_empty_row_is_skipped():
    # row 2 stores nothing and no other row reaches it
    rp = np.array([0, 2, 3, 3, 4], np.int32)
    col = np.array([0, 1, 1, 3], np.int32)
    val = np.array([2.0, -1.0, 3.0, 4.0])
    b = np.array([1.0, 2.0, 5.0, 8.0])
    x0 = np.array([0.5, -0.5, 7.0, 1.0])
    x = K.sweep(4, rp, col, val, b, x0, range(4), 1.0)
    assert x[2] == 7.0
    assert np.array_equal(K.sweep_c(4, rp, col, val, b, x0, range(4), 1.0), x)
    assert abs(4.0 * x[3] - 8.0) <= 1e-15


@pytest.mark.parametrize("name,make", SMALL, ids=[c[0] for c in SMALL])
def test_c_sweep_bit_equal(name, make):
    m = make()
    rng = np.random.default_rng(8)
    b = rng.standard_normal(m.n)
    x0 = rng.standard_normal(m.n)
    order = rng.permutation(m.n)
    for omega in (1.0, 1.3):
        assert np.array_equal(K.sweep_c(m.n, m.row_ptr, m.col, m.val, b, x0, order, omega),
                              K.sweep(m.n, m.row_ptr, m.col, m.val, b, x0, order, omega))
        assert np.array_equal(K.symmetric_sweep_c(m.n, m.row_ptr, m.col, m.val, b, x0, order, omega),
                              K.symmetric_sweep(m.n, m.row_ptr, m.col, m.val, b, x0, order, omega))


def _shuffled(sch, rng):
    lo = [sch.nodes[i].lo for i in sch.leaves]
    hi = [sch.nodes[i].hi for i in sch.leaves]
    order = G.race_order(sch.perm, lo, hi, sch.leaf_phase)
    leaves = list(zip(sch.leaf_phase, lo, hi))
    rng.shuffle(leaves)
    leaves.sort(key=lambda t: t[0])  # stable: phases in order, leaves shuffled inside
    return order, [int(sch.perm[r]) for _, a, b_ in leaves for r in range(a, b_)]


D2_CASES = [
    ("2d5pt_100", matgen.config_2d_small, 64),
    ("3d27pt_14", lambda: matgen.stencil3d_27pt(14, seed=5), 64),
    ("banded_20k", lambda: matgen.banded_irregular(20000, seed=6, band=2000), 64),
    ("rand_islands", lambda: matgen.random_symmetric(400, 0.004, seed=8), 12),
]


@pytest.mark.parametrize("name,make,nt", D2_CASES, ids=[c[0] for c in D2_CASES])
def test_distance2_leaves_of_a_phase_commute(name, make, nt):
    m = make()
    sch = S.build_schedule(m.n, m.row_ptr, m.col, nt, k=2)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(m.n)
    x = rng.standard_normal(m.n)
    order, order2 = _shuffled(sch, rng)
    assert sorted(order2) == sorted(order) and order2 != order
    ref = K.symmetric_sweep_c(m.n, m.row_ptr, m.col, m.val, b, x, order)
    assert np.array_equal(K.symmetric_sweep_c(m.n, m.row_ptr, m.col, m.val, b, x, order2), ref)


def test_distance1_leaves_of_a_phase_do_not_commute():
    """Leaves of a distance-1 phase share no edge but may share a column:
    then the order among them changes the Kaczmarz sweep (the reason it
    runs on distance-2 schedules)."""
    m = matgen.config_2d_small()
    sch = S.build_schedule(m.n, m.row_ptr, m.col, 64, k=1)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(m.n)
    x = rng.standard_normal(m.n)
    order, order2 = _shuffled(sch, rng)
    assert not np.array_equal(K.sweep_c(m.n, m.row_ptr, m.col, m.val, b, x, order2),
                              K.sweep_c(m.n, m.row_ptr, m.col, m.val, b, x, order))
