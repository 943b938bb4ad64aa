"""Pins for the Gauss-Seidel oracle and distance-1 RACE schedules (CPU only).

* A forward sweep in the natural order is the triangular solve
  (D + L) x' = b - U x; a backward sweep is (D + U) x' = b - L x (dense,
  scipy's triangular solver); the symmetric sweep is the two in a row.
* The exact solution is a fixed point; on SPD matrices symmetric sweeps
  lower the energy norm of the error.
* The plain C sweep is bit-equal to the Python sweep.
* Distance-1 schedules (Section 4.2: single levels alternate colors; the
  recursion takes the subgraph of the group alone, Section 4.4.1) pass the
  checker's distance-1 rule and the dense (I + A) check; leaves of one phase
  may then run in any order, so shuffling them leaves the sweep bit-equal.
* Planted mistakes (a Jacobi update with the old values, merged phases) fail.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import matgen
from oracle import checker as C
from oracle import gauss_seidel as G
from oracle import schedule as S
from oracle import symmspmv as O


def dense(m):
    return O.upper_matrix(m.n, m.row_ptr, m.col, m.val).toarray()


def full_dense(m):
    u = dense(m)
    return u + u.T - np.diag(np.diag(u))


SMALL = [
    ("2d5pt_9", lambda: matgen.stencil2d_5pt(9, seed=1)),
    ("3d27pt_5", lambda: matgen.stencil3d_27pt(5, seed=2)),
    ("banded_150", lambda: matgen.banded_irregular(150, seed=3, band=12)),
    ("rand_120", lambda: matgen.random_symmetric(120, 0.05, seed=4)),
]


def spd(m):
    """The same pattern made symmetric positive definite: diagonal = 1 +
    absolute off-diagonal row sum (strict diagonal dominance)."""
    a = full_dense(m)
    off = np.abs(a).sum(axis=1) - np.abs(np.diag(a))
    v = m.val.copy()
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    d = rows == m.col
    v[d] = 1.0 + off[rows[d]]
    return matgen.UpperCSR(m.n, m.row_ptr, m.col, v, m.name + "_spd")


@pytest.mark.parametrize("name,make", SMALL, ids=[c[0] for c in SMALL])
def test_sweeps_are_triangular_solves(name, make):
    m = spd(make())
    a = full_dense(m)
    low = np.tril(a, -1)
    up = np.triu(a, 1)
    dg = np.diag(np.diag(a))
    rng = np.random.default_rng(5)
    b = rng.standard_normal(m.n)
    x = rng.standard_normal(m.n)
    nat = list(range(m.n))
    fwd = G.sweep(m.n, m.row_ptr, m.col, m.val, b, x, nat)
    ref_f = sla.solve_triangular(dg + low, b - up @ x, lower=True)
    assert np.allclose(fwd, ref_f, rtol=1e-12, atol=1e-12 * np.abs(ref_f).max())
    bwd = G.sweep(m.n, m.row_ptr, m.col, m.val, b, x, nat[::-1])
    ref_b = sla.solve_triangular(dg + up, b - low @ x, lower=False)
    assert np.allclose(bwd, ref_b, rtol=1e-12, atol=1e-12 * np.abs(ref_b).max())
    sym = G.symmetric_sweep(m.n, m.row_ptr, m.col, m.val, b, x, nat)
    ref_s = sla.solve_triangular(dg + up, b - low @ ref_f, lower=False)
    assert np.allclose(sym, ref_s, rtol=1e-11, atol=1e-11 * np.abs(ref_s).max())


def test_fixed_point_and_energy_decrease():
    m = spd(matgen.stencil3d_27pt(6, seed=7))
    a = full_dense(m)
    rng = np.random.default_rng(8)
    xs = rng.standard_normal(m.n)
    b = a @ xs
    order = list(rng.permutation(m.n))
    x1 = G.symmetric_sweep(m.n, m.row_ptr, m.col, m.val, b, xs, order)
    assert np.allclose(x1, xs, rtol=0, atol=1e-12 * np.abs(xs).max())
    x = np.zeros(m.n)
    energy = []
    for _ in range(6):
        e = x - xs
        energy.append(float(e @ a @ e))
        x = G.symmetric_sweep(m.n, m.row_ptr, m.col, m.val, b, x, order)
    assert all(e1 < e0 for e0, e1 in zip(energy, energy[1:]))


def test_c_sweep_bit_equal():
    for seed, m in enumerate([matgen.banded_irregular(3000, seed=9, band=200), matgen.stencil3d_27pt(9, seed=10),
                              matgen.random_symmetric(500, 0.01, seed=11)]):
        m = spd(m) if m.n <= 800 else m
        rng = np.random.default_rng(20 + seed)
        b = rng.standard_normal(m.n)
        x = rng.standard_normal(m.n)
        order = rng.permutation(m.n)
        assert np.array_equal(G.sweep(m.n, m.row_ptr, m.col, m.val, b, x, order),
                              G.sweep_c(m.n, m.row_ptr, m.col, m.val, b, x, order))
        assert np.array_equal(G.symmetric_sweep(m.n, m.row_ptr, m.col, m.val, b, x, order),
                              G.symmetric_sweep_c(m.n, m.row_ptr, m.col, m.val, b, x, order))


D1_CASES = [
    ("2d5pt_100", matgen.config_2d_small, 64),
    ("3d27pt_14", lambda: matgen.stencil3d_27pt(14, seed=5), 128),
    ("banded_20k", lambda: matgen.banded_irregular(20000, seed=6, band=2000), 64),
    ("rand_islands", lambda: matgen.random_symmetric(400, 0.004, seed=8), 12),
    ("worked_16x16", lambda: matgen.stencil2d_7pt(16), 8),
]


def _leaf_ranges(sch):
    lo = [sch.nodes[i].lo for i in sch.leaves]
    hi = [sch.nodes[i].hi for i in sch.leaves]
    return lo, hi


@pytest.mark.parametrize("name,make,nt", D1_CASES, ids=[c[0] for c in D1_CASES])
def test_distance1_schedules_pass_the_checker(name, make, nt):
    m = make()
    sch = S.build_schedule(m.n, m.row_ptr, m.col, nt, k=1)
    nodes = sch.nodes
    C.check_schedule(m.n, m.row_ptr, m.col, sch.perm, [nd.lo for nd in nodes], [nd.hi for nd in nodes],
                     [nd.color for nd in nodes], [nd.parent for nd in nodes], sch.leaves, sch.leaf_phase, dist=1)
    lo, hi = _leaf_ranges(sch)
    if m.n <= 2000:
        C.check_dense_distance_k(m.n, m.row_ptr, m.col, sch.perm, lo, hi, sch.leaf_phase, 1)


def test_distance1_stage0_levels_alternate():
    # stage 0 of a distance-1 schedule on the 16 x 16 example with one
    # thread per group: groups of single levels are allowed (>= k = 1 level)
    m = matgen.stencil2d_7pt(16)
    sch = S.build_schedule(m.n, m.row_ptr, m.col, 8, eps=(0.6, 0.6), balance="rows", k=1, max_stages=1)
    st0 = [nd for nd in sch.nodes if nd.stage == 0]
    assert [nd.color for nd in st0] == [i % 2 for i in range(len(st0))]
    assert sum(nd.hi - nd.lo for nd in st0) == m.n


@pytest.mark.parametrize("name,make,nt", D1_CASES[:4], ids=[c[0] for c in D1_CASES[:4]])
def test_shuffled_leaves_within_a_phase_give_the_same_sweep(name, make, nt):
    m = make()
    sch = S.build_schedule(m.n, m.row_ptr, m.col, nt, k=1)
    lo, hi = _leaf_ranges(sch)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(m.n)
    x = rng.standard_normal(m.n)
    order = G.race_order(sch.perm, lo, hi, sch.leaf_phase)
    ref = G.symmetric_sweep_c(m.n, m.row_ptr, m.col, m.val, b, x, order)
    # the same phases with their leaves in a random order
    leaves = list(zip(sch.leaf_phase, lo, hi))
    rng.shuffle(leaves)
    leaves.sort(key=lambda t: t[0])  # stable: phases in order, leaves shuffled inside
    order2 = [int(sch.perm[r]) for _, a, b_ in leaves for r in range(a, b_)]
    assert sorted(order2) == sorted(order)
    assert np.array_equal(G.symmetric_sweep_c(m.n, m.row_ptr, m.col, m.val, b, x, order2), ref)


def test_planted_jacobi_update_fails():
    m = spd(matgen.stencil2d_5pt(7, seed=2))
    a = full_dense(m)
    rng = np.random.default_rng(4)
    b = rng.standard_normal(m.n)
    x = rng.standard_normal(m.n)
    # Jacobi: every row with the old values
    dg = np.diag(a)
    jac = (b - (a - np.diag(dg)) @ x) / dg
    ref = sla.solve_triangular(np.tril(a), b - np.triu(a, 1) @ x, lower=True)
    assert not np.allclose(jac, ref, rtol=1e-12, atol=1e-12)


def test_checker_rejects_merged_distance1_phases():
    m = matgen.config_2d_small()
    sch = S.build_schedule(m.n, m.row_ptr, m.col, 64, k=1)
    nodes = sch.nodes
    with pytest.raises(AssertionError):
        C.check_schedule(m.n, m.row_ptr, m.col, sch.perm, [nd.lo for nd in nodes], [nd.hi for nd in nodes],
                         [nd.color for nd in nodes], [nd.parent for nd in nodes], sch.leaves,
                         np.zeros_like(sch.leaf_phase), dist=1)
