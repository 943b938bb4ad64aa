"""Pins for the RACE schedule oracle (CPU only).

* BFS levels against closed forms on grids and the edge invariant.
* The epsilon aggregation, pair balancing, recursion and eta against the
  numbers the paper prints for its 16 x 16 example (tests/golden).
* Load-balancing invariants (its worked examples and plants are in
  test_oracle_loadbalance.py).
* Every schedule passes the independent brute-force conflict checker, and the
  checker rejects planted conflicts.
"""
import json
import os

import numpy as np
import pytest

import matgen
from oracle import checker as C
from oracle import schedule as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def levels_full(m):
    ptr, idx = S.full_adjacency(m.n, m.row_ptr, m.col)
    scratch = np.full(m.n, -1, dtype=np.int64)
    return S.bfs_levels(ptr, idx, np.arange(m.n), np.ones(m.n, dtype=bool), scratch)


def test_bfs_closed_form_2d5pt():
    side = 13
    lev = levels_full(matgen.stencil2d_5pt(side, seed=1))
    i, j = np.divmod(np.arange(side * side), side)
    assert np.array_equal(lev, i + j)
    assert np.array_equal(np.bincount(lev), np.minimum(np.arange(2 * side - 1) + 1, 2 * side - 1 - np.arange(2 * side - 1)))


def test_bfs_closed_form_3d27pt():
    side = 9
    lev = levels_full(matgen.stencil3d_27pt(side, seed=2))
    z, rem = np.divmod(np.arange(side ** 3), side * side)
    y, x = np.divmod(rem, side)
    assert np.array_equal(lev, np.maximum(np.maximum(x, y), z))
    d = np.arange(side)
    assert np.array_equal(np.bincount(lev), 3 * d * d + 3 * d + 1)


def test_bfs_closed_form_2d7pt():
    side = 16
    lev = levels_full(matgen.stencil2d_7pt(side))
    i, j = np.divmod(np.arange(side * side), side)
    assert np.array_equal(lev, i + j)


@pytest.mark.parametrize("seed", range(5))
def test_bfs_edge_invariant_random(seed):
    m = matgen.random_symmetric(60, 0.06, seed=seed)
    lev = levels_full(m)
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    ptr, idx = S.full_adjacency(m.n, m.row_ptr, m.col)
    assert lev[0] == 0
    # within an island adjacent vertices differ by at most one level, and
    # islands never share a level with the previous one
    assert np.all(np.abs(lev[rows] - lev[m.col]) <= 1)
    # level L > 0 of the first island: every vertex has a neighbour at L - 1
    for v in range(m.n):
        if lev[v] > 0:
            nb = idx[ptr[v]:ptr[v + 1]]
            assert np.any(lev[nb] == lev[v] - 1) or not np.any(lev[nb] < lev[v])


def test_islands_restart_two_levels_up():
    # two disjoint paths 0-1-2 and 3-4
    rp = np.array([0, 2, 4, 5, 7, 8], dtype=np.int32)
    col = np.array([0, 1, 1, 2, 2, 3, 4, 4], dtype=np.int32)
    m = matgen.UpperCSR(5, rp, col, np.ones(8))
    lev = levels_full(m)
    assert lev.tolist() == [0, 1, 2, 4, 5]


def test_worked_example_aggregation():
    g = json.load(open(os.path.join(GOLDEN, "worked_example_16x16.json")))
    sizes = g["level_sizes"]
    assert sum(sizes) == 256
    pairs = S.aggregate_pairs(np.array(sizes), g["n_threads"], g["eps0"], 2)
    p0 = g["first_pair"]
    assert pairs[0] == [p0["levels"][0], p0["levels"][1], p0["b"]]
    assert sum(sizes[p0["levels"][0]:p0["levels"][1]]) == p0["weight_num"]
    p2 = g["third_pair"]
    assert pairs[2] == [p2["levels"][0], p2["levels"][1], p2["b"]]
    assert sum(sizes[p2["levels"][0]:p2["levels"][1]]) == p2["weight_num"]
    # the pair after the first two starts at vertex 66
    assert sum(sizes[:pairs[2][0]]) == g["t0_4_first_vertex"]
    assert sum(p[2] for p in pairs) == g["n_threads"]


def test_worked_example_tree_and_eta():
    g = json.load(open(os.path.join(GOLDEN, "worked_example_16x16.json")))
    m = matgen.stencil2d_7pt(16)
    assert np.array_equal(np.bincount(levels_full(m)), g["level_sizes"])
    sch = S.build_schedule(m.n, m.row_ptr, m.col, g["n_threads"], eps=(g["eps0"], g["eps0"]), balance=g["balance"])
    st0 = [nd for nd in sch.nodes if nd.stage == 0]
    assert st0[0].hi - st0[0].lo == g["n_eff_t0_0"]
    assert (st0[4].lo, st0[4].hi - 1) == (g["t0_4_first_vertex"], g["t0_4_last_vertex"])
    assert [i for i, nd in enumerate(st0) if nd.b > 1] == g["refined_stage0_groups"]
    assert sum(1 for nd in sch.nodes if nd.stage == 1) == g["stage1_groups"]
    assert sch.n_eff_root == g["n_eff_root"]
    assert sch.eta == pytest.approx(g["eta_num"] / g["eta_den"])


def test_aggregation_cases():
    # fewer than two pairs -> no refinement
    assert S.aggregate_pairs(np.array([1, 1, 1, 1, 1]), 4, 0.5, 2) == []
    assert S.aggregate_pairs(np.array([0, 0, 0, 0, 0, 0, 0, 0]), 4, 0.5, 2) == []
    # a short tail joins the previous pair
    pairs = S.aggregate_pairs(np.array([5, 5, 5, 5, 5, 5, 5, 5, 1, 1]), 2, 0.8, 2)
    assert pairs[-1][1] == 10
    # levels always covered contiguously, every pair >= 2k levels
    rng = np.random.default_rng(0)
    for _ in range(200):
        ml = rng.integers(0, 50, size=rng.integers(4, 60))
        nt = int(rng.integers(1, 40))
        pairs = S.aggregate_pairs(ml, nt, float(rng.uniform(0.5, 0.95)), 2)
        if not pairs:
            continue
        assert pairs[0][0] == 0 and pairs[-1][1] == len(ml)
        for (s, e, b), nxt in zip(pairs, pairs[1:] + [None]):
            assert e - s >= 4 and b >= 1
            if nxt:
                assert nxt[0] == e


def test_pair_split_balances_each_pair():
    rng = np.random.default_rng(1)
    for _ in range(300):
        nl = int(rng.integers(4, 20))
        ml = rng.integers(0, 30, size=nl)
        t_ptr, worker = S.split_pairs([[0, nl, 3]], ml, 2)
        r = t_ptr[1]
        assert r - 0 >= 2 and nl - r >= 2
        red, blue = int(ml[:r].sum()), int(ml[r:].sum())
        # no single-level move would strictly improve |red - blue|
        if red > blue and r > 2:
            x = int(ml[r - 1])
            assert not abs((red - x) - (blue + x)) < abs(red - blue)
        if blue > red and nl - r > 2:
            x = int(ml[r])
            assert not abs((red + x) - (blue - x)) < abs(red - blue)


def test_load_balance_invariants():
    rng = np.random.default_rng(2)
    k = 2
    for _ in range(100):
        npairs = int(rng.integers(2, 8))
        nl = int(rng.integers(4 * npairs, 6 * npairs + 8))
        ml = rng.integers(0, 100, size=nl)
        # pairs of >= 4 levels
        cuts = sorted(rng.choice(np.arange(1, nl // 4), size=npairs - 1, replace=False) * 4)
        bounds = [0] + list(cuts) + [nl]
        pairs = [[bounds[i], bounds[i + 1], int(rng.integers(1, 4))] for i in range(npairs)]
        if any(e - s < 4 for s, e, _ in pairs):
            continue
        t0, worker = S.split_pairs(pairs, ml, k)
        prefix = np.concatenate([[0], np.cumsum(ml)])
        _, var0 = S._variance(t0, worker, prefix)
        t1 = S.load_balance(t0, worker, ml, k)
        _, var1 = S._variance(t1, worker, prefix)
        assert t1[0] == t0[0] and t1[-1] == t0[-1]
        assert all(t1[i + 1] - t1[i] >= k for i in range(len(worker)))
        assert var1 <= var0


def _check(m, sch):
    nodes = sch.nodes
    return C.check_schedule(m.n, m.row_ptr, m.col, sch.perm, [nd.lo for nd in nodes], [nd.hi for nd in nodes],
                            [nd.color for nd in nodes], [nd.parent for nd in nodes], sch.leaves, sch.leaf_phase)


CASES = [
    ("2d5pt_100", lambda: matgen.config_2d_small(), 64),
    ("3d27pt_16", lambda: matgen.stencil3d_27pt(16, seed=5), 48),
    ("banded_20k", lambda: matgen.banded_irregular(20000, seed=6, band=2000), 64),
    ("rand_300", lambda: matgen.random_symmetric(300, 0.01, seed=7), 8),
    ("rand_disconnected", lambda: matgen.random_symmetric(200, 0.004, seed=8), 6),
]


@pytest.mark.parametrize("name,make,nt", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("balance", ["nnz", "rows"])
def test_schedule_passes_checker(name, make, nt, balance):
    m = make()
    sch = S.build_schedule(m.n, m.row_ptr, m.col, nt, balance=balance)
    _check(m, sch)
    if m.n <= 2000:
        lo = [sch.nodes[i].lo for i in sch.leaves]
        hi = [sch.nodes[i].hi for i in sch.leaves]
        C.check_dense_distance2(m.n, m.row_ptr, m.col, sch.perm, lo, hi, sch.leaf_phase)


def test_global_lb_schedule_passes_checker():
    m = matgen.stencil3d_27pt(14, seed=9)
    sch = S.build_schedule(m.n, m.row_ptr, m.col, 40, global_lb=True)
    _check(m, sch)


def test_checker_rejects_planted_conflicts():
    m = matgen.config_2d_small()
    sch = S.build_schedule(m.n, m.row_ptr, m.col, 64)
    _check(m, sch)
    # all leaves in one phase: adjacent groups conflict
    with pytest.raises(AssertionError):
        C.check_schedule(m.n, m.row_ptr, m.col, sch.perm, [nd.lo for nd in sch.nodes], [nd.hi for nd in sch.nodes],
                         [nd.color for nd in sch.nodes], [nd.parent for nd in sch.nodes], sch.leaves,
                         np.zeros_like(sch.leaf_phase))
    # wrong permutation: the identity no longer separates the groups
    with pytest.raises(AssertionError):
        C.check_schedule(m.n, m.row_ptr, m.col, np.arange(m.n), [nd.lo for nd in sch.nodes],
                         [nd.hi for nd in sch.nodes], [nd.color for nd in sch.nodes],
                         [nd.parent for nd in sch.nodes], sch.leaves, sch.leaf_phase)
    # the paper's own wrong variant (Section 4.4.2): recursing on the subgraph
    # induced by the group alone, without its neighbourhood, lets two rows of
    # one group meet through a vertex outside it (planted in the oracle)
    orig = S.subgraph_vertices
    caught = 0
    try:
        S.subgraph_vertices = lambda ptr, idx, members, k=2: members
        for seed in range(4):
            g = matgen.banded_irregular(3000, seed=100 + seed, band=300)
            bad = S.build_schedule(g.n, g.row_ptr, g.col, 32)
            try:
                _check(g, bad)
            except AssertionError:
                caught += 1
    finally:
        S.subgraph_vertices = orig
    assert caught > 0
    # and the correct recursion passes on the same inputs
    for seed in range(4):
        g = matgen.banded_irregular(3000, seed=100 + seed, band=300)
        _check(g, S.build_schedule(g.n, g.row_ptr, g.col, 32))
    # swapped colors of two siblings are rejected
    nodes = sch.nodes
    color = [nd.color for nd in nodes]
    c0, c1 = nodes[0].children[0], nodes[0].children[1]
    color[c0], color[c1] = color[c1], color[c0]
    with pytest.raises(AssertionError):
        C.check_schedule(m.n, m.row_ptr, m.col, sch.perm, [nd.lo for nd in nodes], [nd.hi for nd in nodes],
                         color, [nd.parent for nd in nodes], sch.leaves, sch.leaf_phase)


def test_phase_numbering():
    m = matgen.stencil2d_7pt(16)
    sch = S.build_schedule(m.n, m.row_ptr, m.col, 8, eps=(0.6, 0.6), balance="rows")
    assert sch.n_phases == 4
    for leaf, ph in zip(sch.leaves, sch.leaf_phase):
        nd = sch.nodes[leaf]
        if nd.stage == 0:
            assert ph == 2 * nd.color
        else:
            assert ph == 2 * sch.nodes[nd.parent].color + nd.color
    assert list(sch.leaf_phase) == sorted(sch.leaf_phase)


def test_trivial_inputs():
    # one row; a diagonal matrix (all islands); a path shorter than 2k levels
    for m in [matgen.UpperCSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.ones(1)),
              matgen.UpperCSR(6, np.arange(7, dtype=np.int32), np.arange(6, dtype=np.int32), np.ones(6)),
              matgen.stencil2d_5pt(2, seed=3)]:
        sch = S.build_schedule(m.n, m.row_ptr, m.col, 4)
        _check(m, sch)


# ---------------------------------------------------------------------------
# Stage-0 root and in-level numbering (pseudo-peripheral root, Cuthill-McKee)

def _graph(n, edges):
    """Upper CSR (unit values, unit diagonal) of an undirected edge list."""
    rows, cols = [], []
    for i in range(n):
        rows.append(i)
        cols.append(i)
    for a, b in edges:
        rows.append(min(a, b))
        cols.append(max(a, b))
    rows, cols = np.array(rows), np.array(cols)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rp = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    return matgen.UpperCSR(n, rp, cols.astype(np.int32), np.ones(len(cols)))


def _ecc_all(ptr, idx, n):
    """Eccentricity of every vertex by one BFS each (brute force)."""
    out = np.zeros(n, dtype=np.int64)
    for v in range(n):
        dist = np.full(n, -1)
        dist[v] = 0
        q = [v]
        for u in q:
            for w in idx[ptr[u]:ptr[u + 1]]:
                if dist[w] < 0:
                    dist[w] = dist[u] + 1
                    q.append(int(w))
        out[v] = dist.max()
    return out


def test_pseudo_peripheral_path_and_grid():
    # a path from its middle: the finder ends at an end vertex (eccentricity n - 1)
    n = 11
    m = _graph(n, [(i, i + 1) for i in range(n - 1)])
    ptr, idx = S.full_adjacency(m.n, m.row_ptr, m.col)
    assert S.pseudo_peripheral(ptr, idx, 5, n) in (0, n - 1)
    # a 2D grid from its centre: a corner (the diameter is reached)
    side = 9
    m = matgen.stencil2d_5pt(side)
    ptr, idx = S.full_adjacency(m.n, m.row_ptr, m.col)
    x = S.pseudo_peripheral(ptr, idx, (side // 2) * side + side // 2, m.n)
    assert x in (0, side - 1, side * (side - 1), side * side - 1)


def test_pseudo_peripheral_trees_reach_the_diameter():
    # on a tree, a farthest vertex of any vertex is peripheral, so the finder
    # reaches the diameter exactly
    rng = np.random.default_rng(3)
    for t in range(20):
        n = int(rng.integers(2, 60))
        edges = [(i, int(rng.integers(0, i))) for i in range(1, n)]
        m = _graph(n, edges)
        ptr, idx = S.full_adjacency(m.n, m.row_ptr, m.col)
        ecc = _ecc_all(ptr, idx, n)
        start = int(rng.integers(0, n))
        x = S.pseudo_peripheral(ptr, idx, start, n)
        assert ecc[x] == ecc.max(), t


def test_pseudo_peripheral_never_worse_than_the_start():
    rng = np.random.default_rng(4)
    for t in range(20):
        m = matgen.random_symmetric(int(rng.integers(5, 80)), 0.08, seed=100 + t)
        ptr, idx = S.full_adjacency(m.n, m.row_ptr, m.col)
        ecc = _ecc_all(ptr, idx, m.n)
        start = int(rng.integers(0, m.n))
        x = S.pseudo_peripheral(ptr, idx, start, m.n)
        dist, _ = S.level_structure(ptr, idx, start, m.n)
        assert dist[x] >= 0                      # same component
        assert ecc[start] <= ecc[x] <= ecc[dist >= 0].max()


def _check_cm_numbering(ptr, idx, n, lev, order):
    """Cuthill-McKee properties, checked from the definition: levels never
    decrease along the numbering; a vertex's parent (its lowest-numbered
    neighbour one level up) is numbered no later than the parent of the next
    vertex of the same island; children of one parent come by
    non-decreasing degree, equal degrees by index."""
    num = np.empty(n, dtype=np.int64)
    num[order] = np.arange(n)
    deg = np.diff(ptr)
    assert sorted(order.tolist()) == list(range(n))
    prev = None
    for v in order.tolist():
        up = [int(u) for u in idx[ptr[v]:ptr[v + 1]] if lev[u] == lev[v] - 1]
        parent = min(up, key=lambda u: num[u]) if up else None
        if prev is not None:
            pv, pp = prev
            assert lev[v] >= lev[pv] or parent is None
            if parent is not None and pp is not None:
                assert num[parent] >= num[pp]
                if parent == pp:
                    assert (deg[v], v) > (deg[pv], pv)
        prev = (v, parent)


def test_cuthill_mckee_numbering_properties():
    for m in (matgen.stencil2d_5pt(12), matgen.relabel(matgen.stencil2d_5pt(12), 5),
              matgen.random_symmetric(300, 0.01, seed=6), matgen.relabel(matgen.stencil3d_27pt(7, seed=2), 8)):
        ptr, idx = S.full_adjacency(m.n, m.row_ptr, m.col)
        for root_of in (None, lambda v: S.pseudo_peripheral(ptr, idx, v, m.n)):
            lev, order = S.cuthill_mckee_levels(ptr, idx, m.n, root_of)
            ref = levels_full(m) if root_of is None else None
            if ref is not None:
                assert np.array_equal(lev, ref)   # the same BFS levels as the input-order build
            _check_cm_numbering(ptr, idx, m.n, lev, order)


def test_cuthill_mckee_restores_a_banded_order():
    # a randomly relabelled path or grid gets its bandwidth back
    for m0, bw_max in ((_graph(40, [(i, i + 1) for i in range(39)]), 1), (matgen.stencil2d_5pt(15), 15)):
        m = matgen.relabel(m0, 9)
        ptr, idx = S.full_adjacency(m.n, m.row_ptr, m.col)
        _, order = S.cuthill_mckee_levels(ptr, idx, m.n, lambda v: S.pseudo_peripheral(ptr, idx, v, m.n))
        num = np.empty(m.n, dtype=np.int64)
        num[order] = np.arange(m.n)
        rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
        bw = int(np.abs(num[rows] - num[m.col]).max())
        bw_rand = int(np.abs(rows - m.col).max())
        assert bw <= bw_max < bw_rand, (bw, bw_rand)


def test_root_and_order_schedules_pass_the_checker():
    for root in ("first", "peripheral"):
        for lo in ("input", "cm"):
            m = matgen.relabel(matgen.stencil3d_27pt(9, seed=3), 4)
            sch = S.build_schedule(m.n, m.row_ptr, m.col, 16, root=root, level_order=lo)
            C.check_schedule(m.n, m.row_ptr, m.col, sch.perm, [nd.lo for nd in sch.nodes], [nd.hi for nd in sch.nodes],
                             [nd.color for nd in sch.nodes], [nd.parent for nd in sch.nodes], sch.leaves, sch.leaf_phase)


# ---------------------------------------------------------------------------
# Distance-k colorings, k >= 3 (Section 4.2): wider, still race-free

def _leaf_ranges(sch):
    return [sch.nodes[i].lo for i in sch.leaves], [sch.nodes[i].hi for i in sch.leaves]


@pytest.mark.parametrize("k", [1, 3, 4])
def test_distance_k_schedules_pass_the_dense_check(k):
    """Rows of different leaves of one phase are more than k apart ((I+A)^k
    has zeros there); for k >= 2 the touch-set checks hold as well."""
    for m in (matgen.stencil2d_5pt(30), matgen.random_symmetric(600, 0.005, seed=4),
              matgen.banded_irregular(1500, seed=5, band=120), matgen.stencil3d_27pt(9, seed=2)):
        sch = S.build_schedule(m.n, m.row_ptr, m.col, 32, k=k)
        lo, hi = _leaf_ranges(sch)
        C.check_dense_distance_k(m.n, m.row_ptr, m.col, sch.perm, lo, hi, sch.leaf_phase, k)
        if k >= 2:
            _check(m, sch)


def test_distance_k_recursion_needs_the_subgraph():
    """Recursing on the group T alone (no neighbourhood) lets two rows of a
    group meet within distance k through outside vertices; the dense
    distance-3 check catches it (planted in the oracle), and the correct
    recursion passes on the same inputs.  (A path of length k between two
    vertices of T runs within distance floor(k/2) of one of them, so the
    distance-(k-1) neighbourhood the recursion uses is more than enough.)"""
    orig = S.subgraph_vertices
    caught = 0
    mats = [matgen.banded_irregular(1500, seed=100 + s, band=60) for s in range(6)]
    try:
        S.subgraph_vertices = lambda ptr, idx, members, k=2: members
        for g in mats:
            bad = S.build_schedule(g.n, g.row_ptr, g.col, 64, k=3)
            lo, hi = _leaf_ranges(bad)
            try:
                C.check_dense_distance_k(g.n, g.row_ptr, g.col, bad.perm, lo, hi, bad.leaf_phase, 3)
            except AssertionError:
                caught += 1
    finally:
        S.subgraph_vertices = orig
    assert caught > 0
    for g in mats:
        sch = S.build_schedule(g.n, g.row_ptr, g.col, 64, k=3)
        lo, hi = _leaf_ranges(sch)
        C.check_dense_distance_k(g.n, g.row_ptr, g.col, sch.perm, lo, hi, sch.leaf_phase, 3)
