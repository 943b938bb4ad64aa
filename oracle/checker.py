"""Brute-force conflict checker for a SymmSpMV schedule -- test infrastructure only.

Shares no code with ``oracle.schedule``.  A schedule is given as data: the
permutation (new -> old), the tree of level groups (row ranges in the new
order, colors, parents) and the flattened phases of its leaves.

What SymmSpMV needs (Section 3.2 and the distance-k rule of Section 4.2):
two rows may be processed at the same time only if their *touch sets* are
disjoint, where the touch set of row r of the permuted upper triangle is
{r} together with every column stored in row r (the gather reads x there,
the scatter writes b there).  Disjoint touch sets for all pairs is the same
as distance-2 independence of the rows in the matrix graph.

Checks:
* every row belongs to exactly one leaf (the leaves tile [0, N));
* the children of every inner node tile the node's row range, alternate
  colors starting with the first color, and come in pairs;
* for every inner node and each color, the children of that color have
  pairwise disjoint touch sets (any two leaves that may run concurrently meet
  at such a node);
* for every flattened phase, the leaves of that phase have pairwise disjoint
  touch sets;
* for small N, the same with the dense pattern of (I + A)^2.
"""
from __future__ import annotations

import numpy as np


def permuted_upper_pattern(n, row_ptr, col, perm):
    """Rows/cols of the upper triangle of P A P^T (perm: new -> old)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    old2new = np.zeros(n, dtype=np.int64)
    old2new[np.asarray(perm, dtype=np.int64)] = np.arange(n, dtype=np.int64)
    r_old = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    a = old2new[r_old]
    b = old2new[col]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    order = np.argsort(lo, kind="stable")
    return lo[order], hi[order]


def _touch_counts(n, rows, cols, ranges):
    """How many of the given row ranges touch each index (rows sorted)."""
    count = np.zeros(n, dtype=np.int64)
    for lo, hi in ranges:
        if hi <= lo:
            continue
        a, b = np.searchsorted(rows, [lo, hi])
        touched = np.union1d(np.arange(lo, hi, dtype=np.int64), cols[a:b])
        count[touched] += 1
    return count


def _edge_conflicts(n, rows, cols, ranges):
    """Edges of the matrix graph whose two ends lie in two different ranges
    of the given list (distance-1 dependence between them)."""
    owner = np.full(n, -1, dtype=np.int64)
    for t, (lo, hi) in enumerate(ranges):
        owner[lo:hi] = t
    a, b = owner[rows], owner[cols]
    return int(np.count_nonzero((a >= 0) & (b >= 0) & (a != b)))


def check_schedule(n, row_ptr, col, perm, node_lo, node_hi, node_color, node_parent, leaf_ids, leaf_phase, dist=2):
    """Raise AssertionError on the first violated condition; return a summary.
    dist=2: concurrent row sets have disjoint touch sets (SymmSpMV);
    dist=1: no edge joins two concurrent row sets (Gauss-Seidel, Kaczmarz)."""
    perm = np.asarray(perm, dtype=np.int64)
    assert perm.shape == (n,) and np.array_equal(np.sort(perm), np.arange(n)), "perm is not a permutation"
    rows, cols = permuted_upper_pattern(n, row_ptr, col, perm)
    node_lo = np.asarray(node_lo)
    node_hi = np.asarray(node_hi)
    nnodes = node_lo.shape[0]
    children = [[] for _ in range(nnodes)]
    for i in range(nnodes):
        p = int(node_parent[i])
        if p >= 0:
            children[p].append(i)
    # leaves tile the rows
    leaf_ids = [int(i) for i in leaf_ids]
    cover = np.zeros(n, dtype=np.int64)
    for i in leaf_ids:
        assert not children[i], f"leaf {i} has children"
        cover[node_lo[i]:node_hi[i]] += 1
    assert np.all(cover == 1), "leaves do not tile the rows exactly once"
    # tree structure and same-color sibling independence
    for i in range(nnodes):
        ch = sorted(children[i], key=lambda c: (node_lo[c], c))
        if not ch:
            continue
        assert len(ch) % 2 == 0, f"node {i} has an odd number of children"
        assert node_lo[ch[0]] == node_lo[i] and node_hi[ch[-1]] == node_hi[i], f"children of {i} do not span it"
        for j, c in enumerate(ch):
            assert int(node_color[c]) == j % 2, f"child {c} of {i} has the wrong color"
            if j:
                assert node_lo[c] == node_hi[ch[j - 1]], f"children of {i} are not contiguous"
        for color in (0, 1):
            ranges = [(node_lo[c], node_hi[c]) for c in ch if int(node_color[c]) == color]
            if dist == 1:
                assert _edge_conflicts(n, rows, cols, ranges) == 0, f"same-color children of node {i} share an edge"
            else:
                cnt = _touch_counts(n, rows, cols, ranges)
                assert cnt.max(initial=0) <= 1, f"same-color children of node {i} conflict"
    # flattened phases
    phases = {}
    for i, ph in zip(leaf_ids, leaf_phase):
        phases.setdefault(int(ph), []).append(i)
    for ph, ids in phases.items():
        ranges = [(node_lo[i], node_hi[i]) for i in ids]
        if dist == 1:
            assert _edge_conflicts(n, rows, cols, ranges) == 0, f"leaves of phase {ph} share an edge"
        else:
            cnt = _touch_counts(n, rows, cols, ranges)
            assert cnt.max(initial=0) <= 1, f"leaves of phase {ph} conflict"
    return {"leaves": len(leaf_ids), "phases": len(phases)}


def check_dense_distance2(n, row_ptr, col, perm, leaf_lo, leaf_hi, leaf_phase):
    """Small N: rows of different leaves of one phase are at distance > 2 in
    the graph of A, i.e. (I + A)^2 has a zero there."""
    return check_dense_distance_k(n, row_ptr, col, perm, leaf_lo, leaf_hi, leaf_phase, 2)


def check_dense_distance_k(n, row_ptr, col, perm, leaf_lo, leaf_hi, leaf_phase, k):
    """Small N: rows of different leaves of one phase are at distance > k in
    the graph of A, i.e. (I + A)^k has a zero there (distance-k coloring,
    Section 4.2)."""
    assert n <= 2000
    rows, cols = permuted_upper_pattern(n, row_ptr, col, perm)
    # float64 products (exact for these 0/1 patterns) so BLAS does the work
    b = np.eye(n, dtype=np.float64)
    b[rows, cols] = 1.0
    b[cols, rows] = 1.0
    b2 = b.copy()
    for _ in range(k - 1):
        b2 = ((b2 @ b) > 0).astype(np.float64)
    b2 = b2 > 0
    owner = np.full(n, -1, dtype=np.int64)
    for t, (lo, hi) in enumerate(zip(leaf_lo, leaf_hi)):
        owner[lo:hi] = t
    phase_of_row = np.full(n, -1, dtype=np.int64)
    for t, (lo, hi) in enumerate(zip(leaf_lo, leaf_hi)):
        phase_of_row[lo:hi] = leaf_phase[t]
    i, j = np.nonzero(b2)
    bad = (owner[i] != owner[j]) & (phase_of_row[i] == phase_of_row[j])
    assert not np.any(bad), f"{int(bad.sum())} distance-{k} pairs share a phase across leaves"
    return True
