"""Host checks of the dataflow plans of Gauss-Seidel and Kaczmarz sweeps
(race_schedule_gs_flow_plan).  The orderings are rederived from the matrix
and the leaves' row ranges alone: two leaves of different phases that hold
adjacent rows (a stored entry between them) must run in the serial sweep's
order -- forward: the leaf of the earlier phase first; backward: the leaf
of the later phase first; symmetric: every leaf's forward update before
its backward one.  The plan must make each such pair reachable through its
waits, every wait must point to an earlier ticket, every leaf must appear
once per direction, and the leaves of a ticket must share a phase.
A Kaczmarz ticket (one leaf) reads and writes its leaf's window, the rows
of the leaf and their neighbours: every two tickets whose windows share a
row must run in the serial sweep's order."""
import numpy as np
import pytest

import matgen
import paper_1907_06487_amd as R

CASES = [
    ("2d5pt_40", lambda: matgen.stencil2d_5pt(40, seed=3), dict(n_workers=32)),
    ("3d27pt_10", lambda: matgen.stencil3d_27pt(10, seed=4), dict(n_workers=64)),
    ("banded_2000", lambda: matgen.banded_irregular(2000, seed=5, band=100), dict(n_workers=64)),
    ("rand_islands", lambda: matgen.random_symmetric(300, 0.01, seed=8), dict(n_workers=16)),
]


def _leaf_info(s, n):
    tr = s.tree()
    node, phase = s.leaves()
    lo, hi = np.asarray(tr["lo"])[node], np.asarray(tr["hi"])[node]
    row_leaf = np.full(n, -1, dtype=np.int64)
    for i, (a, b) in enumerate(zip(lo, hi)):
        assert np.all(row_leaf[a:b] == -1)
        row_leaf[a:b] = i
    assert np.all(row_leaf >= 0)
    return phase, row_leaf


def _adjacent_pairs(m, perm, row_leaf):
    """Leaf pairs joined by a stored entry, in the permuted numbering."""
    inv = np.empty(m.n, dtype=np.int64)
    inv[perm] = np.arange(m.n)
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    a, b = row_leaf[inv[rows]], row_leaf[inv[m.col]]
    keep = a != b
    return set(zip(a[keep].tolist(), b[keep].tolist())) | set(zip(b[keep].tolist(), a[keep].tolist()))


def _reach(n, ptr, idx):
    """For every ticket, the set of tickets it waits for directly or through others."""
    reach = []
    for t in range(n):
        r = set()
        for d in idx[ptr[t]:ptr[t + 1]]:
            r.add(int(d))
            r |= reach[int(d)]
        reach.append(r)
    return reach


@pytest.mark.parametrize("direction", [0, 1, 2])
@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_gs_flow_plan_orders_every_adjacent_pair(name, make, kw, direction):
    m = make()
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, upload=False, dist_k=1, **kw)
    try:
        phase, row_leaf = _leaf_info(s, m.n)
        pairs = _adjacent_pairs(m, s.perm(), row_leaf)
        plan = s.gs_flow_plan(direction)
        nt = plan["leaf0"].size
        ptr, idx = plan["dep_ptr"], plan["dep_idx"]
        for t in range(nt):
            assert np.all(idx[ptr[t]:ptr[t + 1]] < t)
        ticket = {}
        for t in range(nt):
            leaves = range(plan["leaf0"][t], plan["leaf0"][t] + plan["count"][t])
            assert 1 <= plan["count"][t] <= 4
            assert len({int(phase[l]) for l in leaves}) == 1
            for l in leaves:
                key = (int(plan["back"][t]), l)
                assert key not in ticket
                ticket[key] = t
        dirs = {0: [0], 1: [1], 2: [0, 1]}[direction]
        assert len(ticket) == len(dirs) * len(phase)
        reach = _reach(nt, ptr, idx)
        for a, b in pairs:  # a before b in the serial sweep
            if 0 in dirs and phase[a] < phase[b]:
                assert ticket[(0, a)] in reach[ticket[(0, b)]], ("forward", a, b)
            if 1 in dirs and phase[a] > phase[b]:
                assert ticket[(1, a)] in reach[ticket[(1, b)]], ("backward", a, b)
            assert phase[a] != phase[b]  # a distance-1 coloring
        if direction == 2:
            for l in range(len(phase)):
                assert ticket[(0, l)] in reach[ticket[(1, l)]]
    finally:
        s.close()


def test_gs_exec_arguments():
    g = matgen.config_2d_small()
    s = R.Schedule(g.n, g.row_ptr, g.col, g.val, upload=False, dist_k=1, n_workers=64)
    s2 = R.Schedule(g.n, g.row_ptr, g.col, g.val, upload=False, n_workers=64)
    try:
        s.set_gs_exec("flow")
        s.set_gs_exec("phases")
        with pytest.raises(R.RaceError):
            R._lib.race_schedule_set_gs_exec(s.handle, 2)
        with pytest.raises(R.RaceError):
            s2.set_gs_exec("flow")
        with pytest.raises(R.RaceError):
            s2.gs_flow_plan(0)
        s3 = R.Schedule(g.n, g.row_ptr, g.col, g.val, upload=False, n_workers=64, kaczmarz=True)
        s3.set_gs_exec("flow")
        assert s3.gs_flow_plan(2)["leaf0"].size == 2 * s3.stats()["n_leaves"]
        s3.close()
    finally:
        s.close()
        s2.close()


def _windows(m, perm, lo, hi):
    """Rows (permuted numbering) of every leaf's Kaczmarz window: its own
    rows and their neighbours in the full matrix."""
    inv = np.empty(m.n, dtype=np.int64)
    inv[perm] = np.arange(m.n)
    nb = [set() for _ in range(m.n)]
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    for r, c in zip(inv[rows].tolist(), inv[m.col].tolist()):
        nb[r].add(c)
        nb[c].add(r)
    out = []
    for a, b in zip(lo, hi):
        w = set(range(a, b))
        for r in range(a, b):
            w |= nb[r]
        out.append(w)
    return out


KACZ_CASES = CASES + [("3d27pt_10_dist3", lambda: matgen.stencil3d_27pt(10, seed=4), dict(n_workers=64, dist_k=3))]


@pytest.mark.parametrize("direction", [0, 1, 2])
@pytest.mark.parametrize("name,make,kw", KACZ_CASES, ids=[c[0] for c in KACZ_CASES])
def test_kacz_flow_plan_orders_every_shared_row(name, make, kw, direction):
    m = make()
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, upload=False, kaczmarz=True, **kw)
    try:
        tr = s.tree()
        node, phase = s.leaves()
        lo, hi = np.asarray(tr["lo"])[node], np.asarray(tr["hi"])[node]
        win = _windows(m, s.perm(), lo, hi)
        plan = s.gs_flow_plan(direction)
        nt = plan["leaf0"].size
        ptr, idx = plan["dep_ptr"], plan["dep_idx"]
        assert np.all(plan["count"] == 1)
        seen = set()
        for t in range(nt):
            assert np.all(idx[ptr[t]:ptr[t + 1]] < t)
            key = (int(plan["back"][t]), int(plan["leaf0"][t]))
            assert key not in seen
            seen.add(key)
        dirs = {0: [0], 1: [1], 2: [0, 1]}[direction]
        assert len(seen) == len(dirs) * len(phase)
        # the serial order: forward phases ascending, then backward descending
        ph = [int(phase[int(l)]) for l in plan["leaf0"]]
        bk = plan["back"].tolist()
        for t in range(1, nt):
            if bk[t] == bk[t - 1]:
                assert ph[t] >= ph[t - 1] if bk[t] == 0 else ph[t] <= ph[t - 1]
            else:
                assert bk[t - 1] == 0 and bk[t] == 1
        reach = _reach(nt, ptr, idx)
        holders = {}
        for t in range(nt):
            for r in win[int(plan["leaf0"][t])]:
                holders.setdefault(r, []).append(t)
        for r, ts in holders.items():
            for a, b in zip(ts, ts[1:]):
                assert a in reach[b], (r, a, b)
        # leaves of one phase share no window row
        for p in set(ph):
            ls = [l for l in range(len(phase)) if int(phase[l]) == p]
            allrows = [r for l in ls for r in win[l]]
            assert len(allrows) == len(set(allrows))
    finally:
        s.close()
