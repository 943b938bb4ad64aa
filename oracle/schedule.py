"""RACE schedule oracle -- test infrastructure only.

Follows Section 4 of the paper in its own order:

1. Level construction (Section 4.1, Eq. (level), Algorithm "Construction of
   levels"): the level of a vertex is its BFS distance from the root.
2. Permutation by level; within a level the current order is kept
   (Sections 4.1-4.2).
3. Distance-k coloring by level aggregation (Section 4.2, Eq. (dk) and its
   corollary): level groups hold at least k adjacent levels and alternate
   two colors, so same-colored groups are distance-k independent.
4. Level-group construction with the epsilon criterion and worker counts
   (Section 4.4.3, steps 1-3).
5. Load balancing (Section 4.3, Algorithm "Load Balancing"), run with the
   worker counts of step 4 (Section 4.4.3, step 4).
6. Recursion on every group with more than one worker (Section 4.4): the
   subgraph is the group plus its distance-(k-1) neighbourhood, only the
   group's vertices keep their new levels, disconnected islands restart with
   the level number raised by two (Section 4.4.1), and the group is
   re-permuted by its new levels (Section 4.4.2).
7. The tree of level groups, its execution order (children first color,
   then second color) and the effective row count / parallel efficiency
   eta (Section 5).

Readings taken where the paper is silent or its text is garbled (the same
readings bind the GPU library):

* the stage-0 root is vertex 0 of the input order (``root="first"``); the
  BFS runs until the frontier is empty.  With ``root="peripheral"`` every
  stage-0 island starts instead from a pseudo-peripheral vertex found from
  that first vertex (the bandwidth-reduction root choice the paper's level
  construction refers to, Section 4.1; see ``pseudo_peripheral``);
* inside a stage-0 level the input order is kept (``level_order="input"``)
  or the Cuthill-McKee numbering is used (``level_order="cm"``, Section 4.1
  names RCM as the alternative level construction; only the numbering
  inside each level differs, the levels are the BFS levels either way, and
  the order is not reversed, since the colors need only the levels);
* disconnected input is handled as islands, exactly like the recursion's
  islands: the next root is the unvisited vertex of the group that comes
  first in the current order, and it gets the largest level assigned so far
  plus two;
* the subgraph of a group T is the subgraph induced by T and N(T) (k = 2);
  its root is the vertex of T that comes first in the current order;
* the load metric ``m`` of a row is 1 (balance by rows) or the number of
  stored entries of that row in the full symmetric matrix (balance by
  nonzeros); a group's load is the sum over its rows;
* level weight w(L) = (m(L) * n_t(parent)) / m(parent), in that order, in
  double; a = left-to-right running sum of weights; [a] = floor(a + 0.5);
  b = max(1, [a]); epsilon = 1 - |a - b|; a run qualifies when it holds at
  least 2k levels and epsilon > eps_s (strict);
* after a run qualifies, b is fixed and further levels are added while the
  new sum a' stays <= b and epsilon strictly increases;
* trailing levels that never qualify form a last pair when they are at least
  2k levels (b = max(1, [a])), else they join the previous pair; a node is
  refined only when at least two pairs form (and the total load is nonzero);
* a pair of n levels starts as red = first ceil(n/2) levels, blue = the rest;
  the two groups of a pair share their workers, so they are balanced against
  each other: while the heavier one has more than k levels and giving its
  boundary level to the lighter one strictly lowers |load(red) - load(blue)|,
  the level moves (this reproduces the worked 16 x 16 example: T_0(0) holds
  15 rows, T_0(4) is vertices 66..90 and N_eff(root) = 44);
* the optional global pass (``global_lb``) is Algorithm "Load Balancing" over
  all children of a refined node with their worker counts:
  per-group load per worker, per-color mean over the groups of that color,
  diff = load/worker - mean of its color, var = sum(diff^2)/len (all sums
  left to right); groups are ranked by stable argsort of -|diff| and of
  diff; the group g of the current rank takes one level from the first group
  in descending-diff order that has more than k levels when diff[g] < 0,
  otherwise (if g itself has more than k levels) gives one level to the
  lowest-diff group; a move shifts every group boundary between donor and
  receiver by one level; it is kept iff the variance strictly drops; the
  balancing ends when no rank yields a drop.  It is off by default because
  with it the worked example ends at N_eff(root) = 42, not the printed 44;
* recursion stops at ``max_stages`` stages;
* a leaf's phase is the bit string of colors on its root path (stage 0
  first), padded with zeros to the deepest stage, read as a binary number;
* N_eff(leaf) = its rows; N_eff(inner) = max over its first-color children
  + max over its second-color children; eta = N / (N_eff(root) * n_t).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DEFAULT_EPS = (0.8, 0.8, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5)


@dataclass
class Node:
    stage: int
    color: int
    lo: int
    hi: int
    b: int
    parent: int
    children: list = field(default_factory=list)
    n_levels: int = 0          # levels found when this node was refined (0 for leaves)


@dataclass
class Schedule:
    n: int
    perm: np.ndarray             # new -> old, int64
    nodes: list                  # preorder; nodes[0] is the root (stage -1)
    leaves: np.ndarray           # node ids of leaves, sorted by (phase, lo)
    leaf_phase: np.ndarray
    n_phases: int
    n_eff_root: int
    eta: float
    stage0_levels: int


# ---------------------------------------------------------------------------
# graph helpers

def full_adjacency(n, row_ptr, col):
    """Neighbour lists of the undirected graph of the symmetric matrix
    (off-diagonal pattern of U + U^T), CSR with ascending neighbours."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    off = rows != col
    r, c = rows[off], col[off]
    src = np.concatenate([r, c])
    dst = np.concatenate([c, r])
    order = np.argsort(src * n + dst, kind="stable")
    src, dst = src[order], dst[order]
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=ptr[1:])
    return ptr, dst


def row_loads(n, row_ptr, col, balance):
    """m(row): 1 per row, or the stored entries of the row in the full matrix."""
    if balance == "rows":
        return np.ones(n, dtype=np.int64)
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    upper = np.diff(row_ptr)
    rows = np.repeat(np.arange(n, dtype=np.int64), upper)
    off = rows != col
    lower = np.bincount(col[off], minlength=n)
    return upper + lower


def _neighbors(ptr, idx, frontier):
    starts = ptr[frontier]
    lens = ptr[frontier + 1] - starts
    total = int(lens.sum())
    if total == 0:
        return np.empty(0, dtype=np.int64)
    base = np.repeat(starts - (np.cumsum(lens) - lens), lens)
    return idx[base + np.arange(total, dtype=np.int64)]


def subgraph_vertices(ptr, idx, members, k=2):
    """Vertices of the recursion subgraph of a group T: T and every vertex
    within distance k - 1 of it, so no vertex outside can link two of T's
    vertices at distance k (Section 4.4.2; for k = 2 the distance-1
    neighbourhood N(T))."""
    seen = np.unique(np.asarray(members, dtype=np.int64))
    frontier = seen
    for _ in range(k - 1):
        nb = np.unique(_neighbors(ptr, idx, frontier))
        frontier = np.setdiff1d(nb, seen, assume_unique=True)
        seen = np.union1d(seen, frontier)
    return seen


def level_structure(ptr, idx, root, n):
    """Rooted level structure of the connected component of ``root`` in the
    full graph: BFS distances (-1 outside the component) and the last
    level's vertices in ascending order (Section 4.1, Eq. (level))."""
    dist = np.full(n, -1, dtype=np.int64)
    dist[root] = 0
    frontier = np.array([root], dtype=np.int64)
    last = frontier
    d = 0
    while frontier.size:
        last = frontier
        nb = _neighbors(ptr, idx, frontier)
        nb = np.unique(nb[dist[nb] < 0])
        d += 1
        dist[nb] = d
        frontier = nb
    return dist, np.sort(last)


def pseudo_peripheral(ptr, idx, start, n):
    """Pseudo-peripheral vertex of the component of ``start`` by the node
    finder of George and Liu (1979): from the current vertex r build the
    rooted level structure, take a vertex x of minimum degree in its last
    level (the lowest index among equals), build the structure rooted at x;
    while x reaches farther than r (larger eccentricity), continue from x.
    Returns the last x.  Degrees count off-diagonal neighbours."""
    deg = np.diff(ptr)
    r = int(start)
    dist, last = level_structure(ptr, idx, r, n)
    ecc_r = int(dist.max())
    while True:
        x = int(last[np.argmin(deg[last])])   # argmin returns the first (lowest index) minimum
        dist_x, last_x = level_structure(ptr, idx, x, n)
        ecc_x = int(dist_x.max())
        if ecc_x <= ecc_r:
            return x
        r, ecc_r, last = x, ecc_x, last_x


def cuthill_mckee_levels(ptr, idx, n, root_of=None):
    """Stage-0 levels with the Cuthill-McKee numbering (Cuthill and McKee,
    1969): from each island's root, the vertices are numbered level by
    level, and every numbered vertex numbers its unnumbered neighbours in
    order of increasing degree (ties: lower index first).  Islands start at
    their first unnumbered vertex (or ``root_of`` of it), each two levels
    above the largest so far.  Returns (levels, numbering order).  Plain
    loops: for test-sized graphs."""
    deg = np.diff(ptr)
    lev = np.full(n, -1, dtype=np.int64)
    order = []
    cur_max = -1
    for first in range(n):
        if lev[first] >= 0:
            continue
        root = first if root_of is None else root_of(first)
        lvl = 0 if cur_max < 0 else cur_max + 2
        lev[root] = lvl
        order.append(root)
        frontier = [root]
        while frontier:
            cur_max = max(cur_max, lvl)
            nxt = []
            for v in frontier:
                new = [int(u) for u in idx[ptr[v]:ptr[v + 1]] if lev[u] < 0]
                for u in new:
                    lev[u] = lvl + 1
                new.sort(key=lambda u: (deg[u], u))
                nxt.extend(new)
            order.extend(nxt)
            lvl += 1
            frontier = nxt
    return lev, np.array(order, dtype=np.int64)


def bfs_levels(ptr, idx, members, in_sub, scratch, root_of=None):
    """Levels (BFS distances) inside the subgraph induced by ``in_sub``.

    ``members`` are the group's vertices in current order; roots are taken
    from them (first unvisited, or ``root_of`` of it when given), each new
    island starting two above the largest level assigned so far.  Returns
    the levels of ``members``.  ``scratch`` is an all -1 array of length n,
    restored before returning."""
    touched = []
    cur_max = -1
    p = 0
    nm = members.shape[0]
    while True:
        # first member not yet visited
        while p < nm:
            chunk = members[p:p + 4096]
            unv = np.flatnonzero(scratch[chunk] < 0)
            if unv.size:
                p += int(unv[0])
                break
            p += chunk.shape[0]
        if p >= nm:
            break
        root = members[p] if root_of is None else root_of(int(members[p]))
        lvl = 0 if cur_max < 0 else cur_max + 2
        scratch[root] = lvl
        frontier = np.array([root], dtype=np.int64)
        touched.append(frontier)
        while frontier.size:
            cur_max = max(cur_max, lvl)
            nb = _neighbors(ptr, idx, frontier)
            nb = nb[in_sub[nb]]
            nb = nb[scratch[nb] < 0]
            nb = np.unique(nb)
            lvl += 1
            scratch[nb] = lvl
            touched.append(nb)
            frontier = nb
    out = scratch[members].copy()
    for t in touched:
        scratch[t] = -1
    return out


# ---------------------------------------------------------------------------
# Section 4.4.3 steps 1-3: epsilon aggregation into pairs of level groups

def aggregate_pairs(m_levels, n_t, eps_s, k):
    """Return [start_level, end_level, b] pairs, or [] when fewer than two can
    form.  ``m_levels`` are integer loads per level."""
    nl = len(m_levels)
    m_total = 0
    for m in m_levels:
        m_total += int(m)
    if m_total == 0:
        return []
    mt = float(m_total)
    w = [(float(int(m)) * float(n_t)) / mt for m in m_levels]
    pairs = []
    start = 0
    while start < nl:
        a = 0.0
        i = start
        b = 0
        qualified = False
        while i < nl:
            a += w[i]
            i += 1
            if i - start >= 2 * k:
                b = max(1, math.floor(a + 0.5))
                eps = 1.0 - abs(a - b)
                if eps > eps_s:
                    qualified = True
                    break
        if qualified:
            while i < nl:
                a2 = a + w[i]
                if a2 > b:
                    break
                if not (1.0 - abs(a2 - b)) > (1.0 - abs(a - b)):
                    break
                a = a2
                i += 1
            pairs.append([start, i, b])
            start = i
        else:
            if nl - start >= 2 * k:
                pairs.append([start, nl, max(1, math.floor(a + 0.5))])
            elif pairs:
                pairs[-1][1] = nl
            else:
                return []
            start = nl
    if len(pairs) < 2:
        return []
    return pairs


def split_pairs(pairs, m_levels, k):
    """Split every pair into its red and blue group and balance the two
    (Section 4.4.3 step 4, the groups of a pair are served by the same
    workers): start with red = first ceil(n/2) levels; while the heavier
    group has more than k levels and handing its boundary level to the
    lighter group strictly lowers |load(red) - load(blue)|, do so."""
    t_ptr = [pairs[0][0]]
    worker = []
    for s, e, b in pairs:
        r = s + (e - s + 1) // 2
        red = 0
        for lv in range(s, r):
            red += int(m_levels[lv])
        blue = 0
        for lv in range(r, e):
            blue += int(m_levels[lv])
        while True:
            if red > blue and r - s > k:
                x = int(m_levels[r - 1])
                if abs((red - x) - (blue + x)) < abs(red - blue):
                    red -= x
                    blue += x
                    r -= 1
                    continue
            elif blue > red and e - r > k:
                x = int(m_levels[r])
                if abs((red + x) - (blue - x)) < abs(red - blue):
                    red += x
                    blue -= x
                    r += 1
                    continue
            break
        t_ptr.append(r)
        t_ptr.append(e)
        worker += [b, b]
    return t_ptr, worker


# ---------------------------------------------------------------------------
# Section 4.3, Algorithm "Load Balancing" (with worker counts, Section 4.4.3)

def _variance(t_ptr, worker, prefix):
    ng = len(worker)
    per = []
    for i in range(ng):
        load = int(prefix[t_ptr[i + 1]] - prefix[t_ptr[i]])
        per.append(float(load) / float(worker[i]))
    s_r = 0.0
    n_r = 0
    s_b = 0.0
    n_b = 0
    for i in range(ng):
        if i % 2 == 0:
            s_r += per[i]
            n_r += 1
        else:
            s_b += per[i]
            n_b += 1
    mean_r = s_r / n_r
    mean_b = s_b / n_b
    diff = [per[i] - (mean_r if i % 2 == 0 else mean_b) for i in range(ng)]
    var = 0.0
    for d in diff:
        var += d * d
    var = var / ng
    return diff, var


def _stable_argsort(keys):
    return sorted(range(len(keys)), key=lambda i: keys[i])


def _shift(t_ptr, donor, receiver):
    t = list(t_ptr)
    if receiver < donor:
        for j in range(receiver + 1, donor + 1):
            t[j] += 1
    else:
        for j in range(donor + 1, receiver + 1):
            t[j] -= 1
    return t


def load_balance(t_ptr, worker, m_levels, k):
    prefix = [0]
    for m in m_levels:
        prefix.append(prefix[-1] + int(m))
    t_ptr = list(t_ptr)
    ng = len(worker)
    while True:
        diff, var = _variance(t_ptr, worker, prefix)
        abs_rank = _stable_argsort([-abs(d) for d in diff])
        rank = _stable_argsort(diff)
        improved = False
        for cr in range(ng):
            g = abs_rank[cr]
            donor = receiver = -1
            if diff[g] < 0:
                for el in reversed(rank):
                    if t_ptr[el + 1] - t_ptr[el] > k:
                        donor = el
                        break
                receiver = g
            elif t_ptr[g + 1] - t_ptr[g] > k:
                donor = g
                receiver = rank[0]
            if donor < 0 or donor == receiver:
                continue
            cand = _shift(t_ptr, donor, receiver)
            _, new_var = _variance(cand, worker, prefix)
            if new_var < var:
                t_ptr = cand
                improved = True
                break
        if not improved:
            return t_ptr


# ---------------------------------------------------------------------------
# the recursive construction (Section 4.4)

def build_schedule(n, row_ptr, col, n_t, eps=DEFAULT_EPS, k=2, balance="nnz", max_stages=4,
                   global_lb=False, root="first", level_order="input"):
    if not 1 <= k <= 8:
        raise ValueError("k must be in 1..8 (SymmSpMV needs k >= 2)")
    if root not in ("first", "peripheral"):
        raise ValueError("root must be 'first' or 'peripheral'")
    if level_order not in ("input", "cm"):
        raise ValueError("level_order must be 'input' or 'cm'")
    ptr, idx = full_adjacency(n, row_ptr, col)
    m_row = row_loads(n, row_ptr, col, balance)
    perm = np.arange(n, dtype=np.int64)
    scratch = np.full(n, -1, dtype=np.int64)
    in_sub = np.zeros(n, dtype=bool)
    nodes = [Node(stage=-1, color=0, lo=0, hi=n, b=int(n_t), parent=-1)]
    stage0_levels = [0]

    def eps_for(stage):
        return eps[stage] if stage < len(eps) else eps[-1]

    def refine(nid):
        node = nodes[nid]
        lo, hi = node.lo, node.hi
        if hi - lo == 0:
            return
        members = perm[lo:hi].copy()
        sub = None if node.stage < 0 else subgraph_vertices(ptr, idx, members, k)
        if sub is None:
            in_sub[:] = True
        else:
            in_sub[sub] = True
        root_of = None
        if node.stage < 0 and root == "peripheral":
            root_of = lambda v: pseudo_peripheral(ptr, idx, v, n)
        if node.stage < 0 and level_order == "cm":
            # stage 0 numbered by Cuthill-McKee: the members take that order
            lev_all, members = cuthill_mckee_levels(ptr, idx, n, root_of)
            lev = lev_all[members]
        else:
            lev = bfs_levels(ptr, idx, members, in_sub, scratch, root_of)
        if sub is None:
            in_sub[:] = False
        else:
            in_sub[sub] = False
        nl = int(lev.max()) + 1
        m_levels = np.bincount(lev, weights=m_row[members].astype(np.float64), minlength=nl).astype(np.int64)
        if node.stage < 0:
            stage0_levels[0] = nl
        pairs = aggregate_pairs(m_levels, node.b, eps_for(node.stage + 1), k)
        if not pairs:
            return
        order = np.argsort(lev, kind="stable")
        perm[lo:hi] = members[order]
        counts = np.bincount(lev, minlength=nl)
        level_ptr = np.zeros(nl + 1, dtype=np.int64)
        np.cumsum(counts, out=level_ptr[1:])
        level_ptr += lo
        t_ptr, worker = split_pairs(pairs, m_levels, k)
        if global_lb:
            t_ptr = load_balance(t_ptr, worker, m_levels, k)
        node.n_levels = nl
        for g in range(len(worker)):
            child = Node(stage=node.stage + 1, color=g % 2, lo=int(level_ptr[t_ptr[g]]),
                         hi=int(level_ptr[t_ptr[g + 1]]), b=int(worker[g]), parent=nid)
            nodes.append(child)
            node.children.append(len(nodes) - 1)
        for cid in list(node.children):
            c = nodes[cid]
            if c.b > 1 and c.stage + 1 < max_stages:
                refine(cid)

    refine(0)
    return _finish(n, perm, nodes, int(n_t), stage0_levels[0])


def _finish(n, perm, nodes, n_t, stage0_levels):
    # preorder renumbering (children in order), so the numbering does not
    # depend on the order the refinements ran in
    order = []

    def visit(i):
        order.append(i)
        for c in nodes[i].children:
            visit(c)

    visit(0)
    remap = {old: new for new, old in enumerate(order)}
    pre = []
    for old in order:
        nd = nodes[old]
        pre.append(Node(stage=nd.stage, color=nd.color, lo=nd.lo, hi=nd.hi, b=nd.b,
                        parent=remap[nd.parent] if nd.parent >= 0 else -1,
                        children=[remap[c] for c in nd.children], n_levels=nd.n_levels))
    nodes = pre
    leaves = [i for i, nd in enumerate(nodes) if not nd.children]
    depth = max(nodes[i].stage for i in leaves)
    phases = []
    for i in leaves:
        bits = []
        j = i
        while nodes[j].parent >= 0:
            bits.append(nodes[j].color)
            j = nodes[j].parent
        bits.reverse()  # stage 0 first
        ph = 0
        for s in range(depth + 1):
            ph = ph * 2 + (bits[s] if s < len(bits) else 0)
        phases.append(ph)
    n_phases = 1 << (depth + 1) if depth >= 0 else 1
    srt = sorted(range(len(leaves)), key=lambda t: (phases[t], nodes[leaves[t]].lo, leaves[t]))
    leaves_sorted = np.array([leaves[t] for t in srt], dtype=np.int64)
    phase_sorted = np.array([phases[t] for t in srt], dtype=np.int64)

    def n_eff(i):
        nd = nodes[i]
        if not nd.children:
            return nd.hi - nd.lo
        r = max(n_eff(c) for c in nd.children if nodes[c].color == 0)
        bl = max(n_eff(c) for c in nd.children if nodes[c].color == 1)
        return r + bl

    ne = n_eff(0)
    eta = float(n) / (float(ne) * float(n_t)) if ne > 0 else 1.0
    return Schedule(n=n, perm=perm, nodes=nodes, leaves=leaves_sorted, leaf_phase=phase_sorted,
                    n_phases=n_phases, n_eff_root=ne, eta=eta, stage0_levels=stage0_levels)


def permute_upper(n, row_ptr, col, val, perm):
    """Upper triangle of P A P^T (perm: new -> old), columns ascending."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n, dtype=np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    a, b = inv[rows], inv[col]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    order = np.argsort(lo * n + hi, kind="stable")
    lo, hi = lo[order], hi[order]
    v = np.asarray(val)[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(lo, minlength=n), out=rp[1:])
    return rp.astype(np.int32), hi.astype(np.int32), v
