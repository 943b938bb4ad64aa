"""Dataflow makespan oracle -- test infrastructure only.

Predicted run time of a schedule whose units are handed out in a fixed
order (tickets) to `workers` identical workers: a free worker takes the next
unit; unit u computes for c[u] (needing nothing from other units), then
waits until every unit it depends on has finished, then flushes for f[u].
This is the critical-path view of Section 5 (the effective row count N_eff,
where a node costs the maximum over its first color plus the maximum over
its second) generalised to per-unit costs and conflict edges instead of
whole colors.

Written as a plain event loop over tickets; a unit's dependencies always
have smaller tickets, so they have started (and their finish times are
known) before the unit's flush is placed.
"""
from __future__ import annotations

import heapq


def makespan(compute, flush, deps, workers, order=None):
    """compute, flush: per-unit costs; deps[u]: units that must finish
    before u flushes.  Units are handed out in `order` (a list of units by
    ticket; default 0, 1, 2, ...), and every dependency must have an earlier
    ticket.  Returns (makespan, finish)."""
    n = len(compute)
    if order is None:
        order = list(range(n))
    ticket = {u: i for i, u in enumerate(order)}
    finish = [0.0] * n
    free = [0.0] * max(1, int(workers))     # the time each worker becomes free
    heapq.heapify(free)
    for u in order:
        start = heapq.heappop(free)
        ready = start + compute[u]
        for d in deps[u]:
            assert ticket[d] < ticket[u], "dependencies must point to earlier tickets"
            ready = max(ready, finish[d])
        finish[u] = ready + flush[u]
        heapq.heappush(free, finish[u])
    return (max(finish) if n else 0.0), finish


def bottom_levels(cost, deps):
    """Longest remaining path of every unit: its own cost plus the largest
    bottom level among the units that depend on it (the critical path of
    Section 5, node by node), float64 with cost[u] added to that maximum."""
    n = len(cost)
    succ = [[] for _ in range(n)]
    for u in range(n):
        for d in deps[u]:
            succ[d].append(u)
    memo = {}
    for root in range(n):
        # depth-first over the successors (an explicit stack, so long chains
        # need no deep recursion); a unit is finished once all its
        # successors are
        stack = [root]
        while stack:
            u = stack[-1]
            if u in memo:
                stack.pop()
                continue
            pending = [v for v in succ[u] if v not in memo]
            if pending:
                stack.extend(pending)
                continue
            best = 0.0
            for v in succ[u]:
                best = max(best, memo[v])
            memo[u] = float(cost[u]) + best
            stack.pop()
    return [memo[u] for u in range(n)]


def critical_path_order(cost, deps):
    """List-scheduling order by critical path: repeatedly emit, among the
    units whose dependencies have all been emitted, the one with the largest
    bottom level (ties: the lower unit index)."""
    n = len(cost)
    b = bottom_levels(cost, deps)
    emitted = [False] * n
    order = []
    while len(order) < n:
        best = None
        for u in range(n):
            if emitted[u] or not all(emitted[d] for d in deps[u]):
                continue
            if best is None or b[u] > b[best]:
                best = u
        assert best is not None, "dependencies form a cycle"
        emitted[best] = True
        order.append(best)
    return order
