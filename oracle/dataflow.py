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


def makespan(compute, flush, deps, workers):
    """compute, flush: per-unit costs in ticket order; deps[u]: units (all
    < u) that must finish before u flushes.  Returns (makespan, finish)."""
    n = len(compute)
    finish = [0.0] * n
    free = [0.0] * max(1, int(workers))     # the time each worker becomes free
    heapq.heapify(free)
    for u in range(n):
        start = heapq.heappop(free)
        ready = start + compute[u]
        for d in deps[u]:
            assert d < u, "dependencies must point to earlier tickets"
            ready = max(ready, finish[d])
        finish[u] = ready + flush[u]
        heapq.heappush(free, finish[u])
    return (max(finish) if n else 0.0), finish
