"""Host checks of the diagonal ticket order of the matrix-power launch
(race_schedule_mpk_order): a permutation of all (power, position) tickets,
the static prefix kept in place, and every wait pointing to an earlier
ticket.  The waits are rederived here from the units' touch sets (own rows
and halo entries with their shared flags), not from the library's edge
lists: within a power, two units touching one index in any way other than
two shared touches keep their execution order; from power 1 on, a unit
follows, at the power before, every unit whose touch set meets its own."""
import numpy as np
import pytest

import matgen
import paper_1907_06487_amd as R

CASES = [
    ("2d5pt_40", lambda: matgen.stencil2d_5pt(40, seed=3), dict(n_workers=32, window_max=256, shared_atomics=False)),
    ("3d27pt_12_shared", lambda: matgen.stencil3d_27pt(12, seed=4),
     dict(n_workers=48, window_max=200, shared_atomics=True)),
    ("banded_3000_shared", lambda: matgen.banded_irregular(3000, seed=5, band=200),
     dict(n_workers=24, window_max=128, shared_atomics=True)),
]


def _touches(s, n):
    """(index, unit, shared) of every window touch."""
    u = s.units()
    idx, unit, shared = [], [], []
    for i, (lo, hi) in enumerate(zip(u["lo"], u["hi"])):
        rows = np.arange(lo, hi)
        idx.append(rows)
        unit.append(np.full(rows.size, i))
        shared.append((u["row_flags"][rows] & 2) != 0)
        h0, h1 = u["halo_ptr"][i], u["halo_ptr"][i + 1]
        idx.append(u["halo"][h0:h1])
        unit.append(np.full(h1 - h0, i))
        shared.append((u["halo_flags"][h0:h1] & 2) != 0)
    return np.concatenate(idx), np.concatenate(unit), np.concatenate(shared)


def _constraints(s, n, n_units):
    """Pairs (a, b): unit b after unit a within a power; and for each unit
    the units whose touch sets meet its own."""
    idx, unit, shared = _touches(s, n)
    order = np.argsort(idx, kind="stable")
    idx, unit, shared = idx[order], unit[order], shared[order]
    cuts = np.flatnonzero(np.diff(idx)) + 1
    within = set()
    meets = [set() for _ in range(n_units)]
    for g_unit, g_shared in zip(np.split(unit, cuts), np.split(shared, cuts)):
        for i in range(g_unit.size):
            meets[g_unit[i]].update(int(v) for v in g_unit)
            for j in range(g_unit.size):
                a, b = int(g_unit[i]), int(g_unit[j])
                if a < b and not (g_shared[i] and g_shared[j]):
                    within.add((a, b))
    return within, meets


@pytest.mark.parametrize("powers", [1, 3])
@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_mpk_diagonal_order_is_valid(name, make, kw, powers):
    m = make()
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, upload=False, **kw)
    try:
        st = s.stats()
        nu, nz = st["n_units"], st["n_zero_tasks"]
        per = nu + nz
        assert (kw["shared_atomics"] and st["n_zeroed"] > 0) or nz == 0 or kw["shared_atomics"]
        within, meets = _constraints(s, m.n, nu)
        assert s.ticket_order().tolist() == list(range(nu))  # default: execution order
        for lag in (0, m.n // 4, 10 * m.n):
            s.set_mpk_order(lag, False)
            for n_static in (0, min(per, 7), per):
                order = s.mpk_order(powers, n_static)
                assert sorted(order.tolist()) == list(range(powers * per)), (lag, n_static)
                assert order[:n_static].tolist() == list(range(n_static))
                tick = np.empty(powers * per, dtype=np.int64)
                tick[order] = np.arange(powers * per)
                at = lambda p, u: tick[p * per + nz + u]
                for p in range(powers):
                    for a, b in within:
                        assert at(p, a) < at(p, b), (lag, n_static, p, a, b)
                    if p > 0:
                        for u in range(nu):
                            for v in meets[u]:
                                assert at(p - 1, v) < at(p, u), (lag, n_static, p, u, v)
                if lag >= 10 * m.n and powers > 1:
                    pw = order // per
                    assert np.all(np.diff(pw) >= 0)  # a lag past every row: power by power
                if lag == 0 and powers > 1 and nu > 4:
                    pw = order // per
                    assert np.any(np.diff(pw) < 0)  # powers interleave
        s.set_mpk_order(-1, False)
        assert s.mpk_order(powers, 3).tolist() == list(range(powers * per))
    finally:
        s.close()


def test_mpk_order_arguments():
    m = matgen.stencil2d_5pt(12, seed=1)
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, upload=False, n_workers=4)
    try:
        with pytest.raises(R.RaceError):
            R._lib.race_schedule_set_mpk_order(s.handle, 10, 2)
        per = s.stats()["n_units"] + s.stats()["n_zero_tasks"]
        with pytest.raises(R.RaceError):
            s.mpk_order(0, 0)
        with pytest.raises(R.RaceError):
            s.mpk_order(2, per + 1)
    finally:
        s.close()
