"""GPU parity of dataflow products under other ticket orders.

Any topological order of the conflict edges gives the same y (within
rounding): the first-writer flags and edges are properties of the touch
sets and the phase order, not of the ticket numbering.  Checked against
the oracle for critical-path orders from random and measured unit costs,
a depth-first reversed order, with workgroups forced to join late (the
takeover path maps units back to tickets), and through the entry point
that allocates nothing."""
import numpy as np
import pytest

import matgen
import paper_1907_06487_amd as R
from oracle import symmspmv as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _full_row_len(m):
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    off = rows != m.col
    return int((np.bincount(rows, minlength=m.n) + np.bincount(m.col[off], minlength=m.n)).max(initial=0))


def _check(y, y_ref, absax, mlen, tag):
    u = 2.0 ** -53
    g = (mlen + 1) * u / (1 - (mlen + 1) * u)
    en, ec = O.errors(y, y_ref, absax)
    print(f"[{tag}] err_norm={en:.3e} err_comp={ec:.3e}", flush=True)
    assert en <= 1e-12 and ec <= 4 * g, tag


def _deps(s):
    """Conflict edges between units (clearing tasks left out) from the unit
    ranges and flags, as the schedule's touch sets define them."""
    u = s.units()
    last_plain, shared_since, deps = {}, {}, []
    for i in range(len(u["lo"])):
        idx = np.concatenate([np.arange(u["lo"][i], u["hi"][i]), u["halo"][u["halo_ptr"][i]:u["halo_ptr"][i + 1]]])
        fl = np.concatenate([u["row_flags"][u["lo"][i]:u["hi"][i]], u["halo_flags"][u["halo_ptr"][i]:u["halo_ptr"][i + 1]]])
        d = set()
        for g, f in zip(idx.tolist(), fl.tolist()):
            if g in last_plain:
                d.add(last_plain[g])
            if f & 2:
                shared_since.setdefault(g, set()).add(i)
            else:
                d |= shared_since.pop(g, set())
                last_plain[g] = i
        deps.append(sorted(d))
    return deps


def _depth_reversed(s):
    deps = _deps(s)
    depth = [0] * len(deps)
    for u in range(len(deps)):
        depth[u] = max([depth[d] + 1 for d in deps[u]], default=0)
    return np.asarray(sorted(range(len(deps)), key=lambda i: (depth[i], -i)), np.int32)


CASES = [
    ("3d27pt_24_w128", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=64, window_max=128)),
    ("banded_40k_w96", lambda: matgen.banded_irregular(40000, seed=6, band=4000), dict(n_workers=16, window_max=96)),
    ("3d27pt_24_w128_chain", lambda: matgen.stencil3d_27pt(24, seed=5),
     dict(n_workers=64, window_max=128, shared_atomics=False)),
    ("3d27pt_40_b512", lambda: matgen.stencil3d_27pt(40, seed=71), dict(n_workers=256, block_threads=512)),
]


@pytest.mark.parametrize("name,make,params", CASES, ids=[c[0] for c in CASES])
def test_products_under_other_ticket_orders(name, make, params):
    m = make()
    x = matgen.rhs(m.n, 31)
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, **params)
    try:
        nu = s.stats()["n_units"]
        y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x)[s.perm()]
        absax = O.abs_product(m.n, m.row_ptr, m.col, m.val, x)[s.perm()]
        xd = torch.as_tensor(x, device=DEV)
        xp = torch.empty_like(xd)
        s.permute(xd, xp, True)
        rng = np.random.default_rng(5)
        orders = {"random_costs": lambda: s.order_tickets(rng.uniform(0.1, 10, nu).astype(np.float32)),
                  "depth_reversed": lambda: s.set_ticket_order(_depth_reversed(s)),
                  "measured": lambda: s.tune_order(xp, torch.empty_like(xp), reps=2),
                  "default": lambda: s.order_tickets(None)}
        for tag, apply in orders.items():
            apply()
            print(f"case {name} order={tag}: n={m.n} units={nu}", flush=True)
            for late in (0, 3):
                s.test_late(late)
                yp = torch.full_like(xp, float("nan"))
                s.spmv(xp, yp)
                torch.cuda.synchronize()
                s.check()
                _check(yp.cpu().numpy(), y_ref, absax, _full_row_len(m), f"{name} {tag} late={late}")
            s.test_late(0)
            yp = torch.full_like(xp, float("nan"))
            s.spmv_noalloc(xp, yp)
            torch.cuda.synchronize()
            s.check()
            _check(yp.cpu().numpy(), y_ref, absax, _full_row_len(m), f"{name} {tag} noalloc")
    finally:
        s.close()
