"""Host side of the learned cost model through the C ABI (no GPU): network
inference against the float64 oracle, unit features and predicted makespan
against independent derivations, and schedules built with learned loads."""
import numpy as np
import pytest

import matgen
import paper_1907_06487_amd as R
from paper_1907_06487_amd import _lib
from oracle import checker as C
from oracle import dataflow as D
from oracle import mlp as M
from oracle import schedule as S

U32 = 2.0 ** -24


def _theta(seed, scale=0.3):
    return (M.init_params(seed) + scale * np.random.default_rng(seed).normal(size=M.N_PARAMS)).astype(np.float32)


def _abs_net(theta, X):
    """Forward pass with every weight, bias and input replaced by its
    magnitude and no ReLU: bounds the magnitude of every partial sum."""
    p = M.unpack(np.abs(theta.astype(np.float64)))
    h1 = np.abs(X) @ p["W1"].T + p["b1"]
    h2 = h1 @ p["W2"].T + p["b2"]
    return h2 @ p["w3"] + p["b3"][0]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_forward_host_matches_oracle(seed):
    theta = _theta(seed)
    X = np.random.default_rng(seed + 10).normal(size=(500, 12)).astype(np.float32)
    y = R._lib.race_mlp_forward_host(theta, X)
    ref = M.forward(theta.astype(np.float64), X.astype(np.float64))
    # float32 arithmetic: each of the three dot products (length <= 65)
    # contributes at most about 65 u of the magnitudes it sums
    bound = 3 * 66 * U32 * _abs_net(theta, X.astype(np.float64))
    assert np.all(np.abs(y - ref) <= bound)


def test_forward_host_empty_and_errors():
    assert R._lib.race_mlp_forward_host(_theta(0), np.zeros((0, 12), np.float32)).size == 0


CASES = [
    ("3d27pt_16", lambda: matgen.stencil3d_27pt(16, seed=3), dict(n_workers=64, window_max=256)),
    ("banded_8k", lambda: matgen.banded_irregular(8000, seed=4, band=800), dict(n_workers=32, window_max=200)),
    ("2d5pt_60", lambda: matgen.stencil2d_5pt(60, seed=5), dict(n_workers=16, window_max=300, shared_atomics=False)),
    ("rand_islands", lambda: matgen.random_symmetric(400, 0.004, seed=6), dict(n_workers=8, window_max=64)),
]


def _units_touches(u):
    out = []
    for i in range(len(u["lo"])):
        idx = np.concatenate([np.arange(u["lo"][i], u["hi"][i]), u["halo"][u["halo_ptr"][i]:u["halo_ptr"][i + 1]]])
        fl = np.concatenate([u["row_flags"][u["lo"][i]:u["hi"][i]], u["halo_flags"][u["halo_ptr"][i]:u["halo_ptr"][i + 1]]])
        out.append((idx, fl))
    return out


@pytest.mark.parametrize("k", [1, 4])
@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_unit_features_independent(name, make, kw, k):
    m = make()
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, upload=False, **kw)
    try:
        f = s.features(k)
        u = s.units()
        _, leaf_phase = s.leaves()
        st = s.stats()
        rp, cols, _ = S.permute_upper(m.n, m.row_ptr, m.col, m.val, s.perm())
        phase = leaf_phase[u["unit_leaf"]]
        per_phase = np.bincount(phase, minlength=st["n_phases"])
        touches = _units_touches(u)
        want = np.zeros_like(f, dtype=np.float64)
        for i in range(len(u["lo"])):
            a, b = int(u["lo"][i]), int(u["hi"][i])
            offd, out = [], 0
            for r in range(a, b):
                c = cols[rp[r]:rp[r + 1]]
                c = c[c != r]
                offd.append(c.size)
                out += int((c >= b).sum())
            offd = np.array(offd, dtype=np.float64)
            H = int(u["halo_ptr"][i + 1] - u["halo_ptr"][i])
            idx, fl = touches[i]
            W = idx.size
            mean = offd.mean()
            want[i] = [np.log2(1 + (b - a)), np.log2(1 + rp[b] - rp[a]), mean, offd.max(),
                       offd.std() / mean if mean > 0 else 0.0, H / (b - a), out / offd.sum() if offd.sum() else 0.0,
                       np.sum(fl == 0) / W, np.sum((fl & 2) != 0) / W, np.log2(1 + per_phase[phase[i]]),
                       phase[i] / st["n_phases"], np.log2(k)]
        assert np.allclose(f, want, rtol=2e-6, atol=2e-6)
    finally:
        s.close()


ZERO_CHUNK = 4096  # entries of the zero list one clearing task clears


def independent_deps(u, zero=None):
    """Conflict edges from the flags alone: a plain touch of index g waits
    for the last plain toucher of g and every shared toucher since; a shared
    touch waits for the last plain toucher only.  With the zero list given,
    a shared touch of a cleared entry also waits for the clearing task of
    that entry's chunk (returned separately as task numbers)."""
    chunk = {}
    if zero is not None:
        chunk = {int(g): i // ZERO_CHUNK for i, g in enumerate(zero)}
    last_plain = {}
    shared_since = {}
    deps, tasks = [], []
    for i, (idx, fl) in enumerate(_units_touches(u)):
        d, tk = set(), set()
        for g, f in zip(idx.tolist(), fl.tolist()):
            if g in last_plain:
                d.add(last_plain[g])
            if f & 2:
                if g in chunk:
                    tk.add(chunk[g])
                shared_since.setdefault(g, set()).add(i)
            else:
                d |= shared_since.pop(g, set())
                last_plain[g] = i
        deps.append(sorted(d))
        tasks.append(sorted(tk))
    return (deps, tasks) if zero is not None else deps


@pytest.mark.parametrize("workers", [1, 7, 64])
@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_simulate_matches_oracle(name, make, kw, workers):
    m = make()
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, upload=False, **kw)
    try:
        u = s.units()
        n_units = len(u["lo"])
        cost = np.random.default_rng(workers).uniform(0.5, 3.0, n_units).astype(np.float32)
        frac = 0.25
        got = s.simulate(cost, frac, workers)
        c64 = cost.astype(np.float64)
        want, _ = D.makespan(list((1 - frac) * c64), list(frac * c64), independent_deps(u), workers)
        assert got == pytest.approx(want, rel=1e-12)
        deps, tasks = independent_deps(u, s.zero_list())
        assert s.stats()["n_deps"] == sum(len(d) for d in deps) + sum(len(t) for t in tasks)
    finally:
        s.close()


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_critical_path_order_matches_oracle(name, make, kw):
    """The library's critical-path ticket order is the oracle's, bit for bit,
    on conflict edges derived independently from the flags; the predicted
    makespan under that order matches the oracle's simulation."""
    m = make()
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, upload=False, **kw)
    try:
        u = s.units()
        n_units = len(u["lo"])
        deps = independent_deps(u)
        assert list(s.ticket_order()) == list(range(n_units))
        for seed in range(3):
            cost = np.random.default_rng(seed).uniform(0.5, 3.0, n_units).astype(np.float32)
            if seed == 2:
                cost[:] = 1.0  # all ties: bottom levels are path lengths
            s.order_tickets(cost)
            got = list(s.ticket_order())
            want = D.critical_path_order([float(c) for c in cost], deps)
            assert got == want
            frac = 0.3
            c64 = cost.astype(np.float64)
            ms = s.simulate(cost, frac, 16)
            ref, _ = D.makespan(list((1 - frac) * c64), list(frac * c64), deps, 16, want)
            assert ms == pytest.approx(ref, rel=1e-12)
        s.order_tickets(None)
        assert list(s.ticket_order()) == list(range(n_units))
    finally:
        s.close()


def test_set_ticket_order_validation():
    m = matgen.stencil3d_27pt(16, seed=3)
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, upload=False, n_workers=64, window_max=256)
    try:
        u = s.units()
        n_units = len(u["lo"])
        deps = independent_deps(u)
        v = next(i for i in range(n_units) if deps[i])
        bad = list(range(n_units))
        d = deps[v][0]
        bad[d], bad[v] = bad[v], bad[d]  # v before a unit it waits for
        for order in (bad, list(range(n_units - 1)) + [0], [n_units] + list(range(1, n_units))):
            with pytest.raises(_lib.RaceError) as e:
                s.set_ticket_order(np.asarray(order, np.int32))
            assert e.value.code == -1
        assert list(s.ticket_order()) == list(range(n_units))  # a refused order changes nothing
        with pytest.raises(_lib.RaceError):
            s.order_tickets(np.full(n_units, np.nan, np.float32))
        # any topological order is accepted, e.g. dependency depth first, then descending unit
        depth = _depth(deps)
        rev = sorted(range(n_units), key=lambda i: (depth[i], -i))
        s.set_ticket_order(np.asarray(rev, np.int32))
        assert list(s.ticket_order()) == rev
    finally:
        s.close()


def _depth(deps):
    d = [0] * len(deps)
    for u in range(len(deps)):
        d[u] = max([d[x] + 1 for x in deps[u]], default=0)
    return d


def _constant_net(log_cost):
    theta = np.zeros(M.N_PARAMS, dtype=np.float32)
    theta[-1] = log_cost
    return theta


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_learned_loads_build_valid_schedules(name, make, kw):
    m = make()
    for theta in (_constant_net(np.log(3.0)), _theta(7, 0.05)):
        s = R.Schedule(m.n, m.row_ptr, m.col, m.val, upload=False, balance="model", cost_model=theta, **kw)
        try:
            tr = s.tree()
            node, phase = s.leaves()
            C.check_schedule(m.n, m.row_ptr, m.col, s.perm(), tr["lo"], tr["hi"], tr["color"], tr["parent"], node,
                             phase)
            assert 0 < s.stats()["eta"] <= 1
        finally:
            s.close()


def test_learned_loads_errors():
    m = matgen.stencil2d_5pt(10, seed=1)
    p = R.make_params(balance="model")
    with pytest.raises(_lib.RaceError) as e:
        R.race_build_schedule(m.n, m.row_ptr, m.col, m.val, p)
    assert e.value.code == -1
    p = R.make_params(balance="model", cost_model=np.zeros(100, np.float32))
    with pytest.raises(_lib.RaceError) as e:
        R.race_build_schedule(m.n, m.row_ptr, m.col, m.val, p)
    assert e.value.code == -1


def test_simulate_errors():
    m = matgen.stencil2d_5pt(10, seed=1)
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, upload=False, n_workers=4)
    cost = np.ones(s.stats()["n_units"], np.float32)
    for frac, w in ((1.5, 4), (0.2, 0)):
        with pytest.raises(_lib.RaceError):
            s.simulate(cost, frac, w)
    s.close()


def test_fold_normalisation_is_exact_reparametrisation():
    """The network trained on standardised inputs and the folded network on
    raw inputs give the same outputs (up to float32 rounding)."""
    torch = pytest.importorskip("torch")  # costmodel imports torch for device buffers
    from paper_1907_06487_amd import costmodel as CM
    rng = np.random.default_rng(40)
    X = rng.normal(3.0, 5.0, size=(300, 12)).astype(np.float64)
    mu, sd = X.mean(axis=0), X.std(axis=0)
    theta = _theta(41, 0.1)
    y_std = M.forward(theta.astype(np.float64), (X - mu) / sd)
    y_raw = M.forward(CM.fold_normalisation(theta, mu, sd).astype(np.float64), X)
    assert np.allclose(y_raw, y_std, rtol=1e-4, atol=1e-4 * np.abs(y_std).max())


def test_init_params_shape():
    pytest.importorskip("torch")
    from paper_1907_06487_amd import costmodel as CM
    th = CM.init_params(0)
    assert th.dtype == np.float32 and th.size == M.N_PARAMS and th[-1] == 0.0
