"""Pins of the cost-model oracles (network and dataflow makespan) against
facts fixed by calculus and by construction, independent of the oracles'
own formulas: central finite differences, closed forms in special weight
settings, the first Adam step, and schedules whose makespan is known."""
import numpy as np
import pytest

from oracle import dataflow as D
from oracle import mlp as M


def _data(seed, n=40):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, M.N_IN)), rng.normal(size=n)


def _fd_check(loss_and_grad, seed):
    theta = M.init_params(seed) + 0.05 * np.random.default_rng(seed + 1).normal(size=M.N_PARAMS)
    X, t = _data(seed)
    _, g = loss_and_grad(theta, X, t)
    # a subset of coordinates from every parameter block, plus the b3 end
    idx = np.unique(np.r_[np.arange(0, M.N_PARAMS, 37), np.arange(M.N_PARAMS - 70, M.N_PARAMS)])
    fd = np.empty(idx.size)
    for j, i in enumerate(idx):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += 1e-6
        tm[i] -= 1e-6
        fd[j] = (M.loss_and_grad(tp, X, t)[0] - M.loss_and_grad(tm, X, t)[0]) / 2e-6
    return np.max(np.abs(g[idx] - fd)) / max(np.max(np.abs(fd)), 1e-30)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    assert _fd_check(M.loss_and_grad, seed) <= 1e-6


def test_parameter_count_and_packing():
    assert M.N_PARAMS == 12 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 5057
    theta = np.arange(M.N_PARAMS, dtype=np.float64)
    assert np.array_equal(M.pack(M.unpack(theta)), theta)
    assert M.unpack(theta)["W1"][1, 0] == 12.0  # row-major, output by input


def test_constant_network_when_w2_is_zero():
    """W2 = 0 makes f = w3 . relu(b2) + b3 for every input: the input-side
    gradients vanish and dL/db3 = mean of 2 (f - t)."""
    p = M.unpack(M.init_params(3).copy())
    p = {k: v.copy() for k, v in p.items()}
    p["W2"][:] = 0.0
    p["b2"] = np.linspace(-1, 1, 64)
    theta = M.pack(p)
    X, t = _data(4)
    f_const = float(p["w3"] @ np.maximum(p["b2"], 0) + p["b3"][0])
    assert np.allclose(M.forward(theta, X), f_const, rtol=0, atol=1e-14)
    loss, g = M.loss_and_grad(theta, X, t)
    gp = M.unpack(g)
    assert np.all(gp["W1"] == 0) and np.all(gp["b1"] == 0)
    assert gp["b3"][0] == pytest.approx(np.mean(2 * (f_const - t)), rel=1e-13)
    assert loss == pytest.approx(np.mean((f_const - t) ** 2), rel=1e-13)


def test_linear_regime_is_the_composed_affine_map():
    """With every pre-activation positive the network is the affine map
    x -> w3^T W2 W1 x + (w3^T (W2 b1 + b2) + b3)."""
    rng = np.random.default_rng(5)
    p = {"W1": rng.uniform(0.1, 1, (64, 12)), "b1": rng.uniform(0.1, 1, 64), "W2": rng.uniform(0.1, 1, (64, 64)),
         "b2": rng.uniform(0.1, 1, 64), "w3": rng.normal(size=64), "b3": np.array([0.3])}
    X = rng.uniform(0, 1, (20, 12))
    a = p["w3"] @ p["W2"] @ p["W1"]
    c = p["w3"] @ (p["W2"] @ p["b1"] + p["b2"]) + p["b3"][0]
    assert np.allclose(M.forward(M.pack(p), X), X @ a + c, rtol=1e-13, atol=1e-12)


def test_perfect_fit_has_zero_loss_and_gradient():
    theta = M.init_params(6)
    X, _ = _data(7)
    t = M.forward(theta, X)
    loss, g = M.loss_and_grad(theta, X, t)
    assert loss == 0.0 and np.all(g == 0.0)


def test_first_adam_step_moves_by_lr_times_sign():
    """At step 1 the bias-corrected moments are g and g^2, so every
    parameter moves by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(8)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = M.adam_step(theta, g, np.zeros(50), np.zeros(50), 1, lr=0.01, eps=1e-8)
    assert np.allclose(new, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_minimises_a_quadratic():
    """Many Adam steps on L = |theta - c|^2 end near c."""
    c = np.array([1.5, -2.0, 0.25])
    theta, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for step in range(1, 3001):
        theta, m, v = M.adam_step(theta, 2 * (theta - c), m, v, step, lr=0.01)
    assert np.allclose(theta, c, atol=1e-3)


def _planted_transposed_w2(theta, X, t):
    """A plausible mistake: W2 instead of W2^T in the backward pass."""
    p = M.unpack(theta)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0)
    r = h2 @ p["w3"] + p["b3"][0] - t
    g = 2 * r / X.shape[0]
    dz2 = np.outer(g, p["w3"]) * (z2 > 0)
    dz1 = (dz2 @ p["W2"].T) * (z1 > 0)
    return float(np.mean(r * r)), M.pack({"W1": dz1.T @ X, "b1": dz1.sum(0), "W2": dz2.T @ h1, "b2": dz2.sum(0),
                                          "w3": h2.T @ g, "b3": np.array([g.sum()])})


def _planted_relu_mask_h2(theta, X, t):
    """A plausible mistake: the first layer's gradient masked by the second
    layer's activity pattern."""
    p = M.unpack(theta)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0)
    r = h2 @ p["w3"] + p["b3"][0] - t
    g = 2 * r / X.shape[0]
    dz2 = np.outer(g, p["w3"]) * (z2 > 0)
    dz1 = (dz2 @ p["W2"]) * (z2 > 0)
    return float(np.mean(r * r)), M.pack({"W1": dz1.T @ X, "b1": dz1.sum(0), "W2": dz2.T @ h1, "b2": dz2.sum(0),
                                          "w3": h2.T @ g, "b3": np.array([g.sum()])})


def _planted_missing_factor_two(theta, X, t):
    loss, g = M.loss_and_grad(theta, X, t)
    return loss, g / 2


@pytest.mark.parametrize("planted", [_planted_transposed_w2, _planted_relu_mask_h2, _planted_missing_factor_two])
def test_finite_differences_catch_planted_mistakes(planted):
    assert _fd_check(planted, 0) > 1e-3


# --- dataflow makespan ------------------------------------------------------

def test_makespan_single_worker_is_the_sum():
    c, f = [3.0, 1.0, 2.0], [0.5, 0.5, 1.0]
    assert D.makespan(c, f, [[], [], []], 1)[0] == pytest.approx(8.0)


def test_makespan_enough_workers_independent_is_the_max():
    c, f = [3.0, 1.0, 2.0], [0.5, 0.5, 4.0]
    assert D.makespan(c, f, [[], [], []], 8)[0] == pytest.approx(6.0)


def test_makespan_chain_serialises_flushes_only():
    """With enough workers a chain computes in parallel; flush u starts at
    max(own compute end, flush end of u-1)."""
    c = [2.0, 2.0, 2.0, 2.0]
    f = [1.0, 1.0, 1.0, 1.0]
    deps = [[], [0], [1], [2]]
    # finishes: 3, max(2, 3) + 1 = 4, 5, 6
    ms, fin = D.makespan(c, f, deps, 4)
    assert fin == [3.0, 4.0, 5.0, 6.0] and ms == 6.0


def _brute_force(c, f, deps, workers):
    """Tiny cases: simulate every worker explicitly step by step in time."""
    n = len(c)
    worker_free = [0.0] * workers
    finish = [None] * n
    for u in range(n):
        w = min(range(workers), key=lambda i: (worker_free[i], i))
        start = worker_free[w]
        flush_start = max([start + c[u]] + [finish[d] for d in deps[u]])
        finish[u] = flush_start + f[u]
        worker_free[w] = finish[u]
    return max(finish)


def test_makespan_matches_explicit_worker_simulation():
    rng = np.random.default_rng(11)
    for trial in range(200):
        n = int(rng.integers(1, 9))
        c = list(rng.uniform(0.1, 3, n))
        f = list(rng.uniform(0.1, 1, n))
        deps = [sorted(set(rng.integers(0, u, size=int(rng.integers(0, 3))).tolist())) if u else [] for u in range(n)]
        w = int(rng.integers(1, 4))
        assert D.makespan(c, f, deps, w)[0] == pytest.approx(_brute_force(c, f, deps, w))


def test_makespan_lower_bounds():
    """Never below total work / workers, nor below the longest dependency path."""
    rng = np.random.default_rng(12)
    for trial in range(50):
        n = 30
        c = rng.uniform(0.1, 3, n)
        f = rng.uniform(0.1, 1, n)
        deps = [sorted(set(rng.integers(0, u, size=2).tolist())) if u else [] for u in range(n)]
        w = int(rng.integers(1, 6))
        ms = D.makespan(list(c), list(f), deps, w)[0]
        assert ms >= (c + f).sum() / w - 1e-9
        longest = [0.0] * n
        for u in range(n):
            longest[u] = max([c[u]] + [longest[d] for d in deps[u]]) + f[u]
        assert ms >= max(longest) - 1e-9


# --- critical-path ticket order ---------------------------------------------

def _all_paths_longest(cost, deps):
    """Tiny DAGs: the longest path from every unit to a sink by enumerating
    every path explicitly (no memoisation, no shared maxima)."""
    n = len(cost)
    succ = [[v for v in range(n) if u in deps[v]] for u in range(n)]
    out = []
    for u in range(n):
        best = 0.0
        stack = [(u, cost[u])]
        while stack:
            w, acc = stack.pop()
            if not succ[w]:
                best = max(best, acc)
            for v in succ[w]:
                stack.append((v, acc + cost[v]))
        out.append(best)
    return out


def test_bottom_levels_equal_longest_paths_by_enumeration():
    rng = np.random.default_rng(21)
    for trial in range(100):
        n = int(rng.integers(1, 9))
        cost = [float(v) for v in rng.integers(1, 10, n)]  # integers: sums are exact in any order
        deps = [sorted(set(rng.integers(0, u, size=int(rng.integers(0, 3))).tolist())) if u else [] for u in range(n)]
        assert D.bottom_levels(cost, deps) == _all_paths_longest(cost, deps)


def test_critical_path_order_closed_forms():
    # independent units: descending cost, ties to the lower index
    assert D.critical_path_order([1.0, 5.0, 3.0, 5.0], [[], [], [], []]) == [1, 3, 2, 0]
    # a chain has one order
    assert D.critical_path_order([1.0, 1.0, 1.0], [[], [0], [1]]) == [0, 1, 2]
    # two roots: the one heading the longer chain goes first even though it is cheaper
    #   0 (cost 1) -> 2 (cost 10);  1 (cost 5) alone
    assert D.critical_path_order([1.0, 5.0, 10.0], [[], [], [0]]) == [0, 2, 1]
    # fork-join: 0 -> {1 (2), 2 (7)} -> 3; after 0, unit 2 precedes unit 1
    assert D.critical_path_order([1.0, 2.0, 7.0, 1.0], [[], [0], [0], [1, 2]]) == [0, 2, 1, 3]


def test_critical_path_order_is_topological_and_greedy():
    rng = np.random.default_rng(22)
    for trial in range(100):
        n = int(rng.integers(1, 30))
        cost = list(rng.uniform(0.1, 5, n))
        deps = [sorted(set(rng.integers(0, u, size=int(rng.integers(0, 3))).tolist())) if u else [] for u in range(n)]
        order = D.critical_path_order(cost, deps)
        assert sorted(order) == list(range(n))
        pos = {u: i for i, u in enumerate(order)}
        assert all(pos[d] < pos[u] for u in range(n) for d in deps[u])
        # every step took a ready unit of maximal bottom level
        b = D.bottom_levels(cost, deps)
        done = set()
        for u in order:
            ready = [v for v in range(n) if v not in done and all(d in done for d in deps[v])]
            assert b[u] == max(b[v] for v in ready)
            done.add(u)


def _priority_order(prio, deps):
    n = len(prio)
    done, order = set(), []
    while len(order) < n:
        ready = [v for v in range(n) if v not in done and all(d in done for d in deps[v])]
        u = max(ready, key=lambda v: (prio[v], -v))
        done.add(u)
        order.append(u)
    return order


def test_critical_path_order_planted_priorities_fail():
    """Plausible mistakes fail the closed forms above: priority by a unit's
    own cost, and bottom levels that forget the unit's own cost."""
    cost, deps = [1.0, 5.0, 10.0], [[], [], [0]]
    assert D.critical_path_order(cost, deps) == [0, 2, 1]
    assert _priority_order(cost, deps) == [1, 0, 2]
    cost, deps = [1.0, 2.0, 7.0, 1.0], [[], [0], [0], [1, 2]]
    no_own = [b - c for b, c in zip(D.bottom_levels(cost, deps), cost)]
    assert _priority_order(no_own, deps) == [0, 1, 2, 3] != D.critical_path_order(cost, deps)


def test_makespan_with_order_is_the_reordered_simulation():
    """Reordering is the same simulation over the renumbered units."""
    rng = np.random.default_rng(23)
    for trial in range(50):
        n = int(rng.integers(1, 12))
        c = list(rng.uniform(0.1, 3, n))
        f = list(rng.uniform(0.1, 1, n))
        deps = [sorted(set(rng.integers(0, u, size=int(rng.integers(0, 3))).tolist())) if u else [] for u in range(n)]
        order = D.critical_path_order(list(np.add(c, f)), deps)
        pos = {u: i for i, u in enumerate(order)}
        c2 = [c[u] for u in order]
        f2 = [f[u] for u in order]
        deps2 = [sorted(pos[d] for d in deps[u]) for u in order]
        w = int(rng.integers(1, 4))
        assert D.makespan(c, f, deps, w, order)[0] == pytest.approx(_brute_force(c2, f2, deps2, w))
