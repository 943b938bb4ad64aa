"""Pins for the oracle's load balancing and load metric (CPU only).

* Algorithm "Load Balancing" (Section 4.3) against two examples derived by
  hand step by step (tests/golden/load_balance_examples.json), the property
  Section 4.3 states for its 16 x 16 example with ten level groups, a
  brute-force exit check over the algorithm's moves, and strict variance
  drops on constructed imbalanced inputs.
* The literal global pass on the worked example of Section 4.4.3 is
  recorded next to the printed N_eff(root) = 44 that the pair balancing
  reproduces.
* The nonzero load metric (Section 4.3: balance by rows or by nonzeros)
  against dense row counts and stencil closed forms.
* Planted mistakes (identity balancing, the mean taken over the parent's
  thread count instead of the colour's groups, upper-triangle row counts)
  each fail one of these pins.
"""
import json
import os

import numpy as np
import pytest

import matgen
from oracle import schedule as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden():
    return json.load(open(os.path.join(GOLDEN, "load_balance_examples.json")))


def variance(t_ptr, worker, m_levels):
    prefix = np.concatenate([[0], np.cumsum(m_levels)])
    return S._variance(t_ptr, worker, prefix)


def algorithm_moves(t_ptr, worker, m_levels, k):
    """Every move the algorithm considers from t_ptr (one per rank), as
    candidate T_ptr arrays."""
    diff, _ = variance(t_ptr, worker, m_levels)
    ng = len(worker)
    rank = sorted(range(ng), key=lambda i: diff[i])
    out = []
    for g in range(ng):
        if diff[g] < 0:
            donor = next((el for el in reversed(rank) if t_ptr[el + 1] - t_ptr[el] > k), -1)
            receiver = g
        elif t_ptr[g + 1] - t_ptr[g] > k:
            donor, receiver = g, rank[0]
        else:
            continue
        if donor < 0 or donor == receiver:
            continue
        t = list(t_ptr)
        # one level crosses every boundary between donor and receiver
        for j in range(min(donor, receiver) + 1, max(donor, receiver) + 1):
            t[j] += 1 if receiver < donor else -1
        out.append(t)
    return out


# ---------------------------------------------------------------------------
# load balancing

def check_examples(lb):
    for ex in golden()["examples"]:
        out = lb(ex["t_ptr_in"], ex["worker"], ex["m_levels"], ex["k"])
        assert list(out) == ex["t_ptr_out"], ex["name"]


def test_load_balance_hand_derived_examples():
    check_examples(S.load_balance)
    for ex in golden()["examples"]:
        assert variance(ex["t_ptr_in"], ex["worker"], ex["m_levels"])[1] == ex["var_in"]
        assert variance(ex["t_ptr_out"], ex["worker"], ex["m_levels"])[1] == ex["var_out"]


def paper_property(lb):
    g = golden()["paper_property"]
    sizes = g["level_sizes"]
    nl, ng, k = len(sizes), g["groups"], g["k"]
    t0 = [(i * nl) // ng for i in range(ng + 1)]
    t = lb(t0, [1] * ng, sizes, k)
    nlev = [t[i + 1] - t[i] for i in range(ng)]
    # the middle groups keep two levels, the end groups take more
    assert nlev[ng // 2 - 1] == k and nlev[ng // 2] == k
    assert nlev[0] > k and nlev[-1] > k
    assert all(x >= k for x in nlev)
    return t


def test_load_balance_paper_property_16x16_ten_groups():
    paper_property(S.load_balance)


def test_load_balance_exit_no_move_lowers_variance():
    rng = np.random.default_rng(11)
    for _ in range(150):
        k = int(rng.integers(1, 4))
        ng = 2 * int(rng.integers(1, 5))
        nl = int(rng.integers(k * ng, k * ng + 12))
        ml = rng.integers(0, 40, size=nl)
        worker = [int(w) for w in rng.choice([1, 2, 4], size=ng)]
        t0 = [0]
        for i in range(ng - 1):
            t0.append(t0[-1] + k)
        t0.append(nl)
        t1 = S.load_balance(t0, worker, ml, k)
        _, var1 = variance(t1, worker, ml)
        for cand in algorithm_moves(t1, worker, ml, k):
            assert not variance(cand, worker, ml)[1] < var1


def test_load_balance_strictly_lowers_imbalanced_inputs():
    rng = np.random.default_rng(12)
    for _ in range(50):
        k = 2
        ng = 2 * int(rng.integers(2, 5))
        per = int(rng.integers(3, 6))
        nl = ng * per
        # heavy levels gathered at one end: equal level counts are far from balanced
        ml = np.concatenate([np.ones(nl // 2, dtype=np.int64), rng.integers(20, 40, size=nl - nl // 2)])
        t0 = [i * per for i in range(ng + 1)]
        worker = [1] * ng
        _, var0 = variance(t0, worker, ml)
        t1 = S.load_balance(t0, worker, ml, k)
        _, var1 = variance(t1, worker, ml)
        assert var1 < var0
        assert t1[0] == 0 and t1[-1] == nl
        assert all(t1[i + 1] - t1[i] >= k for i in range(ng))


def test_literal_global_pass_on_worked_example():
    g = golden()["literal_global_pass_on_worked_example"]
    w = json.load(open(os.path.join(GOLDEN, "worked_example_16x16.json")))
    m = matgen.stencil2d_7pt(16)
    kw = dict(eps=(w["eps0"], w["eps0"]), balance=w["balance"])
    lit = S.build_schedule(m.n, m.row_ptr, m.col, w["n_threads"], global_lb=True, **kw)
    pair = S.build_schedule(m.n, m.row_ptr, m.col, w["n_threads"], **kw)
    st0 = [nd for nd in lit.nodes if nd.stage == 0]
    assert lit.n_eff_root == g["n_eff_root"]
    assert (st0[4].lo, st0[4].hi - 1) == (g["t0_4_first_vertex"], g["t0_4_last_vertex"])
    # the printed values are those of the pair balancing alone
    assert pair.n_eff_root == w["n_eff_root"] != lit.n_eff_root


# ---------------------------------------------------------------------------
# the nonzero load metric

def dense_full(m):
    a = np.zeros((m.n, m.n))
    for r in range(m.n):
        for i in range(m.row_ptr[r], m.row_ptr[r + 1]):
            a[r, m.col[i]] = 1.0
            a[m.col[i], r] = 1.0
    return a


def check_row_loads(fn):
    for m in [matgen.stencil2d_5pt(7), matgen.random_symmetric(60, 0.08, seed=3),
              matgen.banded_irregular(80, seed=4, band=9)]:
        got = fn(m.n, m.row_ptr, m.col, "nnz")
        assert np.array_equal(got, np.count_nonzero(dense_full(m), axis=1))
        assert np.array_equal(fn(m.n, m.row_ptr, m.col, "rows"), np.ones(m.n))
    # closed forms: 5-point 5 inside, 4 on an edge, 3 at a corner; 27-point 27 / 8
    s = 6
    m = matgen.stencil2d_5pt(s)
    ld = fn(m.n, m.row_ptr, m.col, "nnz").reshape(s, s)
    assert ld[0, 0] == 3 and ld[0, 3] == 4 and ld[3, 3] == 5
    m = matgen.stencil3d_27pt(5, seed=1)
    ld = fn(m.n, m.row_ptr, m.col, "nnz").reshape(5, 5, 5)
    assert ld[0, 0, 0] == 8 and ld[2, 2, 2] == 27 and ld[0, 2, 2] == 18 and ld[0, 0, 2] == 12


def test_row_loads_dense_counts_and_closed_forms():
    check_row_loads(S.row_loads)


# ---------------------------------------------------------------------------
# planted mistakes: each must fail one of the pins above

def test_planted_identity_balancing_fails():
    ident = lambda t, w, m, k: list(t)
    with pytest.raises(AssertionError):
        check_examples(ident)
    with pytest.raises(AssertionError):
        paper_property(ident)


def test_planted_mean_over_parent_threads_fails(monkeypatch):
    # the listing's mean = sum / nthreads, with nthreads the parent's thread
    # count (the sum of the pairs' workers) instead of the colour's groups
    def var_over_threads(t_ptr, worker, prefix):
        ng = len(worker)
        per = [float(int(prefix[t_ptr[i + 1]] - prefix[t_ptr[i]])) / float(worker[i]) for i in range(ng)]
        nthreads = float(sum(worker[0::2]))
        mean_r = sum(per[0::2]) / nthreads
        mean_b = sum(per[1::2]) / nthreads
        diff = [per[i] - (mean_r if i % 2 == 0 else mean_b) for i in range(ng)]
        return diff, sum(d * d for d in diff) / ng

    monkeypatch.setattr(S, "_variance", var_over_threads)
    with pytest.raises(AssertionError):
        check_examples(S.load_balance)


def test_planted_upper_row_counts_fail():
    def upper_counts(n, row_ptr, col, balance):
        if balance == "rows":
            return np.ones(n, dtype=np.int64)
        return np.diff(np.asarray(row_ptr, dtype=np.int64))

    with pytest.raises(AssertionError):
        check_row_loads(upper_counts)
