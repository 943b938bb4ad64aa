"""Host-side checks of librace.so (CPU only, no device calls).

* the library loads and exports every entry point include/race.h declares;
* the native schedule is bit-exact against the oracle (permutation, tree,
  leaf order, phases, N_eff, eta);
* the kernel layout (units, halos, first-writer flags) is consistent with an
  independent derivation from the exported schedule, and every schedule
  passes the brute-force conflict checker;
* malformed inputs return the documented error codes.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import matgen
import paper_1907_06487_amd as R
from paper_1907_06487_amd import _lib
from oracle import checker as C
from oracle import schedule as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "race.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(race_\w+)\s*\(", hdr, flags=re.M))
    assert declared == set(_lib.EXPORTS)
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


def _oracle(m, nt, **kw):
    return S.build_schedule(m.n, m.row_ptr, m.col, nt, eps=kw.get("eps", S.DEFAULT_EPS),
                            balance=kw.get("balance", "nnz"), max_stages=kw.get("max_stages", 4),
                            global_lb=kw.get("global_lb", False), root=kw.get("root", "first"),
                            level_order=kw.get("level_order", "input"), k=kw.get("dist_k", 2))


def _compare(m, nt, **kw):
    ref = _oracle(m, nt, **kw)
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, upload=False, n_workers=nt, **kw)
    try:
        assert np.array_equal(s.perm(), ref.perm)
        tr = s.tree()
        assert len(tr["lo"]) == len(ref.nodes)
        for key, attr in [("stage", "stage"), ("color", "color"), ("parent", "parent"), ("lo", "lo"), ("hi", "hi"),
                          ("workers", "b")]:
            assert np.array_equal(tr[key], [getattr(nd, attr) for nd in ref.nodes]), key
        node, phase = s.leaves()
        assert np.array_equal(node, ref.leaves)
        assert np.array_equal(phase, ref.leaf_phase)
        st = s.stats()
        assert st["eta"] == ref.eta and st["n_eff_root"] == ref.n_eff_root
        assert st["n_phases"] == ref.n_phases and st["n_levels0"] == ref.stage0_levels
        return s, ref
    except Exception:
        s.close()
        raise


CASES = [
    ("worked_16x16", lambda: matgen.stencil2d_7pt(16), 8, dict(eps=(0.6, 0.6), balance="rows")),
    ("worked_16x16_global", lambda: matgen.stencil2d_7pt(16), 8, dict(eps=(0.6, 0.6), balance="rows", global_lb=True)),
    ("2d5pt_100", matgen.config_2d_small, 64, {}),
    ("2d5pt_100_rows", matgen.config_2d_small, 200, dict(balance="rows")),
    ("3d27pt_20", lambda: matgen.stencil3d_27pt(20, seed=4), 128, {}),
    ("3d27pt_20_global", lambda: matgen.stencil3d_27pt(20, seed=4), 96, dict(global_lb=True, max_stages=6)),
    ("banded_30k", lambda: matgen.banded_irregular(30000, seed=6, band=3000), 256, {}),
    ("rand_islands", lambda: matgen.random_symmetric(400, 0.003, seed=8), 16, {}),
    ("rand_nodiag", lambda: matgen.random_symmetric(300, 0.02, seed=9, with_diag=False), 12, {}),
    ("one_row", lambda: matgen.UpperCSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.ones(1)), 4, {}),
    ("empty", lambda: matgen.UpperCSR(0, np.array([0], np.int32), np.array([], np.int32), np.zeros(0)), 4, {}),
    # stage-0 root and in-level order (pseudo-peripheral root, Cuthill-McKee numbering)
    ("3d27pt_14_relabel_peripheral_cm", lambda: matgen.relabel(matgen.stencil3d_27pt(14, seed=4), 3), 64,
     dict(root="peripheral", level_order="cm")),
    ("3d27pt_14_relabel_peripheral", lambda: matgen.relabel(matgen.stencil3d_27pt(14, seed=4), 3), 64,
     dict(root="peripheral")),
    ("banded_30k_cm", lambda: matgen.banded_irregular(30000, seed=6, band=3000), 256, dict(level_order="cm")),
    ("rand_islands_peripheral_cm", lambda: matgen.random_symmetric(400, 0.003, seed=8), 16,
     dict(root="peripheral", level_order="cm", global_lb=True)),
    # wider colorings (distance 3 and 4)
    ("2d5pt_100_k3", matgen.config_2d_small, 64, dict(dist_k=3)),
    ("3d27pt_20_k3", lambda: matgen.stencil3d_27pt(20, seed=4), 128, dict(dist_k=3)),
    ("banded_30k_k4_global", lambda: matgen.banded_irregular(30000, seed=6, band=3000), 256,
     dict(dist_k=4, global_lb=True)),
    # distance-1 colorings (Gauss-Seidel sweeps)
    ("worked_16x16_k1", lambda: matgen.stencil2d_7pt(16), 8, dict(eps=(0.6, 0.6), balance="rows", dist_k=1)),
    ("2d5pt_100_k1", matgen.config_2d_small, 64, dict(dist_k=1)),
    ("3d27pt_20_k1", lambda: matgen.stencil3d_27pt(20, seed=4), 512, dict(dist_k=1)),
    ("banded_30k_k1_cm", lambda: matgen.banded_irregular(30000, seed=6, band=3000), 1024,
     dict(dist_k=1, level_order="cm", global_lb=True)),
]


@pytest.mark.parametrize("name,make,nt,kw", CASES, ids=[c[0] for c in CASES])
def test_schedule_bit_exact_vs_oracle(name, make, nt, kw):
    m = make()
    s, ref = _compare(m, nt, **kw)
    s.close()


@pytest.mark.slow
def test_schedule_bit_exact_3d27pt_128():
    m = matgen.config_3d_128()
    s, ref = _compare(m, 1024)
    s.close()


def touch_flags(n, unit_leaf, leaf_phase, lo, hi, halo_ptr, halo, shared_atomics):
    """Independent derivation of the flush flags.  An index is shared when two
    or more units of one leaf touch it (only with shared_atomics).  Walking
    units in execution order, the first unit touching an index writes it;
    when that touch is shared the index is cleared before the product
    instead.  Two leaves of one phase must never share an index."""
    n_units = len(lo)
    touches = [np.concatenate([np.arange(lo[u], hi[u]), halo[halo_ptr[u]:halo_ptr[u + 1]]]) for u in range(n_units)]
    shared = [np.zeros(t.size, dtype=bool) for t in touches]
    if shared_atomics:
        for leaf in np.unique(unit_leaf):
            us = np.flatnonzero(unit_leaf == leaf)
            if us.size < 2:
                continue
            cnt = np.bincount(np.concatenate([touches[u] for u in us]), minlength=n)
            for u in us:
                shared[u] = cnt[touches[u]] > 1
    seen_phase = np.full(n, -1, dtype=np.int64)
    seen_leaf = np.full(n, -1, dtype=np.int64)
    row_flags = np.zeros(n, dtype=np.uint8)
    halo_flags = np.zeros(len(halo), dtype=np.uint8)
    zero = []
    for u in range(n_units):
        leaf = unit_leaf[u]
        ph = leaf_phase[leaf]
        idx = touches[u]
        clash = (seen_phase[idx] == ph) & (seen_leaf[idx] != leaf)
        assert not clash.any()
        fresh = seen_phase[idx] < 0
        flags = ((fresh & ~shared[u]).astype(np.uint8)) | (shared[u].astype(np.uint8) << 1)
        zero.append(idx[fresh & shared[u]])
        r = hi[u] - lo[u]
        row_flags[lo[u]:hi[u]] = flags[:r]
        halo_flags[halo_ptr[u]:halo_ptr[u + 1]] = flags[r:]
        seen_phase[idx] = ph
        seen_leaf[idx] = leaf
    zero = np.sort(np.concatenate(zero)) if zero else np.zeros(0, np.int64)
    return row_flags, halo_flags, zero


@pytest.mark.parametrize("shared", [True, False], ids=["shared", "chain"])
@pytest.mark.parametrize("name,make,nt,kw", CASES[:9], ids=[c[0] for c in CASES[:9]])
def test_layout_consistent(name, make, nt, kw, shared):
    m = make()
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, upload=False, n_workers=nt, window_max=256, shared_atomics=shared,
                   **kw)
    try:
        u = s.units()
        node, phase = s.leaves()
        tr = s.tree()
        # units tile each leaf in order
        for t, nd in enumerate(node):
            sel = np.flatnonzero(u["unit_leaf"] == t)
            if tr["hi"][nd] == tr["lo"][nd]:
                assert sel.size == 0
                continue
            assert u["lo"][sel[0]] == tr["lo"][nd] and u["hi"][sel[-1]] == tr["hi"][nd]
            assert np.array_equal(u["lo"][sel[1:]], u["hi"][sel[:-1]])
        # halo = distinct columns at or beyond the unit's end, ascending
        perm = s.perm()
        rp, cols, _ = S.permute_upper(m.n, m.row_ptr, m.col, m.val, perm)
        for k in range(len(u["lo"])):
            a, b = u["lo"][k], u["hi"][k]
            want = np.unique(cols[rp[a]:rp[b]])
            want = want[want >= b]
            got = u["halo"][u["halo_ptr"][k]:u["halo_ptr"][k + 1]]
            assert np.array_equal(got, want)
            assert (b - a) + got.size <= 256
        rf, hf, zero = touch_flags(m.n, u["unit_leaf"], phase, u["lo"], u["hi"], u["halo_ptr"], u["halo"], shared)
        assert np.array_equal(rf, u["row_flags"])
        assert np.array_equal(hf, u["halo_flags"])
        assert np.array_equal(zero, s.zero_list())
        st = s.stats()
        assert st["n_zeroed"] == zero.size
        assert st["shared_touches"] == int(((rf >> 1) & 1).sum() + ((hf >> 1) & 1).sum())
        if not shared:
            assert zero.size == 0 and st["shared_touches"] == 0
        # the schedule itself passes the brute-force checker
        C.check_schedule(m.n, m.row_ptr, m.col, perm, tr["lo"], tr["hi"], tr["color"], tr["parent"], node, phase)
    finally:
        s.close()


def _expect(code, fn):
    with pytest.raises(_lib.RaceError) as ei:
        fn()
    assert ei.value.code == code, str(ei.value)


def test_error_codes():
    ok_rp = np.array([0, 2, 3], np.int32)
    ok_col = np.array([0, 1, 1], np.int32)
    v = np.ones(3)
    h = R.race_build_schedule(2, ok_rp, ok_col, v)
    R.race_schedule_destroy(h)
    _expect(-1, lambda: R.race_build_schedule(2, ok_rp, np.array([1, 0, 1], np.int32), v))       # unsorted
    _expect(-1, lambda: R.race_build_schedule(2, ok_rp, np.array([0, 1, 0], np.int32), v))       # col < row
    _expect(-1, lambda: R.race_build_schedule(2, ok_rp, np.array([0, 2, 1], np.int32), v))       # out of range
    _expect(-1, lambda: R.race_build_schedule(2, np.array([1, 2, 3], np.int32), ok_col, v))       # row_ptr[0]
    _expect(-1, lambda: R.race_build_schedule(2, np.array([0, 2, 1], np.int32), ok_col, v))       # decreasing
    _expect(-1, lambda: R.race_build_schedule(2, ok_rp, np.array([0, 0, 1], np.int32), v))       # duplicate
    p = R.make_params(dist_k=1, value_type="f32")  # distance-1 schedules take float64 values only
    _expect(-4, lambda: R.race_build_schedule(2, ok_rp, ok_col, v, p))
    p = R.make_params(dist_k=1)  # Gauss-Seidel needs every diagonal
    _expect(-1, lambda: R.race_build_schedule(2, ok_rp, ok_col, np.array([1.0, 1.0, 0.0]), p))
    h = R.race_build_schedule(2, ok_rp, ok_col, v, p)
    R.race_schedule_destroy(h)
    p = R.make_params(n_workers=0)
    _expect(-1, lambda: R.race_build_schedule(2, ok_rp, ok_col, v, p))
    p = R.make_params(window_max=100000)
    _expect(-1, lambda: R.race_build_schedule(2, ok_rp, ok_col, v, p))
    p = R.make_params(dist_k=9)
    _expect(-1, lambda: R.race_build_schedule(2, ok_rp, ok_col, v, p))
    p = R.make_params()
    p.root_mode = 2
    _expect(-1, lambda: R.race_build_schedule(2, ok_rp, ok_col, v, p))
    p = R.make_params()
    p.level_order = -1
    _expect(-1, lambda: R.race_build_schedule(2, ok_rp, ok_col, v, p))
    p = R.make_params(block_threads=100)
    _expect(-1, lambda: R.race_build_schedule(2, ok_rp, ok_col, v, p))
    p = R.make_params()
    p.shared_atomics = 2
    _expect(-1, lambda: R.race_build_schedule(2, ok_rp, ok_col, v, p))
    for bad in (-1, 17):
        p = R.make_params(rhs_tile=bad)
        _expect(-1, lambda: R.race_build_schedule(2, ok_rp, ok_col, v, p))
    # a row whose window alone exceeds the budget
    n = 40
    rp = np.array([0, n] + [n + i for i in range(1, n)], np.int32)
    col = np.concatenate([np.arange(n), np.arange(1, n)]).astype(np.int32)
    _expect(-4, lambda: R.race_build_schedule(n, rp, col, np.ones(col.size), R.make_params(window_max=16)))
    # products need an uploaded schedule with values
    h = R.race_build_schedule(2, ok_rp, ok_col, None)
    _expect(-5, lambda: R.race_schedule_upload(h))
    R.race_schedule_destroy(h)


def _fuzz_case(seed):
    """A seeded random matrix and schedule parameters: structure, size,
    density, N_t, eps, depth, load metric and the global pass all drawn."""
    rng = np.random.default_rng(seed)
    kind = int(rng.integers(5))
    if kind == 0:
        m = matgen.random_symmetric(int(rng.integers(50, 1500)), float(rng.uniform(0.001, 0.01)), seed=seed,
                                    with_diag=bool(rng.integers(2)))
    elif kind == 1:
        m = matgen.stencil2d_5pt(int(rng.integers(8, 70)), seed=seed)
    elif kind == 2:
        m = matgen.stencil3d_27pt(int(rng.integers(4, 18)), seed=seed)
    elif kind == 3:
        n = int(rng.integers(500, 8000))
        m = matgen.banded_irregular(n, seed=seed, band=int(rng.integers(2, max(3, n // 8))))
    else:
        m = matgen.stencil2d_7pt(int(rng.integers(8, 50)))
    eps0 = float(rng.choice([0.5, 0.6, 0.7, 0.8, 0.9]))
    kw = dict(eps=(eps0, float(rng.choice([0.5, 0.8])), 0.5), balance=str(rng.choice(["nnz", "rows"])),
              max_stages=int(rng.integers(1, 6)), global_lb=bool(rng.integers(2)))
    nt = int(rng.choice([2, 5, 8, 16, 32, 64, 128, 256]))
    kw["root"] = str(rng.choice(["first", "first", "peripheral"]))
    kw["level_order"] = str(rng.choice(["input", "input", "cm"]))
    kw["dist_k"] = int(rng.choice([2, 2, 2, 3, 4, 1]))
    if rng.integers(4) == 0:
        m = matgen.relabel(m, seed)
    if kw["dist_k"] == 1 and not _full_diagonal(m):
        kw["dist_k"] = 2  # distance-1 schedules carry a Gauss-Seidel layout, which needs every diagonal
    return m, nt, kw


def _full_diagonal(m):
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    d = rows == m.col
    return np.count_nonzero(d & (m.val != 0)) == m.n


@pytest.mark.parametrize("seed", range(150))
def test_schedule_fuzz_bit_exact_and_valid(seed):
    """Random matrices and parameters: the native builder equals the oracle
    bit for bit, and the schedule passes the brute-force conflict checker."""
    m, nt, kw = _fuzz_case(seed)
    s, ref = _compare(m, nt, **kw)
    try:
        tr = s.tree()
        node, phase = s.leaves()
        C.check_schedule(m.n, m.row_ptr, m.col, s.perm(), tr["lo"], tr["hi"], tr["color"], tr["parent"], node, phase,
                         dist=1 if kw["dist_k"] == 1 else 2)
        if kw["dist_k"] != 2 and m.n <= 2000:
            lo, hi = np.asarray(tr["lo"])[node], np.asarray(tr["hi"])[node]
            C.check_dense_distance_k(m.n, m.row_ptr, m.col, s.perm(), lo, hi, phase, kw["dist_k"])
    finally:
        s.close()


def test_complex_schedules_host():
    """Complex value types build on the host (same schedule as real values)
    and refuse the modes that take real values only."""
    m = matgen.stencil3d_27pt(8, seed=2)
    vc = m.val + 1j * np.linspace(-1, 1, m.nnz)
    s_r = R.Schedule(m.n, m.row_ptr, m.col, m.val, upload=False, n_workers=32, window_max=2176)
    for vt in ("c128", "c128h"):
        s = R.Schedule(m.n, m.row_ptr, m.col, vc, upload=False, n_workers=32, value_type=vt, window_max=2176)
        try:
            assert np.array_equal(s.perm(), s_r.perm())
            assert s.stats()["n_units"] == s_r.stats()["n_units"]
            assert s.stats()["bytes_kernel"] > s_r.stats()["bytes_kernel"]
        finally:
            s.close()
    s_r.close()
    p = R.make_params(value_type="c128", exec_mode="phases")
    _expect(-4, lambda: R.race_build_schedule(m.n, m.row_ptr, m.col, vc, p))
    p = R.make_params()
    p.value_type = 4
    _expect(-1, lambda: R.race_build_schedule(m.n, m.row_ptr, m.col, m.val, p))


@pytest.mark.parametrize("name,make,kw,want", [
    ("banded_40k_w96", lambda: matgen.banded_irregular(40000, seed=6, band=4000), dict(n_workers=16, window_max=96), 1),
    ("3d27pt_24", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=256), 0),
    ("2d5pt_100", matgen.config_2d_small, dict(n_workers=64), 0),
])
def test_low_locality_decision(name, make, kw, want):
    """low_locality=auto expands exactly when more than half of all window
    touches (own rows plus halo entries of every unit) carry the shared
    flag, recounted here from the unit flags; race never expands, expanded
    always does; distance-1 and complex schedules never do."""
    m = make()
    for mode, expect in (("auto", None), ("race", 0), ("expanded", 1)):
        s = R.Schedule(m.n, m.row_ptr, m.col, m.val, upload=False, low_locality=mode, **kw)
        try:
            st = s.stats()
            if expect is None:
                u = s.units()
                shared = sum(int(np.count_nonzero(u["row_flags"][lo:hi] & 2)) for lo, hi in zip(u["lo"], u["hi"]))
                shared += int(np.count_nonzero(u["halo_flags"] & 2))
                touches = m.n + len(u["halo"])
                expect = int(2 * shared > touches)
                assert expect == want, (shared, touches)
            assert st["product_path"] == expect, mode
            assert (st["expanded_per_thread"] > 0) == bool(expect)
        finally:
            s.close()
    g = matgen.config_2d_small()
    s = R.Schedule(g.n, g.row_ptr, g.col, g.val, upload=False, low_locality="expanded", dist_k=1, n_workers=64)
    assert s.stats()["product_path"] == 0
    s.close()
    with pytest.raises(_lib.RaceError):
        p = R.make_params()
        p.low_locality = 3
        R.race_build_schedule(m.n, m.row_ptr, m.col, m.val, p)


@pytest.mark.parametrize("name,make,kw", [
    ("3d27pt_16_w256", lambda: matgen.stencil3d_27pt(16, seed=3), dict(n_workers=64, window_max=256)),
    ("banded_8k_w200", lambda: matgen.banded_irregular(8000, seed=4, band=800), dict(n_workers=32, window_max=200)),
    ("rand_islands", lambda: matgen.random_symmetric(400, 0.004, seed=6), dict(n_workers=8, window_max=64)),
])
def test_matrix_power_read_deps(name, make, kw):
    """A unit of power p reads y_(p-1) on its touch set (own rows and halo):
    it must wait for exactly the units whose touch sets meet it, itself
    included.  Recomputed here by brute force over pairs of units."""
    m = make()
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, upload=False, **kw)
    try:
        u = s.units()
        touch = [set(range(u["lo"][i], u["hi"][i])) | set(u["halo"][u["halo_ptr"][i]:u["halo_ptr"][i + 1]].tolist())
                 for i in range(len(u["lo"]))]
        ptr, idx = s.read_deps()
        for i in range(len(touch)):
            want = [j for j in range(len(touch)) if touch[i] & touch[j]]
            assert idx[ptr[i]:ptr[i + 1]].tolist() == want, i
    finally:
        s.close()


def test_gs_quad_knob_arguments():
    """race_schedule_set_gs_quad: distance-1 schedules only, -2..any."""
    g = matgen.config_2d_small()
    s = R.Schedule(g.n, g.row_ptr, g.col, g.val, upload=False, dist_k=1, n_workers=64)
    s2 = R.Schedule(g.n, g.row_ptr, g.col, g.val, upload=False, n_workers=64)
    try:
        for v in (-2, -1, 0, 100):
            s.set_gs_quad(v)
        with pytest.raises(_lib.RaceError):
            s.set_gs_quad(-3)
        with pytest.raises(_lib.RaceError):
            s2.set_gs_quad(0)
    finally:
        s.close()
        s2.close()


def test_kaczmarz_layout_and_refusals():
    """race_params.kaczmarz: built on distance-2 schedules of real values
    (windows reported in the stats), refused with dist_k 1 or complex
    values; race_symm_kacz refuses schedules without the layout and
    schedules not uploaded before touching any device."""
    g = matgen.config_2d_small()
    s = R.Schedule(g.n, g.row_ptr, g.col, g.val, upload=False, n_workers=64, kaczmarz=True)
    s0 = R.Schedule(g.n, g.row_ptr, g.col, g.val, upload=False, n_workers=64)
    try:
        s.set_gs_quad(0)  # the four-leaves-per-wavefront threshold serves Kaczmarz sweeps too
        w = s.stats()["kacz_max_window"]
        assert 0 < w <= 16384
        assert s0.stats()["kacz_max_window"] == 0
        assert _lib.lib().race_symm_kacz(s.handle, None, None, 2, 1.0, None) == -5  # not uploaded
        assert _lib.lib().race_symm_kacz(s0.handle, None, None, 2, 1.0, None) == -5  # no layout
        for kw in (dict(dist_k=1), dict(value_type="c128")):
            with pytest.raises(_lib.RaceError):
                R.Schedule(g.n, g.row_ptr, g.col, g.val, upload=False, n_workers=64, kaczmarz=True, **kw)
        # windows too large for the LDS of one wavefront
        big = matgen.stencil3d_27pt(40, seed=1)
        with pytest.raises(_lib.RaceError):
            R.Schedule(big.n, big.row_ptr, big.col, big.val, upload=False, n_workers=1, max_stages=1, kaczmarz=True)
    finally:
        s.close()
        s0.close()
