"""GPU parity of the Kaczmarz sweep over distance-2 RACE schedules.

The library sweeps in the schedule's order (phase by phase, leaves of one
phase concurrently, rows of a leaf ascending in the permuted numbering).
The oracle runs the plain serial sweep over the same rows in the same order
(the C oracle, bit-equal to the Python one pinned against SOR on the
row-action system).  The GPU sums a row's dot product across 64 lanes and
takes the squared row norm from the host layout, so the results agree
within rounding: ||x - x_ref||_inf / ||x_ref||_inf <= 1e-12 after one or
several sweeps.
"""
import numpy as np
import pytest

import matgen
import paper_1907_06487_amd as R
from oracle import gauss_seidel as G
from oracle import kaczmarz as K
from oracle import symmspmv as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def race_rows(s):
    tr = s.tree()
    node, phase = s.leaves()
    lo = np.asarray(tr["lo"])[node]
    hi = np.asarray(tr["hi"])[node]
    return G.race_order(s.perm(), lo, hi, phase)


def run_kacz(m, b, x0, direction, sweeps, omega, quad=-1, exec_mode="phases", **params):
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, kaczmarz=True, **params)
    try:
        s.set_gs_quad(quad)
        s.set_gs_exec(exec_mode)
        bd = torch.as_tensor(b, device=DEV)
        xd = torch.as_tensor(x0, device=DEV)
        bp, xp = torch.empty_like(bd), torch.empty_like(xd)
        s.permute(bd, bp, to_permuted=True)
        s.permute(xd, xp, to_permuted=True)
        for _ in range(sweeps):
            s.kaczmarz(bp, xp, direction, omega)
        out = torch.empty_like(xd)
        s.permute(xp, out, to_permuted=False)
        torch.cuda.synchronize()
        s.check()  # a dataflow wait that gave up
        return out.cpu().numpy(), race_rows(s), s.stats()
    finally:
        s.close()


def oracle(m, b, x0, order, direction, sweeps, omega):
    x = x0
    for _ in range(sweeps):
        if direction == "forward":
            x = K.sweep_c(m.n, m.row_ptr, m.col, m.val, b, x, order, omega)
        elif direction == "backward":
            x = K.sweep_c(m.n, m.row_ptr, m.col, m.val, b, x, list(reversed(order)), omega)
        else:
            x = K.symmetric_sweep_c(m.n, m.row_ptr, m.col, m.val, b, x, order, omega)
    return x


def _empty_row():
    # row 3 stores nothing (no diagonal, no neighbour): the sweep skips it
    rp = np.array([0, 2, 4, 5, 5, 6], np.int32)
    col = np.array([0, 1, 1, 2, 2, 4], np.int32)
    val = np.array([3.0, -1.0, 4.0, 0.5, 2.0, 1.5])
    return matgen.UpperCSR(5, rp, col, val, "empty_row")


CASES = [
    ("2d5pt_100", matgen.config_2d_small, dict(n_workers=64)),
    ("3d27pt_24", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=256)),
    ("3d27pt_24_stage0", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=64, max_stages=1)),
    # a narrower band than the SymmSpMV cases: with band 4000 the distance-2
    # recursion leaves a leaf of 15,194 rows, past the window limit
    ("banded_40k", lambda: matgen.banded_irregular(40000, seed=6, band=400), dict(n_workers=1024, max_stages=4)),
    ("banded_40k_cm", lambda: matgen.banded_irregular(40000, seed=6, band=400),
     dict(n_workers=1024, max_stages=4, level_order="cm", root="peripheral")),
    ("rand_islands", lambda: matgen.random_symmetric(500, 0.003, seed=8), dict(n_workers=16)),
    ("one_row", lambda: matgen.UpperCSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([3.0])),
     dict(n_workers=4)),
    ("empty_row", _empty_row, dict(n_workers=2)),
    # rows of more than 64 entries take a second round of lanes
    ("long_rows", lambda: matgen.random_symmetric(600, 0.3, seed=10), dict(n_workers=4)),
    # leaves of thousands of rows
    ("3d27pt_24_big_leaves", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=8, max_stages=2)),
    ("3d27pt_17", lambda: matgen.stencil3d_27pt(17, seed=7), dict(n_workers=333, max_stages=3)),
    # a distance-3 schedule (rows of one phase further apart than needed)
    ("3d27pt_17_dist3", lambda: matgen.stencil3d_27pt(17, seed=7), dict(n_workers=64, dist_k=3)),
    # a schedule whose products store float32 values: the sweep keeps float64
    ("3d27pt_17_f32_products", lambda: matgen.stencil3d_27pt(17, seed=7),
     dict(n_workers=333, max_stages=3, value_type="f32")),
]


@pytest.mark.parametrize("quad,exec_mode", [(-2, "phases"), (0, "phases"), (-2, "flow")],
                         ids=["one_leaf_per_wave", "four_leaves_per_wave", "dataflow"])
@pytest.mark.parametrize("omega", [1.0, 1.4])
@pytest.mark.parametrize("direction", ["forward", "backward", "symmetric"])
@pytest.mark.parametrize("name,make,params", CASES, ids=[c[0] for c in CASES])
def test_kaczmarz_parity(name, make, params, direction, omega, quad, exec_mode):
    m = make()
    rng = np.random.default_rng(11)
    b = rng.uniform(-1, 1, m.n)
    x0 = rng.uniform(-1, 1, m.n)
    sweeps = 2 if direction == "symmetric" else 1
    print(f"case kacz {name} {direction} x{sweeps} omega={omega} quad={quad} exec={exec_mode}: n={m.n} nnz={m.nnz} "
          f"{params}", flush=True)
    x, order, st = run_kacz(m, b, x0, direction, sweeps, omega, quad, exec_mode, **params)
    ref = oracle(m, b, x0, order, direction, sweeps, omega)
    err = float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))
    print(f"[kacz {name} {direction}] leaves={st['n_leaves']} phases={st['n_phases_used']} "
          f"window={st['kacz_max_window']} err_norm={err:.3e}", flush=True)
    assert err <= 1e-12


def test_kaczmarz_converges_captures_and_refuses():
    """Symmetric sweeps on a consistent system shrink the error (the method
    is Kaczmarz, not a look-alike); a captured sweep replays like the eager
    one; omega outside (0, 2) and schedules without the layout are refused."""
    m = matgen.stencil3d_27pt(20, seed=12)
    rng = np.random.default_rng(13)
    xs = rng.uniform(-1, 1, m.n)
    b = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, xs)
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=512, max_stages=3, kaczmarz=True)
    s2 = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=64)
    try:
        bd = torch.as_tensor(b, device=DEV)
        bp = torch.empty_like(bd)
        s.permute(bd, bp, True)
        xp = torch.zeros_like(bp)
        errs = []
        for _ in range(4):
            s.kaczmarz(bp, xp)
            x = torch.empty_like(xp)
            s.permute(xp, x, False)
            torch.cuda.synchronize()
            errs.append(float(np.linalg.norm(x.cpu().numpy() - xs)))
        print(f"errors {errs}", flush=True)
        assert all(e1 < e0 for e0, e1 in zip(errs, errs[1:]))
        # graph capture of one symmetric sweep (x updated in place), replays
        # against eager sweeps from the same start
        xg = torch.zeros_like(bp)
        xe = torch.zeros_like(bp)
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side, capture_error_mode="thread_local"):
                s.kaczmarz(bp, xg, stream=side)
        torch.cuda.synchronize()
        for r in range(3):
            xe.add_(0.0)  # eager work between the replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            s.kaczmarz(bp, xe)
            torch.cuda.synchronize()
            d = float(torch.max(torch.abs(xg - xe)))
            print(f"replay {r}: max difference to eager {d:.3e}", flush=True)
            assert d == 0.0
        for bad in (0.0, 2.0, -1.0):
            with pytest.raises(R.RaceError):
                s.kaczmarz(bp, xp, omega=bad)
        with pytest.raises(R.RaceError):
            s2.kaczmarz(bp, xp)
    finally:
        s.close()
        s2.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("quad,exec_mode", [(-1, "phases"), (0, "phases"), (-1, "flow")])
def test_kaczmarz_full_size_3d27pt_128(quad, exec_mode):
    """The 128^3 stencil at the benchmark's schedule (N_t 4096, 3 stages),
    one symmetric sweep, against the C oracle over the same row order."""
    m = matgen.config_3d_128()
    rng = np.random.default_rng(14)
    b = rng.uniform(-1, 1, m.n)
    x0 = np.zeros(m.n)
    print(f"case kacz 3d27pt_128 quad={quad} exec={exec_mode}: n={m.n}", flush=True)
    x, order, st = run_kacz(m, b, x0, "symmetric", 1, 1.0, quad, exec_mode, n_workers=4096, max_stages=3)
    ref = oracle(m, b, x0, order, "symmetric", 1, 1.0)
    err = float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))
    print(f"[kacz 3d27pt_128] leaves={st['n_leaves']} window={st['kacz_max_window']} err_norm={err:.3e}", flush=True)
    assert err <= 1e-12
