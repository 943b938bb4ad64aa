"""GPU parity of the Gauss-Seidel sweep over distance-1 RACE schedules.

The library sweeps in the schedule's order (phase by phase, leaves of one
phase concurrently, rows of a leaf ascending in the permuted numbering).
The oracle runs the plain serial sweep over the same rows in the same
order (the C oracle, bit-equal to the Python one pinned against dense
triangular solves).  Summation order inside a row differs (the GPU sums a
row's products across 64 or, with four leaves per wavefront, 16 lanes), so
the results agree within rounding:
||x - x_ref||_inf / ||x_ref||_inf <= 1e-12 on diagonally dominant matrices,
after one or several sweeps.
"""
import numpy as np
import pytest

import matgen
import paper_1907_06487_amd as R
from oracle import gauss_seidel as G
from oracle import symmspmv as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dominant(m):
    """The matrix with its diagonal replaced by 1 + the absolute
    off-diagonal row sum (Gauss-Seidel converges; rounding stays small)."""
    absrow = O.abs_product(m.n, m.row_ptr, m.col, m.val, np.ones(m.n))
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    d = rows == m.col
    v = m.val.copy()
    v[d] = 1.0 + absrow[rows[d]] - np.abs(m.val[d])
    return matgen.UpperCSR(m.n, m.row_ptr, m.col, v, m.name + "_dominant")


def race_rows(s):
    tr = s.tree()
    node, phase = s.leaves()
    lo = np.asarray(tr["lo"])[node]
    hi = np.asarray(tr["hi"])[node]
    return G.race_order(s.perm(), lo, hi, phase)


def run_gs(m, b, x0, direction, sweeps, quad=-1, exec_mode="phases", **params):
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, dist_k=1, **params)
    try:
        s.set_gs_quad(quad)
        s.set_gs_exec(exec_mode)
        bd = torch.as_tensor(b, device=DEV)
        xd = torch.as_tensor(x0, device=DEV)
        bp, xp = torch.empty_like(bd), torch.empty_like(xd)
        s.permute(bd, bp, to_permuted=True)
        s.permute(xd, xp, to_permuted=True)
        for _ in range(sweeps):
            s.gauss_seidel(bp, xp, direction)
        out = torch.empty_like(xd)
        s.permute(xp, out, to_permuted=False)
        torch.cuda.synchronize()
        s.check()  # a dataflow wait that gave up
        return out.cpu().numpy(), race_rows(s), s.stats()
    finally:
        s.close()


def oracle(m, b, x0, order, direction, sweeps):
    x = x0
    for _ in range(sweeps):
        if direction == "forward":
            x = G.sweep_c(m.n, m.row_ptr, m.col, m.val, b, x, order)
        elif direction == "backward":
            x = G.sweep_c(m.n, m.row_ptr, m.col, m.val, b, x, list(reversed(order)))
        else:
            x = G.symmetric_sweep_c(m.n, m.row_ptr, m.col, m.val, b, x, order)
    return x


CASES = [
    ("2d5pt_100", matgen.config_2d_small, dict(n_workers=64)),
    ("worked_16x16", lambda: dominant(matgen.stencil2d_7pt(16)), dict(n_workers=8, eps=(0.6, 0.6), balance="rows")),
    ("3d27pt_24", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=256)),
    ("3d27pt_24_stage0", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=64, max_stages=1)),
    ("banded_40k", lambda: dominant(matgen.banded_irregular(40000, seed=6, band=4000)), dict(n_workers=1024)),
    ("banded_40k_cm", lambda: dominant(matgen.banded_irregular(40000, seed=6, band=4000)),
     dict(n_workers=1024, level_order="cm", root="peripheral")),
    ("rand_islands", lambda: dominant(matgen.random_symmetric(500, 0.003, seed=8)), dict(n_workers=16)),
    ("one_row", lambda: matgen.UpperCSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([3.0])),
     dict(n_workers=4)),
    ("long_rows", lambda: dominant(matgen.random_symmetric(600, 0.3, seed=10)), dict(n_workers=4)),
    # leaves of thousands of rows: windows past 2048 entries take one leaf per wavefront
    ("3d27pt_24_big_leaves", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=2)),
    # phases whose leaf count is not a multiple of four (four leaves per wavefront)
    ("3d27pt_17", lambda: matgen.stencil3d_27pt(17, seed=7), dict(n_workers=333)),
]


@pytest.mark.parametrize("quad,exec_mode", [(-2, "phases"), (0, "phases"), (-1, "flow")],
                         ids=["one_leaf_per_wave", "four_leaves_per_wave", "dataflow"])
@pytest.mark.parametrize("direction", ["forward", "backward", "symmetric"])
@pytest.mark.parametrize("name,make,params", CASES, ids=[c[0] for c in CASES])
def test_gauss_seidel_parity(name, make, params, direction, quad, exec_mode):
    m = make()
    rng = np.random.default_rng(11)
    b = rng.uniform(-1, 1, m.n)
    x0 = rng.uniform(-1, 1, m.n)
    sweeps = 3 if direction == "symmetric" else 1
    print(f"case gs {name} {direction} x{sweeps} quad={quad} exec={exec_mode}: n={m.n} nnz={m.nnz} {params}",
          flush=True)
    x, order, st = run_gs(m, b, x0, direction, sweeps, quad=quad, exec_mode=exec_mode, **params)
    ref = oracle(m, b, x0, order, direction, sweeps)
    err = float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))
    print(f"[gs {name} {direction}] leaves={st['n_leaves']} phases={st['n_phases_used']} "
          f"window={st['max_window']} err_norm={err:.3e}", flush=True)
    assert err <= 1e-12


def test_gauss_seidel_converges_and_refuses_products():
    """Repeated symmetric sweeps drive the residual of an SPD system down
    (the method is Gauss-Seidel, not a look-alike); a distance-1 schedule
    refuses the SymmSpMV products, a distance-2 one the sweep."""
    m = matgen.stencil3d_27pt(20, seed=12)
    rng = np.random.default_rng(13)
    xs = rng.uniform(-1, 1, m.n)
    b = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, xs)
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, dist_k=1, n_workers=512)
    s2 = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=64)
    try:
        bd = torch.as_tensor(b, device=DEV)
        bp = torch.empty_like(bd)
        s.permute(bd, bp, True)
        xp = torch.zeros_like(bp)
        res = []
        for _ in range(4):
            s.gauss_seidel(bp, xp)
            x = torch.empty_like(xp)
            s.permute(xp, x, False)
            torch.cuda.synchronize()
            xh = x.cpu().numpy()
            res.append(np.linalg.norm(b - O.symm_spmv(m.n, m.row_ptr, m.col, m.val, xh)) / np.linalg.norm(b))
        print(f"relative residuals {res}", flush=True)
        assert all(r1 < 0.5 * r0 for r0, r1 in zip(res, res[1:]))
        y = torch.empty_like(bp)
        with pytest.raises(R.RaceError):
            s.spmv(bp, y)
        with pytest.raises(R.RaceError):
            s2.gauss_seidel(bp, y)
    finally:
        s.close()
        s2.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("nt,exec_mode", [(4096, "phases"), (16384, "phases"), (16384, "flow"), (65536, "flow")])
def test_gauss_seidel_full_size_3d27pt_128(nt, exec_mode):
    """The 128^3 stencil, one symmetric sweep, against the C oracle over
    the same row order (about 2 s on one host core); N_t 16384 with one
    dataflow launch is the benchmark's configuration; with phase launches
    its large phases run four leaves per wavefront (the default threshold)."""
    m = matgen.config_3d_128()
    rng = np.random.default_rng(14)
    b = rng.uniform(-1, 1, m.n)
    x0 = np.zeros(m.n)
    print(f"case gs 3d27pt_128 nt={nt} exec={exec_mode}: n={m.n}", flush=True)
    x, order, st = run_gs(m, b, x0, "symmetric", 1, n_workers=nt, exec_mode=exec_mode)
    ref = oracle(m, b, x0, order, "symmetric", 1)
    err = float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))
    print(f"[gs 3d27pt_128] leaves={st['n_leaves']} window={st['max_window']} err_norm={err:.3e}", flush=True)
    assert err <= 1e-12
