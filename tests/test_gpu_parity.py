"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Inputs are seeded (matgen); the oracle computes y = A x in float64 in the
input order; the library works in its permuted order, so x is permuted on
the device with race_permute and y is brought back the same way.

Tolerance: every y must satisfy ||y - y_ref||_inf / ||y_ref||_inf <= 1e-12
and, per row, |y_i - y_ref,i| <= 4 * gamma_m * (|A||x|)_i where m is the
largest row length of the full matrix (any summation order of m products
stays inside gamma_m; the factor 4 covers the oracle's own rounding and
the float64 atomics' different order).
"""
import math

import numpy as np
import pytest

import matgen
import paper_1907_06487_amd as R
from oracle import symmspmv as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def gamma(m):
    u = 2.0 ** -53
    return m * u / (1.0 - m * u)


def _check(y, y_ref, absax, mlen, tag):
    en, ec = O.errors(y, y_ref, absax)
    bound = 4 * gamma(mlen + 1)
    print(f"[{tag}] err_norm={en:.3e} err_comp={ec:.3e} (bound {bound:.3e})", flush=True)
    assert en <= 1e-12, tag
    assert ec <= bound, tag
    return en, ec


def _full_row_len(m):
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    off = rows != m.col
    deg = np.bincount(rows, minlength=m.n) + np.bincount(m.col[off], minlength=m.n)
    return int(deg.max(initial=0))


def run_race(m, x, k=1, **params):
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, **params)
    try:
        xd = torch.as_tensor(x, device=DEV).contiguous()
        xp = torch.empty_like(xd)
        yp = torch.full_like(xd, float("nan"))  # every entry must be written
        y = torch.empty_like(xd)
        s.permute(xd, xp, to_permuted=True)
        if k == 1:
            s.spmv(xp, yp)
        else:
            s.spmm(xp, yp)
        s.permute(yp, y, to_permuted=False)
        torch.cuda.synchronize()
        s.check()
        return y.cpu().numpy(), s.stats()
    finally:
        s.close()


SMALL = [
    ("2d5pt_100", matgen.config_2d_small, dict(n_workers=64)),
    ("2d5pt_100_nt512", matgen.config_2d_small, dict(n_workers=512)),
    ("worked_16x16", lambda: matgen.stencil2d_7pt(16), dict(n_workers=8, eps=(0.6, 0.6), balance="rows")),
    ("3d27pt_24", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=256)),
    ("3d27pt_24_w128", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=64, window_max=128)),
    ("3d27pt_24_b1024", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=256, block_threads=1024)),
    ("3d27pt_24_b64", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=256, block_threads=64)),
    ("banded_40k", lambda: matgen.banded_irregular(40000, seed=6, band=4000), dict(n_workers=256)),
    ("banded_40k_global", lambda: matgen.banded_irregular(40000, seed=6, band=4000), dict(n_workers=128, global_lb=True)),
    ("rand_islands", lambda: matgen.random_symmetric(500, 0.003, seed=8), dict(n_workers=16)),
    ("rand_nodiag", lambda: matgen.random_symmetric(300, 0.02, seed=9, with_diag=False), dict(n_workers=12)),
    ("one_row", lambda: matgen.UpperCSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([3.0])),
     dict(n_workers=4)),
    ("diag_only", lambda: matgen.UpperCSR(7, np.arange(8, dtype=np.int32), np.arange(7, dtype=np.int32),
                                          np.arange(1.0, 8.0)), dict(n_workers=4)),
    ("2d5pt_100_phases", matgen.config_2d_small, dict(n_workers=64, exec_mode="phases")),
    ("3d27pt_24_w128_phases", lambda: matgen.stencil3d_27pt(24, seed=5),
     dict(n_workers=64, window_max=128, exec_mode="phases")),
    ("banded_40k_phases", lambda: matgen.banded_irregular(40000, seed=6, band=4000),
     dict(n_workers=256, exec_mode="phases")),
    ("rand_islands_phases", lambda: matgen.random_symmetric(500, 0.003, seed=8), dict(n_workers=16, exec_mode="phases")),
    # a leaf's units in order instead of concurrently with shared atomics
    ("3d27pt_24_w128_chain", lambda: matgen.stencil3d_27pt(24, seed=5),
     dict(n_workers=64, window_max=128, shared_atomics=False)),
    ("3d27pt_24_w128_phases_chain", lambda: matgen.stencil3d_27pt(24, seed=5),
     dict(n_workers=64, window_max=128, exec_mode="phases", shared_atomics=False)),
    ("banded_40k_chain", lambda: matgen.banded_irregular(40000, seed=6, band=4000),
     dict(n_workers=256, shared_atomics=False)),
    # many units per leaf: most y entries are shared and combined atomically
    ("banded_40k_w96", lambda: matgen.banded_irregular(40000, seed=6, band=4000), dict(n_workers=16, window_max=96)),
    ("banded_40k_w96_phases", lambda: matgen.banded_irregular(40000, seed=6, band=4000),
     dict(n_workers=16, window_max=96, exec_mode="phases")),
    # stage-0 root and in-level order: a relabelled stencil rebuilt with a
    # pseudo-peripheral root and the Cuthill-McKee numbering
    ("3d27pt_24_relabel_pcm", lambda: matgen.relabel(matgen.stencil3d_27pt(24, seed=5), 3),
     dict(n_workers=256, root="peripheral", level_order="cm")),
    ("3d27pt_24_relabel", lambda: matgen.relabel(matgen.stencil3d_27pt(24, seed=5), 3), dict(n_workers=256)),
    ("banded_40k_cm_phases", lambda: matgen.banded_irregular(40000, seed=6, band=4000),
     dict(n_workers=256, level_order="cm", exec_mode="phases")),
    # wider colorings (distance 3 and 4): still race-free, fewer groups
    ("3d27pt_24_k3", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=256, dist_k=3)),
    ("banded_40k_k4", lambda: matgen.banded_irregular(40000, seed=6, band=4000), dict(n_workers=256, dist_k=4)),
    ("batch_family_irregular", lambda: matgen.batch_family(2, 102), dict(n_workers=4)),
    ("batch_family_irregular_b1024", lambda: matgen.batch_family(5, 105), dict(n_workers=30, block_threads=1024)),
]


@pytest.mark.parametrize("name,make,params", SMALL, ids=[c[0] for c in SMALL])
def test_race_symm_spmv_small(name, make, params):
    m = make()
    print(f"case {name}: n={m.n} nnz={m.nnz} params={params}", flush=True)
    x = matgen.rhs(m.n, 17)
    y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x)
    y, st = run_race(m, x, **params)
    print(f"  phases={st['n_phases_used']} leaves={st['n_leaves']} units={st['n_units']}", flush=True)
    _check(y, y_ref, O.abs_product(m.n, m.row_ptr, m.col, m.val, x), _full_row_len(m), name)


def test_race_empty_matrix():
    m = matgen.UpperCSR(0, np.array([0], np.int32), np.array([], np.int32), np.zeros(0))
    s = R.Schedule(0, m.row_ptr, m.col, m.val, n_workers=4)
    x = torch.zeros(0, dtype=torch.float64, device=DEV)
    y = torch.zeros(0, dtype=torch.float64, device=DEV)
    s.spmv(x, y)
    torch.cuda.synchronize()
    s.close()


@pytest.mark.parametrize("k", [1, 2, 3, 4, 8, 16])
def test_race_symm_spmm(k):
    m = matgen.stencil3d_27pt(16, seed=7)
    X = matgen.rhs(m.n, 23, k=k).reshape(m.n, k) if k > 1 else matgen.rhs(m.n, 23)
    Y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, X)
    window = min(3840, (159 * 1024) // (16 * k + 4) - 16)
    Y, st = run_race(m, X, k=k, n_workers=128, window_max=window)
    absax = O.abs_product(m.n, m.row_ptr, m.col, m.val, np.abs(X))
    for j in range(k):
        yj = Y[:, j] if k > 1 else Y
        rj = Y_ref[:, j] if k > 1 else Y_ref
        aj = absax[:, j] if k > 1 else absax
        _check(yj, rj, aj, _full_row_len(m), f"spmm k={k} col={j}")


@pytest.mark.parametrize("k,tile,window,mode", [(3, 0, 3840, "flow"), (5, 0, 3840, "flow"), (16, 0, 3840, "flow"),
                                               (7, 1, 3840, "flow"), (9, 4, 2000, "flow"), (5, 0, 3840, "phases"),
                                               (9, 2, 3840, "phases")])
def test_race_symm_spmm_tiled(k, tile, window, mode):
    """More right-hand sides than one pass can hold: passes of `tile` columns
    (0: the widest that fits the window) over row-major n x k arrays; with
    four or more passes through contiguous column tiles."""
    m = matgen.stencil3d_27pt(18, seed=8)
    print(f"case spmm tiled k={k} tile={tile} window={window} mode={mode}", flush=True)
    X = matgen.rhs(m.n, 29, k=k).reshape(m.n, k)
    Y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, X)
    Y, st = run_race(m, X, k=k, n_workers=64, window_max=window, rhs_tile=tile, exec_mode=mode)
    absax = O.abs_product(m.n, m.row_ptr, m.col, m.val, np.abs(X))
    for j in range(k):
        _check(Y[:, j], Y_ref[:, j], absax[:, j], _full_row_len(m), f"spmm tiled k={k} col={j}")


def test_race_spmm_column_equals_spmv():
    m = matgen.stencil2d_5pt(60, seed=3)
    X = matgen.rhs(m.n, 31, k=4)
    Y, _ = run_race(m, X, k=4, n_workers=64, window_max=1024)
    for j in range(4):
        yj, _ = run_race(m, np.ascontiguousarray(X[:, j]), n_workers=64, window_max=1024)
        assert np.max(np.abs(Y[:, j] - yj)) <= 1e-12 * np.max(np.abs(yj))


def test_race_float32_values():
    m = matgen.banded_irregular(50000, seed=12, band=5000)
    x = matgen.rhs(m.n, 5)
    v32 = m.val.astype(np.float32)
    y_ref32 = O.symm_spmv(m.n, m.row_ptr, m.col, v32.astype(np.float64), x)
    y_ref64 = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x)
    y, _ = run_race(m, x, n_workers=256, value_type="f32")
    _check(y, y_ref32, O.abs_product(m.n, m.row_ptr, m.col, v32.astype(np.float64), x), _full_row_len(m), "f32 values")
    en64, _ = O.errors(y, y_ref64)
    print(f"[f32 values vs float64 oracle] err_norm={en64:.3e} (stated, not bounded)", flush=True)
    assert en64 < 1e-5


def test_baseline_csr_spmv():
    m = matgen.stencil3d_27pt(20, seed=9)
    x = matgen.rhs(m.n, 9)
    rp, c, v = O.expand_full(m.n, m.row_ptr, m.col, m.val)
    y_ref = O.spmv_full(m.n, rp, c, v, x)
    for lpr in (0, 1, 4, 32):
        h = R.race_csr_create(m.n, rp, c, v, lpr)
        xd = torch.as_tensor(x, device=DEV)
        yd = torch.full_like(xd, float("nan"))
        R.race_csr_spmv(h, xd, yd)
        torch.cuda.synchronize()
        R.race_csr_destroy(h)
        _check(yd.cpu().numpy(), y_ref, O.abs_product(m.n, m.row_ptr, m.col, m.val, x), _full_row_len(m),
               f"csr lpr={lpr}")


def _ragged_crs(n, seed):
    """A general CRS matrix with empty rows (single ones and a run of 3000,
    longer than a row block's row limit), rows longer than every row-block
    capacity (5000 entries), and short rows of random length."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 40, size=n)
    lens[rng.choice(n, n // 10, replace=False)] = 0
    lens[100:3100] = 0
    lens[[0, 7, n // 2, n - 1]] = 5000
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(lens)
    col = np.concatenate([np.sort(rng.choice(n, int(k), replace=False)) for k in lens]).astype(np.int32)
    val = rng.standard_normal(int(rp[-1]))
    return rp, col, val


@pytest.mark.parametrize("per", [4, 8, 16])
@pytest.mark.parametrize("case", ["3d27pt_20", "ragged_9000", "one_row"])
def test_baseline_csr_row_blocks(case, per):
    """The row-block CRS product (lanes_per_row -4/-8/-16) against the
    oracle's SpMV: several blocks and a ragged last one, empty rows, rows
    longer than a block's capacity, a single row."""
    if case == "3d27pt_20":
        m = matgen.stencil3d_27pt(20, seed=9)
        n = m.n
        rp, c, v = O.expand_full(m.n, m.row_ptr, m.col, m.val)
    elif case == "ragged_9000":
        n = 9000
        rp, c, v = _ragged_crs(n, 5)
    else:
        n = 1
        rp, c, v = np.array([0, 1], dtype=np.int32), np.array([0], dtype=np.int32), np.array([3.0])
    x = matgen.rhs(n, 17) if n > 1 else np.array([-2.0])
    y_ref = O.spmv_full(n, rp, c, v, x)
    absax = O.spmv_full(n, rp, c, np.abs(v), np.abs(x))
    print(f"case csr row blocks {case} per={per}: n={n} nnz={int(rp[-1])}", flush=True)
    h = R.race_csr_create(n, rp, c, v, -per)
    try:
        xd = torch.as_tensor(x, device=DEV)
        yd = torch.full_like(xd, float("nan"))
        R.race_csr_spmv(h, xd, yd)
        torch.cuda.synchronize()
    finally:
        R.race_csr_destroy(h)
    y = yd.cpu().numpy()
    mlen = int(np.diff(rp).max(initial=0))
    u = 2.0 ** -53
    g = (mlen + 1) * u / (1 - (mlen + 1) * u)
    en, ec = O.errors(y, y_ref, absax)
    print(f"[csr row blocks {case} per={per}] err_norm={en:.3e} err_comp={ec:.3e}", flush=True)
    assert en <= 1e-12 and ec <= 4 * g
    assert np.all(y[np.diff(rp) == 0] == 0.0)


@pytest.mark.parametrize("lpr", [0, 1, 8, 64])
def test_baseline_atomic_symm(lpr):
    m = matgen.banded_irregular(30000, seed=13, band=3000)
    x = matgen.rhs(m.n, 13)
    y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x)
    h = R.race_atomic_create(m.n, m.row_ptr, m.col, m.val, lpr)
    xd = torch.as_tensor(x, device=DEV)
    yd = torch.full_like(xd, float("nan"))
    R.race_symm_spmv_atomic(h, xd, yd)
    torch.cuda.synchronize()
    R.race_csr_destroy(h)
    _check(yd.cpu().numpy(), y_ref, O.abs_product(m.n, m.row_ptr, m.col, m.val, x), _full_row_len(m),
           f"atomic lpr={lpr}")


def test_race_repeated_calls_and_streams():
    m = matgen.stencil3d_27pt(18, seed=21)
    x = matgen.rhs(m.n, 2)
    y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x)
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=128)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        xd = torch.as_tensor(x, device=DEV)
        xp = torch.empty_like(xd)
        s.permute(xd, xp, True, stream=st)
        outs = []
        for _ in range(3):
            yp = torch.full_like(xd, float("nan"))
            s.spmv(xp, yp, stream=st)
            y = torch.empty_like(xd)
            s.permute(yp, y, False, stream=st)
            outs.append(y)
    st.synchronize()
    s.check()
    for y in outs:
        _check(y.cpu().numpy(), y_ref, O.abs_product(m.n, m.row_ptr, m.col, m.val, x), _full_row_len(m), "repeat")
    s.close()


def _sampled_rows_exact(m, x, rows):
    """Exactly rounded y_i for selected rows (math.fsum of the full row)."""
    out = []
    rp, col, val = m.row_ptr, m.col, m.val
    # lower part of row i = entries (j, i) stored in rows j < i
    for i in rows:
        terms = [val[k] * x[col[k]] for k in range(rp[i], rp[i + 1])]
        out.append(terms)
    cols_i = {int(i): [] for i in rows}
    sel = np.isin(col, rows)
    owners = np.repeat(np.arange(m.n), np.diff(rp))[sel]
    for k, j in zip(np.flatnonzero(sel), owners):
        c = int(col[k])
        if c != j:
            cols_i[c].append(val[k] * x[j])
    return np.array([math.fsum(t + cols_i[int(i)]) for t, i in zip(out, rows)])


@pytest.mark.parametrize("nt,mode,block,stages,window", [(256, "flow", 512, 2, 4064), (256, "flow", 512, 4, 3840),
                                                         (256, "flow", 256, 4, 3840), (1024, "flow", 256, 4, 3840),
                                                         (512, "phases", 256, 4, 3840)])
def test_race_full_size_3d27pt_128(nt, mode, block, stages, window):
    """The 128^3 stencil at full size; the first case is the benchmark's
    configuration (N_t 256, 2 stages, 512 threads, window 4064, dataflow,
    shared atomics)."""
    m = matgen.config_3d_128()
    print(f"case 3d27pt_128 n_workers={nt} mode={mode} block={block} stages={stages} window={window}: n={m.n} "
          f"nnz={m.nnz}", flush=True)
    x = matgen.rhs(m.n, 2)
    y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x)
    y, st = run_race(m, x, n_workers=nt, exec_mode=mode, block_threads=block, window_max=window, shared_atomics=True,
                     max_stages=stages)
    _check(y, y_ref, O.abs_product(m.n, m.row_ptr, m.col, m.val, x), _full_row_len(m), f"3d27pt_128 nt={nt}")
    rows = np.random.default_rng(0).choice(m.n, size=200, replace=False)
    exact = _sampled_rows_exact(m, x, rows)
    assert np.all(np.abs(y[rows] - exact) <= 1e-12 * np.max(np.abs(y_ref)))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("value_type,path", [("f64", "race"), ("f32", "race"), ("f64", "auto"), ("f32", "auto")])
def test_race_full_size_banded_4m(value_type, path):
    """Irregular banded N = 4M: FP64 values within the FP64 bound; FP32 values
    (promoted, FP64 accumulation) against the oracle on the same FP32-rounded
    values, and their error against the FP64 matrix stated.  With
    low_locality=auto the schedule predicts no window reuse here and the
    product runs as a CRS product of the expanded permuted matrix."""
    m = matgen.config_banded_4m()
    print(f"case banded_4m {value_type} {path}: n={m.n} nnz={m.nnz}", flush=True)
    x = matgen.rhs(m.n, 3)
    vals = m.val if value_type == "f64" else m.val.astype(np.float32).astype(np.float64)
    y, st = run_race(m, x, n_workers=1024, value_type=value_type, low_locality=path)
    print(f"  units={st['n_units']} leaves={st['n_leaves']} eta={st['eta']:.3f} shared={st['shared_touches']} "
          f"zeroed={st['n_zeroed']} product_path={st['product_path']}", flush=True)
    assert st["product_path"] == (1 if path == "auto" else 0)
    y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, vals, x)
    _check(y, y_ref, O.abs_product(m.n, m.row_ptr, m.col, vals, x), _full_row_len(m), f"banded_4m {value_type}")
    if value_type == "f32":
        y64 = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x)
        rel = np.linalg.norm(y - y64) / np.linalg.norm(y64)
        print(f"  FP32-value error vs the FP64 matrix: {rel:.3e} (unit roundoff of FP32 {2.0 ** -24:.3e})", flush=True)
        assert rel < 2.0 ** -20


@pytest.mark.parametrize("k", [5, 9])
def test_batch_tiled_replays(k):
    """A batch whose windows cannot hold all k columns runs in passes (k = 9:
    five passes, through contiguous column tiles); graph replays stay
    correct."""
    mats = _batch_mats()
    scheds = [R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=max(4, m.n // 500)) for m in mats]
    batch = R.Batch(scheds, k)
    xs = [torch.empty((m.n, k), dtype=torch.float64, device=DEV) for m in mats]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    batch.bind(xs, ys)
    gen = torch.Generator(device=DEV)
    gen.manual_seed(77)
    for rep in range(3):
        for x in xs:
            x.uniform_(-1.0, 1.0, generator=gen)
        for y in ys:
            y.fill_(float("nan"))
        batch.run(use_graph=(rep != 1))
        torch.cuda.synchronize()
        batch.check()
        for m, s, x, y in zip(mats, scheds, xs, ys):
            perm = s.perm()
            xp = x.cpu().numpy()
            x_orig = np.empty_like(xp)
            x_orig[perm] = xp
            y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x_orig)[perm]
            absax = O.abs_product(m.n, m.row_ptr, m.col, m.val, np.abs(x_orig))[perm]
            yh = y.cpu().numpy()
            for j in range(k):
                _check(yh[:, j], y_ref[:, j], absax[:, j], _full_row_len(m), f"batch tiled rep={rep} {m.name} col={j}")
    batch.close()
    for s in scheds:
        s.close()


def _batch_mats():
    return [matgen.stencil2d_5pt(40, seed=51), matgen.stencil3d_27pt(14, seed=52),
            matgen.banded_irregular(6000, seed=53, band=600), matgen.stencil2d_5pt(23, seed=54),
            matgen.random_symmetric(300, 0.02, seed=55), matgen.stencil3d_27pt(9, seed=56)]


@pytest.mark.parametrize("k,low_locality,value_type", [
    (1, "race", "f64"), (4, "race", "f64"), (16, "race", "f64"), (1, "auto", "f64"), (1, "expanded", "f64"),
    (4, "expanded", "f64"), (4, "auto", "f64"), (16, "auto", "f64"), (1, "auto", "f32"), (3, "expanded", "f32"),
    (16, "expanded", "f32")])
def test_batch_graph_replays(k, low_locality, value_type):
    """Graph replays and direct launches of a small batch against the oracle.
    Members whose product is the expanded CRS product (all of them with
    "expanded", the banded one with "auto") take no tickets: with k = 1 they
    run the batched row-block launch, with k > 1 a CRS SpMM each.  FP32
    values are checked against the oracle on the same rounded values."""
    mats = _batch_mats()
    window = min(3840, (159 * 1024) // (16 * k + 4) - 16)  # x, y windows of k doubles + the index, per entry
    scheds = [R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=max(4, m.n // 500), window_max=window,
                         low_locality=low_locality, value_type=value_type) for m in mats]
    paths = [sc.stats()["product_path"] for sc in scheds]
    if low_locality == "expanded":
        assert all(p == 1 for p in paths)
    batch = R.Batch(scheds, k)
    info = batch.info()
    print(f"batch k={k} low_locality={low_locality} paths={paths}: {info}", flush=True)
    if low_locality == "expanded":
        assert info["n_tickets"] == 0  # every member runs outside the persistent launch
    gen = torch.Generator(device=DEV)
    gen.manual_seed(7 + k)
    xs = [torch.empty((m.n, k) if k > 1 else (m.n,), dtype=torch.float64, device=DEV) for m in mats]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    batch.bind(xs, ys)
    for rep in range(3):
        for x in xs:  # eager work between replays: new right-hand sides
            x.uniform_(-1.0, 1.0, generator=gen)
        for y in ys:
            y.fill_(float("nan"))
        batch.run(use_graph=(rep != 1))
        torch.cuda.synchronize()
        batch.check()
        for m, s, x, y in zip(mats, scheds, xs, ys):
            perm = s.perm()
            xp = x.cpu().numpy()
            x_orig = np.empty_like(xp)
            x_orig[perm] = xp
            vals = m.val if value_type == "f64" else m.val.astype(np.float32).astype(np.float64)
            y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, vals, x_orig)[perm]
            absax = O.abs_product(m.n, m.row_ptr, m.col, vals, np.abs(x_orig))[perm]
            yh = y.cpu().numpy()
            for j in range(k):
                sl = (slice(None), j) if k > 1 else slice(None)
                _check(yh[sl], y_ref[sl], absax[sl], _full_row_len(m), f"batch k={k} rep={rep} {m.name} col={j}")
    batch.close()
    for s in scheds:
        s.close()


def test_traced_product_stamps():
    m = matgen.stencil3d_27pt(20, seed=61)
    x = matgen.rhs(m.n, 61)
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=64)
    st = s.stats()
    xd = torch.as_tensor(x, device=DEV)
    xp = torch.empty_like(xd)
    s.permute(xd, xp, True)
    yp = torch.full_like(xd, float("nan"))
    tr = torch.zeros(4 * st["n_units"], dtype=torch.int64, device=DEV)
    s.traced(xp, yp, tr)
    torch.cuda.synchronize()
    s.check()
    t = tr.cpu().numpy().reshape(-1, 4)
    assert np.all(t[:, 0] > 0)
    assert np.all(np.diff(t, axis=1) >= 0)
    y = torch.empty_like(xd)
    s.permute(yp, y, False)
    y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x)
    _check(y.cpu().numpy(), y_ref, O.abs_product(m.n, m.row_ptr, m.col, m.val, x), _full_row_len(m), "traced")
    s.close()


@pytest.mark.parametrize("stride,shared", [(2, True), (5, False)])
def test_flow_late_workgroups_taken_over(stride, shared):
    """Workgroups forced from the host to join about 0.2 ms late claim
    nothing at start: running workgroups that wait for their static tickets,
    or that are free, claim and run them.  The product is the same and the
    takeovers are counted; with the forcing off again the next product is
    correct too."""
    m = matgen.stencil3d_27pt(40, seed=71)
    x = matgen.rhs(m.n, 71)
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=64, window_max=512, shared_atomics=shared)
    try:
        y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x)
        absax = O.abs_product(m.n, m.row_ptr, m.col, m.val, x)
        xd = torch.as_tensor(x, device=DEV)
        xp = torch.empty_like(xd)
        s.permute(xd, xp, True)
        before = s.takeovers()
        for late in (stride, 0):
            print(f"case late stride={late} shared={shared}: n={m.n} units={s.stats()['n_units']}", flush=True)
            s.test_late(late)
            yp = torch.full_like(xd, float("nan"))
            s.spmv(xp, yp)
            y = torch.empty_like(xd)
            s.permute(yp, y, False)
            torch.cuda.synchronize()
            s.check()
            _check(y.cpu().numpy(), y_ref, absax, _full_row_len(m), f"late{late}")
            if late:
                taken = s.takeovers() - before
                print(f"  takeovers {taken}", flush=True)
                assert taken > 0
    finally:
        s.close()


COMPLEX = [
    ("3d27pt_24", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=256, window_max=2176)),
    ("3d27pt_24_w3840", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=256, block_threads=512)),
    ("banded_40k", lambda: matgen.banded_irregular(40000, seed=6, band=4000), dict(n_workers=256, window_max=2176)),
    ("banded_40k_w96", lambda: matgen.banded_irregular(40000, seed=6, band=4000), dict(n_workers=16, window_max=96)),
    ("rand_islands", lambda: matgen.random_symmetric(500, 0.003, seed=8), dict(n_workers=16)),
    ("rand_nodiag", lambda: matgen.random_symmetric(300, 0.02, seed=9, with_diag=False), dict(n_workers=12)),
]


@pytest.mark.parametrize("hermitian", [False, True], ids=["symmetric", "hermitian"])
@pytest.mark.parametrize("name,make,params", COMPLEX, ids=[c[0] for c in COMPLEX])
def test_race_complex(name, make, params, hermitian):
    """Complex symmetric and Hermitian matrices against the complex oracle:
    normwise within 1e-12, componentwise within the summation bound of
    |A||x| (a complex product adds two real products per part)."""
    m = make()
    rng = np.random.default_rng(77)
    vals = m.val * (1 + 0.5j) + 1j * rng.standard_normal(m.nnz)
    x = rng.standard_normal(m.n) + 1j * rng.standard_normal(m.n)
    print(f"case complex {name} hermitian={hermitian}: n={m.n} nnz={m.nnz} {params}", flush=True)
    s = R.Schedule(m.n, m.row_ptr, m.col, vals, value_type="c128h" if hermitian else "c128", **params)
    try:
        xd = torch.as_tensor(x, device=DEV)
        xp = torch.empty_like(xd)
        yp = torch.full_like(xd, complex(float("nan"), float("nan")))
        y = torch.empty_like(xd)
        s.permute(xd, xp, to_permuted=True)
        s.spmv(xp, yp)
        s.permute(yp, y, to_permuted=False)
        torch.cuda.synchronize()
        s.check()
        got = y.cpu().numpy()
    finally:
        s.close()
    ref = O.symm_spmv_complex(m.n, m.row_ptr, m.col, vals, x, hermitian)
    scale = O.abs_product_complex(m.n, m.row_ptr, m.col, vals, x)
    err = np.abs(got - ref)
    en = float(err.max() / np.abs(ref).max())
    with np.errstate(divide="ignore", invalid="ignore"):
        ec = float(np.max(np.where(scale > 0, err / scale, 0.0)))
    bound = 4 * gamma(2 * (_full_row_len(m) + 1))
    print(f"[complex {name}] err_norm={en:.3e} err_comp={ec:.3e} (bound {bound:.3e})", flush=True)
    assert en <= 1e-12 and ec <= bound


def test_complex_unsupported_paths():
    m = matgen.stencil3d_27pt(8, seed=2)
    vc = m.val + 0.5j
    s = R.Schedule(m.n, m.row_ptr, m.col, vc, value_type="c128", n_workers=32, window_max=2176)
    try:
        X = torch.zeros(m.n, 3, dtype=torch.complex128, device=DEV)
        with pytest.raises(R.RaceError):
            s.spmm(X, torch.empty_like(X))
        with pytest.raises(R.RaceError):
            R.Batch([s], 1)
    finally:
        s.close()


def test_product_fuzz():
    """Seeded random matrices and parameters (window, workgroup size,
    execution mode, shared atomics, value type, right-hand sides) against the
    oracle, one case after another in this process."""
    for seed in range(40):
        rng = np.random.default_rng(500 + seed)
        kind = int(rng.integers(4))
        if kind == 0:
            m = matgen.random_symmetric(int(rng.integers(50, 1500)), float(rng.uniform(0.001, 0.01)), seed=seed,
                                        with_diag=bool(rng.integers(2)))
        elif kind == 1:
            m = matgen.stencil2d_5pt(int(rng.integers(8, 70)), seed=seed)
        elif kind == 2:
            m = matgen.stencil3d_27pt(int(rng.integers(4, 18)), seed=seed)
        else:
            n = int(rng.integers(500, 8000))
            m = matgen.banded_irregular(n, seed=seed, band=int(rng.integers(2, max(3, n // 8))))
        k = int(rng.choice([1, 1, 2, 3, 5]))
        vt = str(rng.choice(["f64", "f64", "f32"]))
        params = dict(n_workers=int(rng.choice([2, 8, 32, 128, 512])), window_max=int(rng.choice([96, 256, 1000, 3840])),
                      block_threads=int(rng.choice([64, 128, 256, 512, 1024])),
                      exec_mode=str(rng.choice(["flow", "flow", "phases"])), shared_atomics=bool(rng.integers(2)),
                      max_stages=int(rng.integers(1, 5)), value_type=vt)
        print(f"case fuzz seed={seed}: n={m.n} nnz={m.nnz} k={k} {params}", flush=True)
        vals = m.val if vt == "f64" else m.val.astype(np.float32).astype(np.float64)
        X = matgen.rhs(m.n, 900 + seed, k=k).reshape(m.n, k) if k > 1 else matgen.rhs(m.n, 900 + seed)
        Y, st = run_race(m, X, k=k, **params)
        Y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, vals, X)
        absax = O.abs_product(m.n, m.row_ptr, m.col, vals, np.abs(X))
        for j in range(k):
            sl = (slice(None), j) if k > 1 else slice(None)
            _check(Y[sl], Y_ref[sl], absax[sl], _full_row_len(m), f"fuzz seed={seed} col={j}")


@pytest.fixture(scope="module")
def batch64():
    """The 64 seeded matrices of the batch workload (10k..500k rows, 2D
    5-point / 3D 27-point / irregular banded), generated once."""
    return matgen.config_batch(64, 100)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("k", [1, 4, 16])
def test_batch_full_64(batch64, k):
    """The full 64-matrix batch of the benchmark for k = 1, 4, 16 in one
    graph replay, every matrix and column element-wise against the oracle
    (shapes: N_t of one worker per 4000 rows, the widest window holding all
    k columns, 512 threads; for k = 16 also the largest window in passes;
    for k = 1 also with low_locality "auto", the low-locality members on the
    batched row-block product)."""
    from paper_1907_06487_amd import autotune
    mats = batch64
    cases = [(autotune.max_window(k), "race")] + ([(3840, "race")] if k > 2 else []) + \
        ([(autotune.max_window(k), "auto")] if k == 1 else [])
    for window, low_locality in cases:
        print(f"case batch64 k={k} window={window} low_locality={low_locality}: {sum(m.n for m in mats)} rows",
              flush=True)
        scheds = [R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=int(min(4096, max(4, m.n // 4000))),
                             window_max=window, block_threads=512, low_locality=low_locality) for m in mats]
        batch = R.Batch(scheds, k, threads=512)
        print(f"  {sum(sc.stats()['product_path'] for sc in scheds)} members on the expanded product, "
              f"{batch.info()}", flush=True)
        gen = torch.Generator(device=DEV)
        gen.manual_seed(1000 + k)
        xs = [torch.rand((m.n, k) if k > 1 else (m.n,), dtype=torch.float64, device=DEV, generator=gen) * 2 - 1
              for m in mats]
        ys = [torch.full_like(x, float("nan")) for x in xs]
        batch.bind(xs, ys)
        batch.run(use_graph=True)
        torch.cuda.synchronize()
        batch.check()
        worst = 0.0
        for m, s, x, y in zip(mats, scheds, xs, ys):
            perm = s.perm()
            xp = x.cpu().numpy()
            x_orig = np.empty_like(xp)
            x_orig[perm] = xp
            y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x_orig)[perm]
            absax = O.abs_product(m.n, m.row_ptr, m.col, m.val, np.abs(x_orig))[perm]
            yh = y.cpu().numpy()
            mlen = _full_row_len(m)
            for j in range(k):
                sl = (slice(None), j) if k > 1 else slice(None)
                en, _ = _check(yh[sl], y_ref[sl], absax[sl], mlen, f"batch64 k={k} w={window} {m.name} col={j}")
                worst = max(worst, en)
        print(f"  batch64 k={k} window={window}: worst err_norm {worst:.3e}", flush=True)
        batch.close()
        for s in scheds:
            s.close()


def _arrow(n, seed):
    """Row 0 coupled to every row (a full row of n entries, longer than any
    row block), the diagonal, and a random sparse upper part."""
    rng = np.random.default_rng(seed)
    r = rng.integers(1, n, size=4 * n)
    c = rng.integers(1, n, size=4 * n)
    lo, hi = np.minimum(r, c), np.maximum(r, c)
    keys = np.unique(np.concatenate([np.arange(n) * n + np.arange(n), np.arange(1, n), lo * n + hi]))
    rows, cols = keys // n, keys % n
    return matgen._csr_from_sorted(n, rows, cols, rng.standard_normal(keys.shape[0]), f"arrow_{n}")


EXPANDED = [
    ("arrow_3000_expanded", lambda: _arrow(3000, 4), dict(n_workers=8, low_locality="expanded"), 1),
    ("banded_40k_w96_auto", lambda: matgen.banded_irregular(40000, seed=6, band=4000),
     dict(n_workers=16, window_max=96, low_locality="auto"), 1),
    ("3d27pt_24_auto", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=256, low_locality="auto"), 0),
    ("3d27pt_24_expanded", lambda: matgen.stencil3d_27pt(24, seed=5), dict(n_workers=256, low_locality="expanded"), 1),
    ("rand_nodiag_expanded", lambda: matgen.random_symmetric(300, 0.02, seed=9, with_diag=False),
     dict(n_workers=12, low_locality="expanded"), 1),
]


@pytest.mark.parametrize("value_type", ["f64", "f32"])
@pytest.mark.parametrize("name,make,params,path", EXPANDED, ids=[c[0] for c in EXPANDED])
def test_expanded_product_path(name, make, params, path, value_type):
    """Products of schedules that switch to the expanded CRS product (and of
    those that do not) against the oracle, through race_symm_spmv and
    race_symm_spmv_noalloc, and SymmSpMM with 2, 3, 5 and 16 columns (the
    expanded CRS SpMM on expanded schedules)."""
    m = make()
    vals = m.val if value_type == "f64" else m.val.astype(np.float32).astype(np.float64)
    x = matgen.rhs(m.n, 41)
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, value_type=value_type, **params)
    try:
        st = s.stats()
        print(f"case {name} {value_type}: n={m.n} product_path={st['product_path']} per_thread={st['expanded_per_thread']}",
              flush=True)
        assert st["product_path"] == path
        perm = s.perm()
        y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, vals, x)[perm]
        absax = O.abs_product(m.n, m.row_ptr, m.col, vals, x)[perm]
        xd = torch.as_tensor(x, device=DEV)
        xp = torch.empty_like(xd)
        s.permute(xd, xp, True)
        for entry in ("spmv", "noalloc"):
            yp = torch.full_like(xp, float("nan"))
            (s.spmv if entry == "spmv" else s.spmv_noalloc)(xp, yp)
            torch.cuda.synchronize()
            s.check()
            _check(yp.cpu().numpy(), y_ref, absax, _full_row_len(m), f"{name} {value_type} {entry}")
        for k in (2, 3, 5, 16):  # lane groups of 2, 4 (one idle lane), 8 (three idle) and 16 columns
            fs = [(j + 1.0) * (-1.0) ** j for j in range(k)]
            X = torch.stack([f * xp for f in fs], dim=1).contiguous()
            Y = torch.full_like(X, float("nan"))
            s.spmm(X, Y)
            torch.cuda.synchronize()
            s.check()
            for j, f in enumerate(fs):
                _check(Y[:, j].cpu().numpy(), f * y_ref, abs(f) * absax, _full_row_len(m), f"{name} spmm k={k} col {j}")
    finally:
        s.close()
