"""race_symm_spmv_noalloc: the dataflow product with its state in the
library's fixed per-device array instead of device memory the schedule
allocates.  Checked against race_symm_spmv on the same schedules (and both
against the oracle) on two calls in a row, the second on a smaller matrix;
its refusal of a schedule whose state exceeds the array; and replays of a
captured graph of it, with eager work between the replays."""
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


def _setup(m, seed, **params):
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, **params)
    x = matgen.rhs(m.n, seed)
    xd = torch.as_tensor(x, device=DEV)
    xp = torch.empty_like(xd)
    s.permute(xd, xp, to_permuted=True)
    perm = s.perm()
    y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x)[perm]
    absax = O.abs_product(m.n, m.row_ptr, m.col, m.val, x)[perm]
    return s, xp, y_ref, absax


def test_noalloc_matches_existing_entry_two_calls():
    big = matgen.stencil3d_27pt(40, seed=81)
    small = matgen.banded_irregular(9000, seed=82, band=900)
    cases = [(big, 81, dict(n_workers=256, block_threads=512)),
             (small, 82, dict(n_workers=64, window_max=256))]  # shared entries and clearing tasks
    setups = [_setup(m, seed, **p) for m, seed, p in cases]
    try:
        outs = []
        # two calls in a row through the entry point that allocates nothing,
        # the second with a smaller input
        for (m, _, p), (s, xp, _, _) in zip(cases, setups):
            print(f"case noalloc n={m.n} units={s.stats()['n_units']} {p}", flush=True)
            y = torch.full_like(xp, float("nan"))
            s.spmv_noalloc(xp, y)
            outs.append(y)
        torch.cuda.synchronize()
        for (m, _, p), (s, xp, y_ref, absax), y in zip(cases, setups, outs):
            s.check()
            y_old = torch.full_like(xp, float("nan"))
            s.spmv(xp, y_old)
            torch.cuda.synchronize()
            s.check()
            a, b = y.cpu().numpy(), y_old.cpu().numpy()
            # the same kernel on the same schedule: only the order of shared atomic adds may differ
            assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
            _check(a, y_ref, absax, _full_row_len(m), f"noalloc n={m.n}")
            _check(b, y_ref, absax, _full_row_len(m), f"spmv n={m.n}")
    finally:
        for s, *_ in setups:
            s.close()


def test_noalloc_refuses_state_beyond_the_array():
    # a tridiagonal matrix with two-entry windows: one unit per row, more
    # completion flags than the array holds
    n = (1 << 20) + 1000
    rp = np.arange(0, 2 * n, 2, dtype=np.int32)
    rp = np.append(rp, 2 * n - 1).astype(np.int32)
    col = np.empty(2 * n - 1, dtype=np.int32)
    col[0::2] = np.arange(n)
    col[1::2] = np.arange(1, n)
    val = np.ones(2 * n - 1)
    val[0::2] = 4.0
    s = R.Schedule(n, rp, col, val, n_workers=4, window_max=2, max_stages=1)
    try:
        print(f"case noalloc oversized: units={s.stats()['n_units']}", flush=True)
        x = torch.zeros(n, dtype=torch.float64, device=DEV)
        y = torch.zeros_like(x)
        with pytest.raises(R.RaceError) as ei:
            s.spmv_noalloc(x, y)
        assert ei.value.code == -4
    finally:
        s.close()


def test_noalloc_graph_replays():
    m = matgen.stencil3d_27pt(30, seed=83)
    s, xp, y_ref, absax = _setup(m, 83, n_workers=128, window_max=512)
    try:
        y = torch.full_like(xp, float("nan"))
        s.spmv_noalloc(xp, y)  # eager first: kernel attributes and the array address outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side, capture_error_mode="thread_local"):
                s.spmv_noalloc(xp, y, stream=side)
        torch.cuda.synchronize()
        for rep in range(4):
            y.fill_(float("nan"))  # eager work between the replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            s.check()
            _check(y.cpu().numpy(), y_ref, absax, _full_row_len(m), f"noalloc graph replay {rep}")
    finally:
        s.close()
