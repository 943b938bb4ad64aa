"""GPU tests of the yardsticks and measurement kernels: rocSPARSE's SpMV
(full matrix and its own symmetric product), the attainable-bandwidth read
and copy kernels, and the refusal of stream capture for the dataflow
product (its epoch is a launch argument, so a replayed graph would run no
unit)."""
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


@pytest.mark.parametrize("symmetric", [False, True], ids=["general", "symmetric"])
@pytest.mark.parametrize("alg", ["adaptive", "rowsplit", "lrb"])
def test_vendor_spmv(alg, symmetric):
    m = matgen.banded_irregular(30000, seed=14, band=3000)
    x = matgen.rhs(m.n, 14)
    y_ref = O.symm_spmv(m.n, m.row_ptr, m.col, m.val, x)
    if symmetric:
        rp, c, v = m.row_ptr, m.col, m.val
    else:
        rp, c, v = O.expand_full(m.n, m.row_ptr, m.col, m.val)
    print(f"case vendor alg={alg} symmetric={symmetric}: n={m.n}", flush=True)
    try:
        h = R.race_vendor_create(m.n, rp, c, v, symmetric, alg)
    except R.RaceError as e:
        if symmetric and e.code == -4 and alg != "adaptive":
            pytest.skip(f"rocSPARSE does not implement the symmetric product with {alg}: {e}")
        raise
    try:
        xd = torch.as_tensor(x, device=DEV)
        for rep in range(2):  # the second call reuses the analysis
            yd = torch.full_like(xd, float("nan"))
            R.race_vendor_spmv(h, xd, yd)
            torch.cuda.synchronize()
            _check(yd.cpu().numpy(), y_ref, O.abs_product(m.n, m.row_ptr, m.col, m.val, x), _full_row_len(m),
                   f"vendor {alg} symmetric={symmetric} rep={rep}")
    finally:
        R.race_vendor_destroy(h)


def test_stream_copy_and_read():
    n = (64 << 20) // 8 + 6  # not a multiple of the grid stride: a ragged tail
    src = torch.arange(n, dtype=torch.float64, device=DEV)
    dst = torch.full_like(src, -1.0)
    sink = torch.zeros(4, dtype=torch.int32, device=DEV)
    for grid in (1, 37, 2048):
        dst.fill_(-1.0)
        R.race_stream_copy(src, dst, grid)
        R.race_stream_read(src, sink, grid)
        torch.cuda.synchronize()
        assert torch.equal(src, dst), grid
    with pytest.raises(R.RaceError):  # a length that is not a multiple of 16 bytes
        R.race_stream_copy(src[:3], dst[:3], 8)


def test_dataflow_product_refuses_capture():
    m = matgen.stencil3d_27pt(12, seed=3)
    s = R.Schedule(m.n, m.row_ptr, m.col, m.val, n_workers=32)
    try:
        x = torch.rand(m.n, dtype=torch.float64, device=DEV)
        y = torch.empty_like(x)
        s.spmv(x, y)  # eager first: kernel attributes set outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side, capture_error_mode="thread_local"):
                with pytest.raises(R.RaceError) as ei:
                    s.spmv(x, y)
                y.add_(1.0)  # the capture itself stays valid
        assert ei.value.code == -4
        torch.cuda.synchronize()
    finally:
        s.close()
