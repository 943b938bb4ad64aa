"""Schedule-shape autotuner.

Picks, per matrix and number of right-hand sides k, the RACE worker count
(N_t, Section 5), the unit window and the workgroup size by timing candidate
schedules on the device (HIP events around the library's own product
calls).  For k > 2 it also weighs the right-hand-side tile: windows that
hold all k columns in one pass (small, so little reuse) against the largest
window taken in passes of the widest tile that fits (the matrix re-read
per pass).  A batch needs one workgroup size for all matrices; `tune_batch`
chooses it, and the window mode, by timing the whole batch.
"""
from __future__ import annotations

import torch

from . import Batch, Schedule


def max_window(k: int) -> int:
    """Largest unit window whose LDS (x and y windows of k doubles plus a
    4-byte index per entry) fits a 159 KiB workgroup allocation."""
    return min(3840, (159 * 1024) // (16 * k + 4) - 16)


def candidates(n: int, k: int, block: int, window: int = 0, low_locality: str = "race"):
    """Worker counts of 8000, 4000 and 2000 rows per worker at the given
    window (0: the largest that holds all k columns).  With low_locality
    "auto" and four or more right-hand sides the expanded CRS product is one
    more candidate, so the choice between it and the RACE kernels is
    measured per matrix: from four columns on, a full-matrix CRS SpMM can
    beat passes of RACE windows even where the windows have reuse.  With one
    or two columns the schedule's own prediction decides; a matrix timed
    alone there favours the expanded product more than the same matrix in a
    batch, where the RACE members share one persistent launch."""
    wm = window or max_window(k)
    nts = sorted({int(min(4096, max(4, n // r))) for r in (8000, 4000, 2000)})
    out = [dict(n_workers=nt, window_max=wm, block_threads=block, low_locality=low_locality) for nt in nts]
    if low_locality == "auto" and k >= 4:
        out.append(dict(n_workers=nts[len(nts) // 2], window_max=wm, block_threads=block, low_locality="expanded"))
    return out


def _time(fn, reps):
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_matrix(m, k: int, block: int, reps: int = 5, device: str = "cuda:0", window: int = 0,
                low_locality: str = "race"):
    """Best shape for one matrix: returns (params, ms, all results)."""
    shape = (m.n, k) if k > 1 else (m.n,)
    x = torch.rand(shape, dtype=torch.float64, device=device)
    y = torch.empty_like(x)
    results = []
    for c in candidates(m.n, k, block, window, low_locality):
        s = Schedule(m.n, m.row_ptr, m.col, m.val, **c)
        ms = _time(lambda: s.spmm(x, y) if k > 1 else s.spmv(x, y), reps)
        s.close()
        results.append((ms, c))
    results.sort(key=lambda r: r[0])
    return results[0][1], results[0][0], results


def tune_batch(mats, k: int, blocks=(256, 512, 1024), reps: int = 5, device: str = "cuda:0", log=None,
               low_locality: str = "race"):
    """Per-matrix shapes (timed at 512 threads) for each window mode, then the
    mode and workgroup size whose whole batch replay runs fastest.  Returns
    (schedules, batch, chosen).  low_locality as for Schedule ("auto": with
    k = 1 the matrices without window reuse run the row-block CRS product)."""
    modes = [0] if max_window(k) >= 3840 else [0, 3840]  # one pass of k columns; or the largest window, tiled
    xs = [torch.rand((m.n, k) if k > 1 else (m.n,), dtype=torch.float64, device=device) for m in mats]
    ys = [torch.empty_like(x) for x in xs]
    best = None
    for window in modes:
        params = []
        for i, m in enumerate(mats):
            params.append(tune_matrix(m, k, 512, reps=3, device=device, window=window, low_locality=low_locality)[0])
            if log and i % 16 == 15:
                log(f"autotune k={k} window {window or max_window(k)}: {i + 1}/{len(mats)} matrices")
        scheds = [Schedule(m.n, m.row_ptr, m.col, m.val, **p) for m, p in zip(mats, params)]
        for blk in blocks:
            batch = Batch(scheds, k, threads=blk)
            batch.bind(xs, ys)
            ms = _time(lambda: batch.run(use_graph=True), reps)
            if best is None or ms < best[0]:
                if best is not None:
                    best[1].close()
                    if best[2] is not scheds:
                        for sc in best[2]:
                            sc.close()
                best = (ms, batch, scheds, params, blk)
            else:
                batch.close()
        if best[2] is not scheds:
            for sc in scheds:
                sc.close()
    ms, batch, scheds, params, blk = best
    return scheds, batch, {"block_threads": blk, "params": params, "ms": ms}
