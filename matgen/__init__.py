"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module only *makes* inputs: symmetric sparse matrices stored as the upper
triangle in CRS (int32 row pointers and columns, float64 values, columns
ascending inside a row so the diagonal comes first when present) and dense
right-hand sides.  It holds none of the SymmSpMV or RACE arithmetic.

Families (the paper's benchmark suite is replaced by these stand-ins):

* ``stencil2d_5pt(n, seed)`` -- 2D 5-point Laplacian on an n x n grid,
  lexicographic order; diagonal 4.0, each symmetric off-diagonal pair
  -1 + U[-0.1, 0.1], drawn in upper-CRS order.
* ``stencil3d_27pt(n, seed)`` -- 3D 27-point stencil on an n^3 grid,
  lexicographic order (x fastest); off-diagonal pairs U[-1, 1] drawn in
  upper-CRS order; diagonal = 27 + absolute row sum of the full row.
* ``banded_irregular(n, seed, band=2**16)`` -- irregular banded matrix: in
  band order row i draws d_i = min(Geometric(1/13), 64) upper offsets
  uniform in {1..band}; entries past n are dropped, duplicates merged, the
  diagonal is always present, every stored value is N(0, 1); the rows are
  then relabelled by a seeded random permutation applied symmetrically.
* ``stencil2d_7pt(n)`` -- the small artificial 2D stencil used to walk through
  the method (axis neighbours plus the (+1,-1)/(-1,+1) diagonal), values 1.

Random streams: ``numpy.random.Generator(PCG64(seed))`` with a fixed draw
order per family; right-hand sides use seed + 1_000_000.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

X_SEED_OFFSET = 1_000_000


@dataclass
class UpperCSR:
    """Upper triangle (diagonal included) of a symmetric matrix in CRS."""

    n: int
    row_ptr: np.ndarray  # int32, n+1
    col: np.ndarray      # int32, nnz
    val: np.ndarray      # float64, nnz
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _csr_from_sorted(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray, name: str) -> UpperCSR:
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32")
    return UpperCSR(n, row_ptr.astype(np.int32), cols.astype(np.int32), np.ascontiguousarray(vals, dtype=np.float64), name)


def _stencil_upper(dims: tuple[int, ...], offsets: list[tuple[int, ...]]):
    """Rows/cols (lexicographic, last axis fastest) of the upper part of a stencil
    pattern; ``offsets`` must be the strictly-upper offsets in ascending column
    order.  Returns (rows, cols) sorted by (row, col) with the diagonal first."""
    n = int(np.prod(dims))
    coords = np.indices(dims).reshape(len(dims), -1)  # axis 0 slowest
    strides = [int(np.prod(dims[i + 1:])) for i in range(len(dims))]
    k = len(offsets) + 1
    cols = np.full((n, k), -1, dtype=np.int64)
    idx = np.arange(n, dtype=np.int64)
    cols[:, 0] = idx
    for j, off in enumerate(offsets, start=1):
        ok = np.ones(n, dtype=bool)
        delta = 0
        for ax, o in enumerate(off):
            c = coords[ax] + o
            ok &= (c >= 0) & (c < dims[ax])
            delta += o * strides[ax]
        cols[ok, j] = idx[ok] + delta
    mask = cols >= 0
    rows = np.broadcast_to(idx[:, None], cols.shape)[mask]
    return n, rows, cols[mask]


def stencil2d_5pt(side: int, seed: int = 1) -> UpperCSR:
    """2D 5-point Laplacian, lexicographic (j fastest)."""
    # upper offsets in ascending column order: (0,+1) then (+1,0)
    n, rows, cols = _stencil_upper((side, side), [(0, 1), (1, 0)])
    rng = _rng(seed)
    off = rows != cols
    vals = np.empty(rows.shape[0], dtype=np.float64)
    vals[~off] = 4.0
    vals[off] = -1.0 + rng.uniform(-0.1, 0.1, size=int(off.sum()))
    return _csr_from_sorted(n, rows, cols, vals, f"2d5pt_{side}")


def _upper_offsets_27pt():
    offs = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dz, dy, dx) > (0, 0, 0):
                    offs.append((dz, dy, dx))
    return sorted(offs)  # lexicographic == ascending column offset


def stencil3d_27pt(side: int, seed: int = 2) -> UpperCSR:
    """3D 27-point stencil, lexicographic order (x fastest)."""
    n, rows, cols = _stencil_upper((side, side, side), _upper_offsets_27pt())
    rng = _rng(seed)
    off = rows != cols
    vals = np.empty(rows.shape[0], dtype=np.float64)
    offv = rng.uniform(-1.0, 1.0, size=int(off.sum()))
    vals[off] = offv
    a = np.abs(offv)
    rowsum = np.bincount(rows[off], weights=a, minlength=n) + np.bincount(cols[off], weights=a, minlength=n)
    vals[~off] = 27.0 + rowsum
    return _csr_from_sorted(n, rows, cols, vals, f"3d27pt_{side}")


def stencil2d_7pt(side: int) -> UpperCSR:
    """Small artificial 2D stencil: axis neighbours plus the anti-diagonal pair
    (i+1, j-1)/(i-1, j+1); unit values.  From the corner (0, 0) its BFS levels
    are the anti-diagonals i + j."""
    # upper offsets ascending: (0,+1), (+1,-1), (+1,0)
    n, rows, cols = _stencil_upper((side, side), [(0, 1), (1, -1), (1, 0)])
    vals = np.ones(rows.shape[0], dtype=np.float64)
    return _csr_from_sorted(n, rows, cols, vals, f"2d7pt_{side}")


def banded_irregular(n: int, seed: int = 3, band: int = 2**16, mean_deg: float = 13.0, cap: int = 64) -> UpperCSR:
    rng = _rng(seed)
    deg = np.minimum(rng.geometric(1.0 / mean_deg, size=n), cap).astype(np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    offs = rng.integers(1, band + 1, size=src.shape[0], dtype=np.int64)
    dst = src + offs
    keep = dst < n
    src, dst = src[keep], dst[keep]
    key = np.unique(src * n + dst)  # merge duplicates, sorted by (src, dst)
    del src, dst
    diag = np.arange(n, dtype=np.int64)
    key = np.sort(np.concatenate([diag * n + diag, key]))  # (row, col) order, keys unique
    r, c = key // n, key % n
    del key
    vals = rng.standard_normal(r.shape[0])
    pi = rng.permutation(n).astype(np.int64)
    pr, pc = pi[r], pi[c]
    del r, c
    lo, hi = np.minimum(pr, pc), np.maximum(pr, pc)
    del pr, pc
    order = np.argsort(lo * n + hi)  # keys unique, so any sort is the same order
    return _csr_from_sorted(n, lo[order], hi[order], vals[order], f"banded_{n}")


def rhs(n: int, seed: int, k: int = 1) -> np.ndarray:
    """Right-hand side(s) uniform in [-1, 1]; shape (n,) or row-major (n, k)."""
    rng = _rng(seed + X_SEED_OFFSET)
    if k == 1:
        return rng.uniform(-1.0, 1.0, size=n)
    return rng.uniform(-1.0, 1.0, size=(n, k))


def random_symmetric(n: int, density: float, seed: int, with_diag: bool = True) -> UpperCSR:
    """Small random symmetric pattern (for property tests); values N(0, 1)."""
    rng = _rng(seed)
    m = rng.random((n, n)) < density
    m = np.triu(m, 1)
    if with_diag:
        m |= np.eye(n, dtype=bool)
    r, c = np.nonzero(m)
    vals = rng.standard_normal(r.shape[0])
    return _csr_from_sorted(n, r, c, vals, f"rand_{n}_{seed}")


# --- the named workloads --------------------------------------------------

def config_2d_small() -> UpperCSR:
    """2D 5-point Laplacian on a 100 x 100 grid (N = 10,000), seed 1."""
    return stencil2d_5pt(100, seed=1)


def config_3d_128() -> UpperCSR:
    """3D 27-point stencil on a 128^3 grid (N = 2,097,152), seed 2."""
    return stencil3d_27pt(128, seed=2)


def config_banded_4m() -> UpperCSR:
    """Irregular banded matrix with 2^22 rows, seed 3."""
    return banded_irregular(2**22, seed=3)


def relabel(m: UpperCSR, seed: int) -> UpperCSR:
    """The same symmetric matrix under a seeded random symmetric permutation
    (P A P^T): entry (i, j) moves to (p[i], p[j]), stored again as the upper
    triangle.  The input order then says nothing about the graph, as for a
    matrix with no bandwidth-reducing preordering."""
    p = _rng(seed).permutation(m.n).astype(np.int64)
    rows = np.repeat(np.arange(m.n, dtype=np.int64), np.diff(m.row_ptr))
    a, b = p[rows], p[m.col.astype(np.int64)]
    r, c = np.minimum(a, b), np.maximum(a, b)
    order = np.lexsort((c, r))
    return _csr_from_sorted(m.n, r[order], c[order], m.val[order], f"{m.name}_relabel{seed}")


def config_3d_128_relabel() -> UpperCSR:
    """The 128^3 27-point stencil (seed 2) under a random symmetric
    relabelling (seed 7): vertex 0 is an arbitrary grid point."""
    return relabel(config_3d_128(), 7)


def config_3d_160() -> UpperCSR:
    """3D 27-point stencil on a 160^3 grid (N = 4,096,000), seed 2000."""
    return stencil3d_27pt(160, seed=2000)


def batch_family(index: int, seed: int) -> UpperCSR:
    """One matrix of the uneven batch: size log-uniform in [1e4, 5e5] drawn
    from ``seed``; families cycle 2D 5-pt / 3D 27-pt / irregular banded."""
    rng = _rng(seed)
    target = int(round(math.exp(rng.uniform(math.log(1e4), math.log(5e5)))))
    fam = index % 3
    if fam == 0:
        return stencil2d_5pt(max(2, int(round(math.sqrt(target)))), seed=seed)
    if fam == 1:
        return stencil3d_27pt(max(2, int(round(target ** (1.0 / 3.0)))), seed=seed)
    return banded_irregular(target, seed=seed, band=max(1, min(2**16, target // 4)))


def config_batch(count: int = 64, first_seed: int = 100) -> list[UpperCSR]:
    return [batch_family(i, first_seed + i) for i in range(count)]


# --- format conversions for the yardsticks --------------------------------
# (input preparation only: the same matrix in other storage, for the
# baselines that need it)

def full_crs(m: UpperCSR):
    """The full symmetric matrix of ``m`` (both triangles, columns
    ascending) as int32 row pointers, int32 columns and float64 values: the
    storage a plain CRS SpMV reads."""
    rows = np.repeat(np.arange(m.n, dtype=np.int64), np.diff(m.row_ptr))
    cols = m.col.astype(np.int64)
    off = rows != cols
    r = np.concatenate([rows, cols[off]])
    c = np.concatenate([cols, rows[off]])
    v = np.concatenate([m.val, m.val[off]])
    order = np.argsort(r * m.n + c, kind="stable")
    rp = np.zeros(m.n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=m.n), out=rp[1:])
    return rp.astype(np.int32), c[order].astype(np.int32), np.ascontiguousarray(v[order])


def permuted(m: UpperCSR, new2old: np.ndarray) -> UpperCSR:
    """The upper triangle of P A P^T, where row i of the result is row
    new2old[i] of ``m`` (columns ascending)."""
    inv = np.empty(m.n, dtype=np.int64)
    inv[np.asarray(new2old, dtype=np.int64)] = np.arange(m.n, dtype=np.int64)
    rows = inv[np.repeat(np.arange(m.n, dtype=np.int64), np.diff(m.row_ptr))]
    cols = inv[m.col.astype(np.int64)]
    lo, hi = np.minimum(rows, cols), np.maximum(rows, cols)
    order = np.argsort(lo * m.n + hi, kind="stable")
    return _csr_from_sorted(m.n, lo[order], hi[order], m.val[order], f"{m.name}_permuted")
