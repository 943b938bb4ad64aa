"""Roofline model of Section 3 -- test infrastructure only.

* Eq. (upper_performance): P = I * b_S.
* Eq. (SpMV_intensity): I_SpMV(alpha) = 2 / (8 + 4 + 8 alpha + 20 / N_nzr)
  flop/byte (8-byte values, 4-byte indices; x traffic 8 alpha per nonzero,
  row pointer + LHS 20 bytes per row).
* Eq. (SymmSpMV_intensity): I_SymmSpMV(alpha) = 4 / (8 + 4 + 24 alpha +
  4 / N_nzr^symm) with Eq. (NNZR_symm): N_nzr^symm = (N_nzr - 1)/2 + 1
  (x read plus y read and written through the indirect updates: 24 alpha).
* alpha from a measured traffic per nonzero: the SpMV denominator solved for
  alpha (Section 3.3).
"""
from __future__ import annotations


def nnzr_symm(nnzr: float) -> float:
    return (nnzr - 1.0) / 2.0 + 1.0


def intensity_spmv(alpha: float, nnzr: float) -> float:
    return 2.0 / (8.0 + 4.0 + 8.0 * alpha + 20.0 / nnzr)


def intensity_symmspmv(alpha: float, nnzr: float) -> float:
    """``nnzr`` is the full matrix's nonzeros per row; N_nzr^symm follows."""
    return 4.0 / (8.0 + 4.0 + 24.0 * alpha + 4.0 / nnzr_symm(nnzr))


def performance(intensity: float, bandwidth: float) -> float:
    return intensity * bandwidth


def alpha_from_traffic(bytes_per_nnz: float, nnzr: float) -> float:
    """Solve 8 + 4 + 8 alpha + 20 / N_nzr = bytes_per_nnz for alpha."""
    return (bytes_per_nnz - 12.0 - 20.0 / nnzr) / 8.0


def optimal_alpha_spmv(nnzr: float) -> float:
    """x loaded once: alpha = 1 / N_nzr."""
    return 1.0 / nnzr


def optimal_alpha_symmspmv(nnzr: float) -> float:
    return 1.0 / nnzr_symm(nnzr)
