/*
 * Serial Gauss-Seidel sweep oracle -- test infrastructure only.
 *
 * Plain C rendering of one Gauss-Seidel sweep over a given row order for a
 * symmetric matrix stored as its upper triangle in CRS (Section 3.2
 * storage): row i takes x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii with the
 * newest x.  The full rows are assembled first (off-diagonal columns
 * ascending, as in the Python oracle), so the sum runs in the same order as
 * there.  Built with -O2 -ffp-contract=off.
 */
#include <stdint.h>
#include <stdlib.h>

int oracle_gs_sweep(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val, const double* b,
                    double* x, const int32_t* order, int32_t n_order) {
  /* full off-diagonal rows: counts, then fill by ascending source row, which
     leaves every row's columns ascending (lower part first, then upper) */
  int64_t* fp = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  double* diag = (double*)calloc((size_t)n > 0 ? (size_t)n : 1, sizeof(double));
  if (!fp || !diag) {
    free(fp);
    free(diag);
    return 1;
  }
  for (int32_t r = 0; r < n; ++r)
    for (int32_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k)
      if (col[k] != r) {
        fp[r + 1]++;
        fp[col[k] + 1]++;
      }
  for (int32_t r = 0; r < n; ++r) fp[r + 1] += fp[r];
  int32_t* fc = (int32_t*)malloc((size_t)(fp[n] > 0 ? fp[n] : 1) * sizeof(int32_t));
  double* fv = (double*)malloc((size_t)(fp[n] > 0 ? fp[n] : 1) * sizeof(double));
  int64_t* fill = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!fc || !fv || !fill) {
    free(fp);
    free(diag);
    free(fc);
    free(fv);
    free(fill);
    return 1;
  }
  for (int32_t r = 0; r <= n; ++r) fill[r] = fp[r];
  /* lower part of row c: entries (r, c) stored in rows r < c, by ascending r */
  for (int32_t r = 0; r < n; ++r)
    for (int32_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
      const int32_t c = col[k];
      if (c == r) {
        diag[r] = val[k];
      } else {
        fc[fill[c]] = r;
        fv[fill[c]] = val[k];
        fill[c]++;
      }
    }
  /* upper part of row r after its lower part */
  for (int32_t r = 0; r < n; ++r)
    for (int32_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k)
      if (col[k] != r) {
        fc[fill[r]] = col[k];
        fv[fill[r]] = val[k];
        fill[r]++;
      }
  for (int32_t t = 0; t < n_order; ++t) {
    const int32_t i = order[t];
    double s = 0.0;
    for (int64_t k = fp[i]; k < fp[i + 1]; ++k) s += fv[k] * x[fc[k]];
    x[i] = (b[i] - s) / diag[i];
  }
  free(fp);
  free(diag);
  free(fc);
  free(fv);
  free(fill);
  return 0;
}
