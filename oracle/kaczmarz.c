/*
 * Serial Kaczmarz sweep oracle -- test infrastructure only.
 *
 * Plain C rendering of one Kaczmarz sweep over a given row order for a
 * symmetric matrix stored as its upper triangle in CRS (Section 3.2
 * storage): row i (the full row, diagonal included) takes
 *     x <- x + omega (b_i - a_i . x) / |a_i|^2  a_i
 * with the newest x; a row with no stored value is skipped.  The full rows
 * are assembled with columns ascending and the diagonal in its place, as in
 * the Python oracle, so the dot product and the norm are summed in the same
 * order.  Built with -O2 -ffp-contract=off.
 */
#include <stdint.h>
#include <stdlib.h>

int oracle_kacz_sweep(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val, const double* b,
                      double* x, const int32_t* order, int32_t n_order, double omega) {
  /* full rows: counts, then fill by ascending source row; the entries of
     row c stored in rows r < c come first (ascending r), then the row's own
     stored entries, whose columns ascend from the diagonal */
  int64_t* fp = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!fp) return 1;
  for (int32_t r = 0; r < n; ++r)
    for (int32_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
      fp[r + 1]++;
      if (col[k] != r) fp[col[k] + 1]++;
    }
  for (int32_t r = 0; r < n; ++r) fp[r + 1] += fp[r];
  const size_t total = (size_t)(fp[n] > 0 ? fp[n] : 1);
  int32_t* fc = (int32_t*)malloc(total * sizeof(int32_t));
  double* fv = (double*)malloc(total * sizeof(double));
  int64_t* fill = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!fc || !fv || !fill) {
    free(fp);
    free(fc);
    free(fv);
    free(fill);
    return 1;
  }
  for (int32_t r = 0; r <= n; ++r) fill[r] = fp[r];
  for (int32_t r = 0; r < n; ++r)
    for (int32_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
      const int32_t c = col[k];
      if (c != r) {
        fc[fill[c]] = r;
        fv[fill[c]] = val[k];
        fill[c]++;
      }
    }
  /* the stored part of row r (diagonal first if stored, then columns > r) */
  for (int32_t r = 0; r < n; ++r)
    for (int32_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
      fc[fill[r]] = col[k];
      fv[fill[r]] = val[k];
      fill[r]++;
    }
  for (int32_t t = 0; t < n_order; ++t) {
    const int32_t i = order[t];
    double dot = 0.0, nrm = 0.0;
    for (int64_t k = fp[i]; k < fp[i + 1]; ++k) {
      dot += fv[k] * x[fc[k]];
      nrm += fv[k] * fv[k];
    }
    if (nrm == 0.0) continue;
    const double coef = omega * (b[i] - dot) / nrm;
    for (int64_t k = fp[i]; k < fp[i + 1]; ++k) x[fc[k]] += coef * fv[k];
  }
  free(fp);
  free(fc);
  free(fv);
  free(fill);
  return 0;
}
