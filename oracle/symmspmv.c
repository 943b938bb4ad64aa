/*
 * Serial SymmSpMV oracle -- test infrastructure only.
 *
 * Plain C rendering of the SymmSpMV kernel of Section 3.2 (Algorithm
 * "SymmSpMV"): A is symmetric and stored as its upper triangle (diagonal
 * included) in CRS; for each row the diagonal contributes A[r,r]*x[r], each
 * stored off-diagonal A[r,c] adds A[r,c]*x[c] to a row accumulator (the
 * gather) and A[r,c]*x[r] to b[c] (the scatter); the accumulator is added to
 * b[r] after the row.  b is cleared first.  A row whose first stored column
 * is not the row itself has a zero diagonal.
 *
 * Built with -O2 -ffp-contract=off so the products and sums round as written.
 */
#include <stdint.h>

void oracle_symm_spmv(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                      const double* x, double* b) {
  for (int32_t i = 0; i < n; ++i) b[i] = 0.0;
  for (int32_t row = 0; row < n; ++row) {
    int32_t idx = row_ptr[row];
    const int32_t end = row_ptr[row + 1];
    const double xr = x[row];
    if (idx < end && col[idx] == row) {
      b[row] += val[idx] * xr;
      ++idx;
    }
    double tmp = 0.0;
    for (; idx < end; ++idx) {
      const int32_t c = col[idx];
      tmp += val[idx] * x[c];
      b[c] += val[idx] * xr;
    }
    b[row] += tmp;
  }
}

/* Same with float32 matrix values, each promoted to double before use. */
void oracle_symm_spmv_f32(int32_t n, const int32_t* row_ptr, const int32_t* col, const float* val,
                          const double* x, double* b) {
  for (int32_t i = 0; i < n; ++i) b[i] = 0.0;
  for (int32_t row = 0; row < n; ++row) {
    int32_t idx = row_ptr[row];
    const int32_t end = row_ptr[row + 1];
    const double xr = x[row];
    if (idx < end && col[idx] == row) {
      b[row] += (double)val[idx] * xr;
      ++idx;
    }
    double tmp = 0.0;
    for (; idx < end; ++idx) {
      const int32_t c = col[idx];
      const double v = (double)val[idx];
      tmp += v * x[c];
      b[c] += v * xr;
    }
    b[row] += tmp;
  }
}
