// Vendor yardstick: rocSPARSE's CSR SpMV timed as a black box on the same
// device, for the full matrix (general) or for the stored upper triangle of
// a symmetric matrix (rocSPARSE's own symmetric product).  The paper's
// comparison takes the best variant of the vendor library of its machines
// (Section 6); rocSPARSE is this device's vendor library.
#include <hip/hip_runtime.h>
#include <rocsparse/rocsparse.h>

#include <algorithm>
#include <cstdint>
#include <new>
#include <string>

#include "../../include/race.h"
#include "errors.hpp"

struct race_vendor {
  int device = -1;
  int32_t n = 0;
  int64_t nnz = 0;
  rocsparse_spmv_alg alg = rocsparse_spmv_alg_default;
  rocsparse_handle handle = nullptr;
  rocsparse_spmat_descr A = nullptr;
  rocsparse_dnvec_descr vx = nullptr, vy = nullptr;
  int32_t* rp = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
  void* buffer = nullptr;
  size_t buffer_size = 0;
};

namespace {

int sparse_fail(rocsparse_status st, const char* what) {
  return race::set_error(RACE_EHIP, std::string(what) + ": rocSPARSE status " + std::to_string(static_cast<int>(st)));
}

void vendor_release(race_vendor* h) {
  if (h->vx) (void)rocsparse_destroy_dnvec_descr(h->vx);
  if (h->vy) (void)rocsparse_destroy_dnvec_descr(h->vy);
  if (h->A) (void)rocsparse_destroy_spmat_descr(h->A);
  if (h->handle) (void)rocsparse_destroy_handle(h->handle);
  for (void* p : {static_cast<void*>(h->rp), static_cast<void*>(h->col), static_cast<void*>(h->val), h->buffer})
    if (p) (void)hipFree(p);
}

// the library's stage-wise SpMV (buffer size, preprocessing, product)
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wdeprecated-declarations"
rocsparse_status spmv_stage(race_vendor* h, rocsparse_spmv_stage stage, size_t* size, void* buf) {
  const double one = 1.0, zero = 0.0;
  return rocsparse_spmv(h->handle, rocsparse_operation_none, &one, h->A, h->vx, &zero, h->vy,
                        rocsparse_datatype_f64_r, h->alg, stage, size, buf);
}
#pragma clang diagnostic pop

}  // namespace

extern "C" {

int race_vendor_create(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                       int32_t symmetric_upper, int32_t alg, race_vendor_t* out) {
  if (!out) return race::set_error(RACE_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || !row_ptr || !col || !val) return race::set_error(RACE_EINVAL, "need n >= 1 and host CRS arrays");
  if (row_ptr[0] != 0) return race::set_error(RACE_EINVAL, "row_ptr[0] must be 0");
  for (int32_t r = 0; r < n; ++r) {
    if (row_ptr[r + 1] < row_ptr[r]) return race::set_error(RACE_EINVAL, "row_ptr decreases");
    for (int32_t i = row_ptr[r]; i < row_ptr[r + 1]; ++i)
      if (col[i] < (symmetric_upper ? r : 0) || col[i] >= n)
        return race::set_error(RACE_EINVAL, "column out of range (upper triangle: col >= row)");
  }
  static const rocsparse_spmv_alg algs[] = {rocsparse_spmv_alg_csr_adaptive, rocsparse_spmv_alg_csr_rowsplit,
                                            rocsparse_spmv_alg_csr_lrb};
  // (the library's nnz-split CSR algorithm answers "invalid value" to the
  // stage-wise interface on this ROCm, so it is not offered)
  if (alg < 0 || alg > 2) return race::set_error(RACE_EINVAL, "alg must be 0 (adaptive), 1 (row split) or 2 (LRB)");
  race_vendor* h = new (std::nothrow) race_vendor();
  if (!h) return race::set_error(RACE_ENOMEM, "out of host memory");
  h->n = n;
  h->nnz = row_ptr[n];
  h->alg = algs[alg];
  double* tx = nullptr;
  double* ty = nullptr;
  auto fail_hip = [&](hipError_t e, const char* what) {
    if (tx) (void)hipFree(tx);
    if (ty) (void)hipFree(ty);
    vendor_release(h);
    delete h;
    return race::set_hip_error(e, what);
  };
  auto fail_sp = [&](rocsparse_status st, const char* what) {
    if (tx) (void)hipFree(tx);
    if (ty) (void)hipFree(ty);
    vendor_release(h);
    delete h;
    return st == rocsparse_status_not_implemented
               ? race::set_error(RACE_EUNSUPPORTED, std::string(what) + ": not implemented by rocSPARSE")
               : sparse_fail(st, what);
  };
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  const size_t nnz = static_cast<size_t>(h->nnz);
  e = hipMalloc(&h->rp, sizeof(int32_t) * (static_cast<size_t>(n) + 1));
  if (e == hipSuccess) e = hipMalloc(&h->col, sizeof(int32_t) * std::max<size_t>(nnz, 1));
  if (e == hipSuccess) e = hipMalloc(&h->val, sizeof(double) * std::max<size_t>(nnz, 1));
  if (e == hipSuccess) e = hipMalloc(&tx, sizeof(double) * n);
  if (e == hipSuccess) e = hipMalloc(&ty, sizeof(double) * n);
  if (e != hipSuccess) return fail_hip(e, "hipMalloc");
  e = hipMemcpy(h->rp, row_ptr, sizeof(int32_t) * (static_cast<size_t>(n) + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess && nnz) e = hipMemcpy(h->col, col, sizeof(int32_t) * nnz, hipMemcpyHostToDevice);
  if (e == hipSuccess && nnz) e = hipMemcpy(h->val, val, sizeof(double) * nnz, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(tx, 0, sizeof(double) * n);
  if (e != hipSuccess) return fail_hip(e, "hipMemcpy");
  rocsparse_status st = rocsparse_create_handle(&h->handle);
  if (st != rocsparse_status_success) return fail_sp(st, "rocsparse_create_handle");
  st = rocsparse_create_csr_descr(&h->A, n, n, h->nnz, h->rp, h->col, h->val, rocsparse_indextype_i32,
                                  rocsparse_indextype_i32, rocsparse_index_base_zero, rocsparse_datatype_f64_r);
  if (st != rocsparse_status_success) return fail_sp(st, "rocsparse_create_csr_descr");
  if (symmetric_upper) {
    const rocsparse_matrix_type mt = rocsparse_matrix_type_symmetric;
    const rocsparse_fill_mode fm = rocsparse_fill_mode_upper;
    st = rocsparse_spmat_set_attribute(h->A, rocsparse_spmat_matrix_type, &mt, sizeof(mt));
    if (st == rocsparse_status_success)
      st = rocsparse_spmat_set_attribute(h->A, rocsparse_spmat_fill_mode, &fm, sizeof(fm));
    if (st != rocsparse_status_success) return fail_sp(st, "symmetric matrix attributes");
  }
  st = rocsparse_create_dnvec_descr(&h->vx, n, tx, rocsparse_datatype_f64_r);
  if (st == rocsparse_status_success) st = rocsparse_create_dnvec_descr(&h->vy, n, ty, rocsparse_datatype_f64_r);
  if (st != rocsparse_status_success) return fail_sp(st, "rocsparse_create_dnvec_descr");
  st = spmv_stage(h, rocsparse_spmv_stage_buffer_size, &h->buffer_size, nullptr);
  if (st != rocsparse_status_success) return fail_sp(st, "SpMV buffer size");
  e = hipMalloc(&h->buffer, std::max<size_t>(h->buffer_size, 16));
  if (e != hipSuccess) return fail_hip(e, "hipMalloc of the SpMV buffer");
  st = spmv_stage(h, rocsparse_spmv_stage_preprocess, &h->buffer_size, h->buffer);
  if (st != rocsparse_status_success) return fail_sp(st, "SpMV preprocessing");
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return fail_hip(e, "hipDeviceSynchronize");
  (void)hipFree(tx);
  (void)hipFree(ty);
  tx = ty = nullptr;
  *out = h;
  return RACE_OK;
}

int race_vendor_spmv(race_vendor_t h, const double* x, double* y, void* stream) {
  if (!h) return race::set_error(RACE_EINVAL, "handle is NULL");
  if (!x || !y) return race::set_error(RACE_EINVAL, "x or y is NULL");
  rocsparse_status st = rocsparse_set_stream(h->handle, static_cast<hipStream_t>(stream));
  if (st == rocsparse_status_success) st = rocsparse_dnvec_set_values(h->vx, const_cast<double*>(x));
  if (st == rocsparse_status_success) st = rocsparse_dnvec_set_values(h->vy, y);
  if (st == rocsparse_status_success) st = spmv_stage(h, rocsparse_spmv_stage_compute, &h->buffer_size, h->buffer);
  if (st != rocsparse_status_success) return sparse_fail(st, "rocSPARSE SpMV");
  return RACE_OK;
}

void race_vendor_destroy(race_vendor_t h) {
  if (!h) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (h->device >= 0) (void)hipSetDevice(h->device);
  vendor_release(h);
  (void)hipSetDevice(cur);
  delete h;
}

}  // extern "C"
