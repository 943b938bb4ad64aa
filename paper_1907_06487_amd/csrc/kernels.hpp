// Device-side argument blocks and launchers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace race {

// Device pointers of one schedule's layout (see layout.hpp for the meaning).
template <typename ValT>
struct UnitArgs {
  const int32_t* leaf_unit_ptr;
  const int32_t* unit_lo;
  const int32_t* unit_hi;
  const int32_t* unit_halo_ptr;
  const uint32_t* halo;
  const uint32_t* row_first_bits;
  const int32_t* unit_chunk_ptr;
  const uint32_t* chunk_off;
  const int32_t* chunk_len;
  const uint16_t* lane_slot;
  const ValT* lane_diag;
  const ValT* sell_val;
  const uint16_t* sell_slot;
};

// One phase: n_leaves workgroups starting at leaf_base; k right-hand sides
// (1..16) in row-major x/y; wmax = largest unit window of the phase.
template <typename ValT>
hipError_t launch_race_phase(const UnitArgs<ValT>& a, int32_t leaf_base, int32_t n_leaves, int32_t k, const double* x,
                             double* y, int32_t wmax, int32_t threads, hipStream_t st);

hipError_t launch_csr_spmv(int32_t n, const int32_t* rp, const int32_t* col, const double* val, const double* x,
                           double* y, int32_t lanes_per_row, hipStream_t st);
hipError_t launch_atomic_symm(int32_t n, const int32_t* rp, const int32_t* col, const double* val, const double* x,
                              double* y, int32_t lanes_per_row, hipStream_t st);
hipError_t launch_permute(int32_t n, int32_t k, const int32_t* new2old, const double* in, double* out,
                          int32_t to_permuted, hipStream_t st);

}  // namespace race
