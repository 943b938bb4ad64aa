// Device arguments and launcher of the Gauss-Seidel sweep kernel.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace race {

constexpr int32_t kGsMaxWindowBytes = 16384 * 8;  // LDS of the largest leaf window
constexpr int32_t kGsQuadMaxWindow = 2048;        // phases whose windows fit run four leaves per wavefront

// Device copies of a GsLayout (gauss_seidel.hpp).
struct GsArgs {
  const int32_t* leaf_lo;
  const int32_t* leaf_hi;
  const int32_t* halo_ptr;
  const int32_t* halo;
  const int32_t* row_ptr;
  const uint16_t* slot;
  const double* val;
  const double* diag;  // Gauss-Seidel: 1 / a_ii; Kaczmarz: a_ii (0 where none is stored)
  const double* nrm;   // Kaczmarz: 1 / |a_i|^2 of the full row (0 for a row with no value); else unused
};

// A whole sweep in one cooperative launch over the tickets of a GsFlow
// (gauss_seidel.hpp): device copies of its arrays, one completion flag per
// ticket (set to epoch when done), a status word (bit 0: a bounded wait gave
// up) and a drain word.
struct GsFlowArgs {
  const int32_t* ticket_item;
  const int32_t* ticket_back;
  const int32_t* item_leaf0;
  const int32_t* item_count;
  const int32_t* dep_ptr;
  const int32_t* dep_idx;
  uint32_t* flags;
  uint32_t* status;
  uint32_t* drain;  // set to epoch when a wait of this launch gave up
  int32_t n_tickets;
  uint32_t epoch;
};
// Workgroups of the cooperative launch: as many as the CUs hold at once.
hipError_t gs_flow_grid(int32_t wmax, int32_t n_cus, int32_t* grid);
hipError_t launch_gs_flow(const GsArgs& a, const GsFlowArgs& f, int32_t wmax, int32_t grid, const double* b, double* x,
                          hipStream_t st);

// Leaves leaf0 .. leaf0 + count - 1 (one phase), with windows of at most
// wmax entries: four per wavefront (16 lanes each) when wmax <=
// kGsQuadMaxWindow and count >= quad_min_leaves (more leaves than the
// device holds wavefronts: then a quarter of the wavefronts run them in
// fewer rounds), else one per wavefront; rows in order (backward: reversed).
// b and x are device arrays of n in the permuted order; x is updated in place.
hipError_t launch_gs_phase(const GsArgs& a, int32_t leaf0, int32_t count, int32_t wmax, bool backward,
                           int32_t quad_min_leaves, const double* b, double* x, hipStream_t st);

// A whole Kaczmarz sweep in one cooperative launch over the tickets of a
// plan from build_kacz_flow (one leaf per ticket); wmax: the largest leaf
// window.
hipError_t kacz_flow_grid(int32_t wmax, int32_t n_cus, int32_t* grid);
hipError_t launch_kacz_flow(const GsArgs& a, const GsFlowArgs& f, int32_t wmax, int32_t grid, double omega,
                            const double* b, double* x, hipStream_t st);

// Kaczmarz sweep over leaves leaf0 .. leaf0 + count - 1 of one phase of a
// distance-2 schedule (GsArgs of a Kaczmarz layout, nrm set): one leaf per
// wavefront, or four (16 lanes each) when wmax <= kGsQuadMaxWindow and
// count >= quad_min_leaves; a leaf's window (own rows and halo) is staged in
// LDS, updated row by row with x <- x + omega (b_i - a_i . x) / |a_i|^2 a_i
// in order (backward: reversed) and written back whole.  b and x: device
// arrays of n in the permuted order; x is updated in place.
hipError_t launch_kacz_phase(const GsArgs& a, int32_t leaf0, int32_t count, int32_t wmax, bool backward, double omega,
                             int32_t quad_min_leaves, const double* b, double* x, hipStream_t st);

}  // namespace race
