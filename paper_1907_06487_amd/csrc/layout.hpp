// Device data layout of a RACE schedule for the gfx950 kernels.
//
// The permuted upper triangle is cut into *units*: a leaf of the tree is
// split into consecutive row ranges whose LDS window (own rows + halo) fits
// the budget; the units of a leaf run in order on one workgroup.  Inside a
// unit the off-diagonal entries are stored as slices of up to 64 rows (one
// row per lane; slot j of lane l of a slice of width w sits at element
// off + j * w + l), rows sorted by descending length inside the unit, with
// window-local 16-bit column slots:
//   slot < R      -> own row  lo + slot
//   slot >= R     -> halo[slot - R]  (a row after the unit, written by it)
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "schedule.hpp"

namespace race {

constexpr int32_t kSlice = 64;           // rows per slice (one wavefront)
constexpr uint16_t kNoRow = 0xFFFF;      // padding lane
constexpr uint32_t kFirstBit = 0x80000000u;

struct Layout {
  int32_t n = 0;
  int32_t value_type = 0;  // 0 f64, 1 f32
  // upper(P A P^T): CRS, columns ascending
  std::vector<int32_t> prow_ptr, pcol;
  std::vector<double> pval;
  int64_t n_diag = 0;

  // execution structure
  std::vector<int32_t> phase_leaf_ptr;  // n_phases + 1, into the leaves list
  std::vector<int32_t> leaf_units;      // 2 per leaf (tree order): first unit, one past the last
  std::vector<int32_t> unit_order_leaves;  // leaves in execution order (phase, then descending work)
  std::vector<int32_t> unit_leaf, unit_lo, unit_hi;
  std::vector<int32_t> unit_halo_ptr;   // n_units + 1
  std::vector<uint32_t> halo;           // index | kFirstBit when first writer
  std::vector<uint32_t> row_first_bits; // bit r: the row's own unit writes y[r] first
  std::vector<int32_t> unit_chunk_ptr;  // n_units + 1
  std::vector<uint32_t> chunk_off;      // element offset of a slice
  std::vector<int32_t> chunk_len;       // slots per row | (slice width << 16)
  std::vector<uint16_t> lane_slot;      // n_chunks * 64: window slot of each lane's row
  std::vector<double> lane_diag;        // n_chunks * 64: diagonal of that row (0 if none)
  std::vector<double> sell_val;         // padded slice elements
  std::vector<uint16_t> sell_slot;
  std::vector<int32_t> phase_max_window;  // per phase, largest unit window
  // conflict edges for dataflow execution: unit u waits for dep_idx[dep_ptr[u]
  // .. dep_ptr[u+1]), the latest earlier units touching each of its indices
  std::vector<int32_t> dep_ptr, dep_idx;

  int32_t max_window = 0;
  int64_t halo_total = 0, rows_rmw = 0, halo_rmw = 0;
};

// Builds the layout; returns "" or an error message.  *code receives the
// RACE_E* code for errors (RACE_EUNSUPPORTED when a single row does not fit
// the window, RACE_EINTERNAL when concurrent units would touch one index).
std::string build_layout(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val, const Tree& tree,
                         int32_t window_max, int32_t value_type, Layout& out, int* code);

}  // namespace race
