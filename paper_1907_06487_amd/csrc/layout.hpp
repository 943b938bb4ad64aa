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
//
// Every y index a unit touches carries two flags:
//   first  - the unit is the first (in execution order) to write y[g]: it
//            stores instead of read-modify-write;
//   shared - (shared_atomics mode) two or more units of the unit's own leaf
//            touch g.  Those units run concurrently and combine their
//            contributions to y[g] with global atomic adds; y[g] is cleared
//            before the product when such a unit is its first toucher.
// Without shared entries the units of a leaf follow each other through
// conflict edges instead.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "schedule.hpp"

namespace race {

constexpr int32_t kSlice = 64;           // rows per slice (one wavefront)
constexpr uint16_t kNoRow = 0xFFFF;      // padding lane
constexpr uint32_t kFirstBit = 0x80000000u;
constexpr uint32_t kSharedBit = 0x40000000u;
constexpr uint32_t kIndexMask = 0x3fffffffu;  // indices are below 2^30
constexpr int32_t kZeroChunk = 4096;          // y entries one clearing task clears

struct Layout {
  int32_t n = 0;
  int32_t value_type = 0;  // 0 f64, 1 f32
  // upper(P A P^T): CRS, columns ascending
  std::vector<int32_t> prow_ptr, pcol;
  std::vector<double> pval;
  std::vector<double> pval_im;  // imaginary parts (complex values only, else empty)
  int64_t n_diag = 0;

  // execution structure
  std::vector<int32_t> phase_leaf_ptr;  // n_phases + 1, into the leaves list
  std::vector<int32_t> phase_unit_ptr;  // n_phases + 1, into the units (execution order is phase-major)
  std::vector<int32_t> leaf_units;      // 2 per leaf (tree order): first unit, one past the last
  std::vector<int32_t> unit_order_leaves;  // leaves in execution order (phase, then descending work)
  std::vector<int32_t> unit_leaf, unit_lo, unit_hi;
  std::vector<int32_t> unit_halo_ptr;   // n_units + 1
  std::vector<uint32_t> halo;           // index | kFirstBit | kSharedBit
  std::vector<uint32_t> row_flags;      // 2 bits per row (word r / 16, bits 2 (r % 16) + {0 first, 1 shared})
  std::vector<int32_t> zero_idx;        // ascending: y indices cleared before a product (first touch is shared)
  int32_t n_zero_tasks = 0;             // ceil(zero_idx / kZeroChunk): clearing tasks of a dataflow product
  std::vector<int32_t> unit_chunk_ptr;  // n_units + 1
  std::vector<uint32_t> chunk_off;      // element offset of a slice
  std::vector<int32_t> chunk_len;       // slots per row | (slice width << 16)
  std::vector<uint16_t> lane_slot;      // n_chunks * 64: window slot of each lane's row
  std::vector<double> lane_diag;        // n_chunks * 64: diagonal of that row (0 if none)
  std::vector<double> sell_val;         // padded slice elements
  std::vector<double> lane_diag_im, sell_val_im;  // imaginary parts (complex values only, else empty)
  std::vector<uint16_t> sell_slot;
  std::vector<int32_t> phase_max_window;  // per phase, largest unit window
  // conflict edges for dataflow execution: unit u waits for dep_idx[dep_ptr[u]
  // .. dep_ptr[u+1]), the earlier units touching one of its indices that it
  // cannot run beside (every pair except two shared touches), and for a
  // shared touch of a cleared entry, the clearing task of that entry's chunk
  // (encoded as n_units + task; the tasks are the first tickets of a product)
  std::vector<int32_t> dep_ptr, dep_idx;

  int32_t max_window = 0;
  int64_t halo_total = 0, rows_rmw = 0, halo_rmw = 0, shared_touches = 0;
};

inline uint32_t row_flag(const std::vector<uint32_t>& f, int32_t r) {
  return (f[static_cast<size_t>(r) >> 4] >> (2 * (r & 15))) & 3u;
}

// Builds the layout; returns "" or an error message.  *code receives the
// RACE_E* code for errors (RACE_EUNSUPPORTED when a single row does not fit
// the window or n >= 2^30, RACE_EINTERNAL when units of two leaves of one
// phase would touch one index).
// val_im: imaginary parts of the values (complex matrices), else NULL.
std::string build_layout(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                         const double* val_im, const Tree& tree, int32_t window_max, int32_t value_type,
                         bool shared_atomics, Layout& out, int* code);

// Read dependencies for matrix powers: for every unit u, the units whose
// touch sets (own rows and halo) meet u's touch set, u included, ascending
// (CSR over units).  A unit of power p reads x = y_(p-1) on exactly its
// touch set, which is final once these units have flushed power p - 1.
void build_read_deps(const Layout& L, std::vector<int32_t>& ptr, std::vector<int32_t>& idx);

// Ticket order of a P-power matrix-power launch.  Tickets are (power p,
// position r) pairs, r over one power's sequence (the n_zero_tasks clearing
// tasks, then the units in the order `ticket_unit`); order[t] is the
// power-major index p * per_power + r of ticket t.  The first n_static
// tickets stay the first n_static positions of power 0 (their owners claim
// them by index); the rest follow a topological order of every wait -- a
// unit's conflict edges within its power, and from power 1 on its read
// dependencies (rdep_ptr/rdep_idx) in the power before -- emitted by
// smallest key first, key = first row of the unit (0 for a clearing task)
// + p * lag_rows, ties by the power-major index.  lag_rows large gives the
// power-major order; small lets a unit's next power follow it closely, so
// its part of the matrix may still be cached.
void mpk_ticket_order(const Layout& L, const std::vector<int32_t>& ticket_unit, const std::vector<int32_t>& rdep_ptr,
                      const std::vector<int32_t>& rdep_idx, int32_t powers, int32_t n_static, int64_t lag_rows,
                      std::vector<int32_t>& order);

}  // namespace race
