// Device data layout of a Gauss-Seidel sweep over a distance-1 RACE
// schedule (host side).
//
// The paper names Gauss-Seidel as the prime user of distance-1 colorings
// (Section 1, Section 4.2): leaves of one phase share no edge, so their rows
// can be updated at the same time.  A leaf runs on one wavefront, its rows
// in order; its LDS window holds the x of its own rows (updated in place)
// and of its halo, the rows outside the leaf that its rows read (they
// belong to other phases and do not change while the leaf runs).  Every
// row's off-diagonal entries of the FULL permuted matrix are stored with a
// 16-bit window slot (slot < R: own row lo + slot; else halo[slot - R]).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "schedule.hpp"

namespace race {

constexpr int32_t kGsMaxWindow = 16384;  // own rows + halo of one leaf (128 KiB of LDS)

struct GsLayout {
  int32_t n = 0;
  std::vector<int32_t> leaf_lo, leaf_hi;  // leaves in execution order (phase, then first row)
  std::vector<int32_t> phase_leaf_ptr;    // n_phases + 1
  std::vector<int32_t> phase_max_window;  // per phase, largest leaf window
  std::vector<int32_t> halo_ptr;          // n_leaves + 1
  std::vector<int32_t> halo;              // permuted row index of each halo slot
  std::vector<int32_t> row_ptr;           // n + 1: off-diagonal entries of the full permuted rows
  std::vector<uint16_t> slot;             // window slot of each entry (columns ascending within a row)
  std::vector<double> val;
  std::vector<double> diag;               // n
  int32_t max_window = 0;
  int32_t max_row = 0;                    // longest row (off-diagonals)
  int64_t halo_total = 0;
};

// Builds the layout for the tree's leaves.  Returns "" or an error message;
// *code receives RACE_EINVAL (a zero or missing diagonal) or
// RACE_EUNSUPPORTED (a leaf window above kGsMaxWindow, or more than 2^31
// entries).
std::string build_gs_layout(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                            const Tree& tree, GsLayout& out, int* code);

}  // namespace race
