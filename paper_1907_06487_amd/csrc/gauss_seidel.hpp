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
  std::vector<double> diag;               // n (0 where none is stored: Kaczmarz layouts only)
  std::vector<double> nrm;                // Kaczmarz layouts: squared norm of every full row, diagonal included
  int32_t max_window = 0;
  int32_t max_row = 0;                    // longest row (off-diagonals)
  int64_t halo_total = 0;
};

// Builds the layout for the tree's leaves.  Returns "" or an error message;
// *code receives RACE_EINVAL (a zero or missing diagonal) or
// RACE_EUNSUPPORTED (a leaf window above kGsMaxWindow, or more than 2^31
// entries).
//
// kaczmarz: the layout of Kaczmarz sweeps over a distance-2 schedule.  A
// Kaczmarz row reads and writes x at every column it holds, so a leaf's
// whole window (own rows and halo) is written back, a missing or zero
// diagonal is allowed, every row's squared norm is kept (summed in
// ascending column order), and the build checks that the windows of the
// leaves of one phase are disjoint (the rows of a distance-2 phase are at
// distance 3 or more; *code RACE_EINTERNAL otherwise).
std::string build_gs_layout(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                            const Tree& tree, GsLayout& out, int* code, bool kaczmarz = false);

// Dataflow plan of a sweep in one persistent launch.  Items are up to
// kGsFlowLeaves consecutive leaves of one phase; tickets are the items of
// the forward sweep in phase order, or of the backward sweep in reverse
// phase order, or both (symmetric: forward, then backward).  A forward
// ticket waits for the forward tickets of the items holding its leaves'
// halo rows in earlier phases (their new x); a backward ticket for the
// backward tickets of those in later phases and, in a symmetric sweep, for
// its own forward ticket.  Leaves of one phase share no edge, so these are
// all the orderings the serial sweep fixes: every later reader or writer
// of a row this ticket reads or writes waits for it in turn, and every wait
// points to an earlier ticket.
constexpr int32_t kGsFlowLeaves = 4;
struct GsFlow {
  int32_t direction = -1;
  std::vector<int32_t> item_leaf0, item_count;  // items in execution order
  std::vector<int32_t> ticket_item;             // per ticket
  std::vector<int32_t> ticket_back;             // per ticket: 1 for the backward sweep
  std::vector<int32_t> dep_ptr, dep_idx;        // per ticket: the earlier tickets it waits for
};
void build_gs_flow(const GsLayout& G, int32_t direction, GsFlow& f);

// Dataflow plan of a Kaczmarz sweep over a Kaczmarz layout: one leaf per
// item and ticket, tickets in the serial sweep's order (forward: phases
// ascending; backward: descending; symmetric: both).  A leaf reads and
// writes its whole window, so a ticket waits for the latest earlier ticket
// whose window holds each of its window's rows: every pair of tickets that
// share a row then runs in the serial order (leaves of one phase share
// none).
void build_kacz_flow(const GsLayout& K, int32_t direction, GsFlow& f);

}  // namespace race
