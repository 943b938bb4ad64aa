// Learned cost model: host side (features, makespan, learned loads).
//
// A unit's cost (its compute plus flush time in microseconds) is predicted
// from 12 features of the unit by a small ReLU network (12 -> 64 -> 64 -> 1,
// float32) that outputs the natural log of the cost.  The network is trained
// on the device (mlp kernels) from traced products; on the host it is used
//   * as the load m of Sections 4.3-4.4 (balance_by = 2): every stage-0 BFS
//     level is cut into window-sized pieces as the layout would cut it, each
//     piece's predicted cost is shared among its rows by their nonzeros;
//   * through `simulate`, to compare schedules by their predicted makespan.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "layout.hpp"
#include "mlp.hpp"
#include "schedule.hpp"

namespace race {

// Network output for n feature rows (float32 arithmetic).
void mlp_forward_host(const float* theta, const float* X, int64_t n, float* y);

// Features of every unit (n_units x 12, units in execution order):
//  0 log2(1 + rows)          1 log2(1 + stored entries)
//  2 mean off-diagonals/row  3 max off-diagonals/row   4 their coefficient of variation
//  5 halo / rows             6 fraction of off-diagonals scattering past the unit's rows
//  7 fraction of the window flushed read-modify-write   8 fraction flushed by shared atomics
//  9 log2(1 + units of the unit's phase)   10 phase / phases   11 log2(k)
void unit_features(const Layout& L, const Tree& t, int32_t k, std::vector<float>& out);

// Predicted makespan of a dataflow product: tickets in the given order
// (`order` lists the units by ticket; empty: the layout's execution order)
// on `workers` workgroups, each taking the next ticket when it becomes free;
// unit u computes for (1 - flush_frac) cost[u], waits for its conflict
// edges, then flushes for flush_frac cost[u].  The clearing tasks are not
// modelled (their edges count as met).
double simulate(const Layout& L, const float* cost, double flush_frac, int32_t workers,
                const std::vector<int32_t>& order);

// Ticket order by critical path (Section 5's N_eff generalised to per-unit
// costs, with the longest remaining path as list-scheduling priority): the
// bottom level of a unit is its cost plus the largest bottom level among
// the units whose conflict edges point to it (float64, cost[u] added to
// that maximum); units are emitted one at a time, always the unit with the
// largest bottom level among those whose edges all point to emitted units
// (ties: lower unit index).  The result is a topological order of the
// conflict edges, so every first-writer flag and edge stays valid.
void critical_path_order(const Layout& L, const float* cost, std::vector<int32_t>& order);

// Row loads from the network (see above); loads are in nanoseconds, >= 1.
void learned_row_loads(const Graph& g, int32_t n, const int32_t* row_ptr, const int32_t* col, const float* theta,
                       int32_t window_max, int32_t root_mode, int32_t level_order, std::vector<int64_t>& m);

}  // namespace race
