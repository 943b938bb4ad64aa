// RACE schedule construction on the host (Section 4 of the paper).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace race {

// Undirected graph of the matrix: off-diagonal pattern of U + U^T.
struct Graph {
  int32_t n = 0;
  std::vector<int64_t> ptr;  // n + 1
  std::vector<int32_t> adj;
};

struct TreeNode {
  int32_t stage = -1;  // -1 for the root
  int32_t color = 0;   // 0 = first color (red), 1 = second (blue)
  int32_t lo = 0, hi = 0;  // rows [lo, hi) in the final permuted order
  int32_t workers = 1;     // threads assigned (n_t of the level group)
  int32_t parent = -1;
  int32_t n_levels = 0;    // levels found when refined, 0 for leaves
  std::vector<int32_t> children;
};

struct TreeParams {
  int32_t n_workers = 1024;
  int32_t max_stages = 4;
  int32_t dist_k = 2;
  bool global_lb = false;
  int32_t root_mode = 0;    // stage-0 island roots: 0 first vertex in input order, 1 pseudo-peripheral
  int32_t level_order = 0;  // stage-0 order inside a level: 0 input order, 1 Cuthill-McKee discovery order
  double eps[8] = {0.8, 0.8, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5};
};

struct Tree {
  int32_t n = 0;
  int32_t n_workers = 0;
  std::vector<int32_t> perm;        // new -> old
  std::vector<TreeNode> nodes;      // preorder, nodes[0] = root
  std::vector<int32_t> leaves;      // sorted by (phase, lo, id)
  std::vector<int32_t> leaf_phase;  // aligned with leaves
  int32_t depth = -1;               // deepest leaf stage
  int32_t n_phases = 1;
  int32_t n_eff_root = 0;
  double eta = 1.0;
  int32_t n_levels0 = 0;
};

void build_graph(int32_t n, const int32_t* row_ptr, const int32_t* col, Graph& g);

// Load per row: stored entries of the full row (balance by nonzeros) or 1.
void row_loads(int32_t n, const int32_t* row_ptr, const int32_t* col, bool by_rows, std::vector<int64_t>& m);

// Builds the tree.  row_load gives m(row) for every row (length n).
// Returns an empty string on success, else an error message.
std::string build_tree(const Graph& g, const std::vector<int64_t>& row_load, const TreeParams& p, Tree& out);

// Pseudo-peripheral vertex of the connected component of `start` (George
// and Liu's node finder, see schedule.cpp).  `dist` is an all -1 scratch
// array of length g.n, restored before returning.
int32_t pseudo_peripheral(const Graph& g, int32_t start, std::vector<int32_t>& dist);

// Stage-0 level structure of the whole graph (Section 4.1): islands in the
// order of their first vertex, each rooted there (root_mode 0) or at the
// pseudo-peripheral vertex found from it (1), levels two above the largest
// so far; `order` lists the vertices by level, inside a level in input order
// (level_order 0) or in Cuthill-McKee discovery order (1: every vertex's new
// neighbours by increasing degree, ties by index).
void stage0_order(const Graph& g, int32_t root_mode, int32_t level_order, std::vector<int32_t>& lev,
                  std::vector<int32_t>& order);

// Exposed for unit tests through the ABI-free C++ layer.
struct Pair {
  int32_t start, end;  // levels [start, end)
  int64_t b;
};
std::vector<Pair> aggregate_pairs(const std::vector<int64_t>& m_levels, int64_t n_t, double eps_s, int32_t k);
void split_pairs(const std::vector<Pair>& pairs, const std::vector<int64_t>& m_levels, int32_t k,
                 std::vector<int32_t>& t_ptr, std::vector<int64_t>& worker);
void load_balance(std::vector<int32_t>& t_ptr, const std::vector<int64_t>& worker, const std::vector<int64_t>& m_levels,
                  int32_t k);

}  // namespace race
