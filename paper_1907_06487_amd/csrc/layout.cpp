// Device data layout of a RACE schedule (see layout.hpp).
#include "layout.hpp"

#include <algorithm>
#include <numeric>
#include <queue>
#include <stdexcept>

#include "../../include/race.h"

namespace race {

static void permute_upper(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                          const double* val_im, const std::vector<int32_t>& perm, Layout& L) {
  std::vector<int32_t> old2new(static_cast<size_t>(n));
  for (int32_t i = 0; i < n; ++i) old2new[perm[i]] = i;
  const int64_t nnz = row_ptr[n];
  L.prow_ptr.assign(static_cast<size_t>(n) + 1, 0);
  for (int32_t r = 0; r < n; ++r)
    for (int32_t i = row_ptr[r]; i < row_ptr[r + 1]; ++i) {
      const int32_t a = old2new[r], b = old2new[col[i]];
      ++L.prow_ptr[std::min(a, b) + 1];
    }
  for (int32_t i = 0; i < n; ++i) L.prow_ptr[i + 1] += L.prow_ptr[i];
  L.pcol.resize(static_cast<size_t>(nnz));
  L.pval.resize(static_cast<size_t>(nnz));
  if (val_im) L.pval_im.resize(static_cast<size_t>(nnz));
  std::vector<int32_t> fill(L.prow_ptr.begin(), L.prow_ptr.end() - 1);
  for (int32_t r = 0; r < n; ++r)
    for (int32_t i = row_ptr[r]; i < row_ptr[r + 1]; ++i) {
      const int32_t a = old2new[r], b = old2new[col[i]];
      const int32_t lo = std::min(a, b), hi = std::max(a, b);
      const int32_t at = fill[lo]++;
      L.pcol[at] = hi;
      L.pval[at] = val ? val[i] : 0.0;
      // a Hermitian entry that lands below the diagonal is stored as its
      // mirror above it, which holds the conjugate
      if (val_im) L.pval_im[at] = (L.value_type == 3 && a > b) ? -val_im[i] : val_im[i];
    }
  struct Entry {
    int32_t c;
    double v, w;
  };
  std::vector<Entry> tmp;
  L.n_diag = 0;
  for (int32_t r = 0; r < n; ++r) {
    const int32_t s = L.prow_ptr[r], e = L.prow_ptr[r + 1];
    tmp.clear();
    for (int32_t i = s; i < e; ++i) tmp.push_back({L.pcol[i], L.pval[i], val_im ? L.pval_im[i] : 0.0});
    std::sort(tmp.begin(), tmp.end(), [](const Entry& x, const Entry& y) { return x.c < y.c; });
    for (int32_t i = s; i < e; ++i) {
      L.pcol[i] = tmp[i - s].c;
      L.pval[i] = tmp[i - s].v;
      if (val_im) L.pval_im[i] = tmp[i - s].w;
    }
    if (s < e && L.pcol[s] == r) ++L.n_diag;
  }
}

std::string build_layout(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                         const double* val_im, const Tree& tree, int32_t window_max, int32_t value_type,
                         bool shared_atomics, Layout& L, int* code) {
  *code = RACE_OK;
  L = Layout();
  if (n >= (1 << 30)) {
    *code = RACE_EUNSUPPORTED;
    return "n must be below 2^30";
  }
  L.n = n;
  L.value_type = value_type;
  permute_upper(n, row_ptr, col, val, val_im, tree.perm, L);
  const std::vector<int32_t>& rp = L.prow_ptr;
  const std::vector<int32_t>& pc = L.pcol;

  // phases -> leaves
  const int32_t n_leaves = static_cast<int32_t>(tree.leaves.size());
  L.phase_leaf_ptr.assign(static_cast<size_t>(tree.n_phases) + 1, 0);
  for (int32_t t = 0; t < n_leaves; ++t) ++L.phase_leaf_ptr[tree.leaf_phase[t] + 1];
  for (int32_t p = 0; p < tree.n_phases; ++p) L.phase_leaf_ptr[p + 1] += L.phase_leaf_ptr[p];

  // units: greedy row ranges of each leaf whose window fits
  std::vector<uint8_t> marked(static_cast<size_t>(n), 0);
  std::vector<int32_t> mark_list;
  std::vector<int32_t> slot_of(static_cast<size_t>(n), -1);
  L.leaf_units.assign(2 * static_cast<size_t>(n_leaves), 0);
  // execution order: phase by phase; inside a phase (no conflicts between its
  // leaves) the heaviest leaves first, so the large units start early
  L.unit_order_leaves.resize(static_cast<size_t>(n_leaves));
  std::iota(L.unit_order_leaves.begin(), L.unit_order_leaves.end(), 0);
  {
    std::vector<int64_t> work(static_cast<size_t>(n_leaves));
    for (int32_t t = 0; t < n_leaves; ++t) {
      const TreeNode& nd = tree.nodes[tree.leaves[t]];
      work[t] = static_cast<int64_t>(rp[nd.hi] - rp[nd.lo]) + (nd.hi - nd.lo);
    }
    std::stable_sort(L.unit_order_leaves.begin(), L.unit_order_leaves.end(), [&](int32_t a, int32_t b) {
      if (tree.leaf_phase[a] != tree.leaf_phase[b]) return tree.leaf_phase[a] < tree.leaf_phase[b];
      return work[a] > work[b];
    });
  }
  L.unit_halo_ptr.assign(1, 0);
  L.unit_chunk_ptr.assign(1, 0);
  std::vector<int32_t> rows_sorted;
  uint64_t elems = 0;
  for (int32_t t : L.unit_order_leaves) {
    const TreeNode& leaf = tree.nodes[tree.leaves[t]];
    L.leaf_units[2 * static_cast<size_t>(t)] = static_cast<int32_t>(L.unit_lo.size());
    int32_t a = leaf.lo;
    while (a < leaf.hi) {
      int64_t w = 0;
      int32_t b = a;
      while (b < leaf.hi) {
        const int32_t r = b;
        int64_t new_h = 0;
        for (int32_t i = rp[r]; i < rp[r + 1]; ++i)
          if (pc[i] > r && !marked[pc[i]]) ++new_h;
        const int64_t w_new = w + (marked[r] ? 0 : 1) + new_h;
        if (w_new > window_max) {
          if (b == a) {
            *code = RACE_EUNSUPPORTED;
            return "row " + std::to_string(r) + " alone needs a window of " + std::to_string(w_new) +
                   " entries, more than window_max " + std::to_string(window_max);
          }
          break;
        }
        if (!marked[r]) { marked[r] = 1; mark_list.push_back(r); }
        for (int32_t i = rp[r]; i < rp[r + 1]; ++i)
          if (!marked[pc[i]]) { marked[pc[i]] = 1; mark_list.push_back(pc[i]); }
        w = w_new;
        ++b;
      }
      // unit [a, b): halo = marked indices >= b, ascending
      const int32_t R = b - a;
      const size_t h0 = L.halo.size();
      for (int32_t v : mark_list)
        if (v >= b) L.halo.push_back(static_cast<uint32_t>(v));
      std::sort(L.halo.begin() + h0, L.halo.end());
      const int32_t H = static_cast<int32_t>(L.halo.size() - h0);
      for (int32_t v : mark_list) marked[v] = 0;
      mark_list.clear();
      for (int32_t j = 0; j < H; ++j) slot_of[L.halo[h0 + j]] = R + j;
      L.max_window = std::max<int32_t>(L.max_window, R + H);
      L.unit_leaf.push_back(t);
      L.unit_lo.push_back(a);
      L.unit_hi.push_back(b);
      L.unit_halo_ptr.push_back(static_cast<int32_t>(L.halo.size()));
      // slices, rows by descending off-diagonal count (stable)
      rows_sorted.resize(static_cast<size_t>(R));
      std::iota(rows_sorted.begin(), rows_sorted.end(), a);
      auto offd = [&](int32_t r) {
        const int32_t len = rp[r + 1] - rp[r];
        return len - ((len > 0 && pc[rp[r]] == r) ? 1 : 0);
      };
      std::stable_sort(rows_sorted.begin(), rows_sorted.end(), [&](int32_t x, int32_t y) { return offd(x) > offd(y); });
      for (int32_t c0 = 0; c0 < R; c0 += kSlice) {
        const int32_t cn = std::min(kSlice, R - c0);
        int32_t len = 0;
        for (int32_t l = 0; l < cn; ++l) len = std::max(len, offd(rows_sorted[c0 + l]));
        L.chunk_off.push_back(static_cast<uint32_t>(elems));
        L.chunk_len.push_back(len | (cn << 16));
        const size_t base = L.sell_val.size();
        const bool cplx = !L.pval_im.empty();
        L.sell_val.resize(base + static_cast<size_t>(len) * cn, 0.0);
        if (cplx) L.sell_val_im.resize(base + static_cast<size_t>(len) * cn, 0.0);
        L.sell_slot.resize(base + static_cast<size_t>(len) * cn, 0);
        for (int32_t l = 0; l < kSlice; ++l) {
          if (l >= cn) {
            L.lane_slot.push_back(kNoRow);
            L.lane_diag.push_back(0.0);
            if (cplx) L.lane_diag_im.push_back(0.0);
            continue;
          }
          const int32_t r = rows_sorted[c0 + l];
          const uint16_t own = static_cast<uint16_t>(r - a);
          L.lane_slot.push_back(own);
          int32_t i = rp[r];
          double d = 0.0, d_im = 0.0;
          if (i < rp[r + 1] && pc[i] == r) {
            d = L.pval[i];
            if (cplx) d_im = L.pval_im[i];
            ++i;
          }
          L.lane_diag.push_back(d);
          if (cplx) L.lane_diag_im.push_back(d_im);
          int32_t j = 0;
          for (; i < rp[r + 1]; ++i, ++j) {
            const int32_t c = pc[i];
            const int32_t s = c < b ? c - a : slot_of[c];
            L.sell_val[base + static_cast<size_t>(j) * cn + l] = L.pval[i];
            if (cplx) L.sell_val_im[base + static_cast<size_t>(j) * cn + l] = L.pval_im[i];
            L.sell_slot[base + static_cast<size_t>(j) * cn + l] = static_cast<uint16_t>(s);
          }
          for (; j < len; ++j) L.sell_slot[base + static_cast<size_t>(j) * cn + l] = own;
        }
        elems += static_cast<uint64_t>(len) * cn;
        if (elems >= (1ull << 32)) {
          *code = RACE_EUNSUPPORTED;
          return "sliced layout exceeds 2^32 elements";
        }
      }
      L.unit_chunk_ptr.push_back(static_cast<int32_t>(L.chunk_len.size()));
      for (int32_t j = 0; j < H; ++j) slot_of[L.halo[h0 + j]] = -1;
      a = b;
    }
    L.leaf_units[2 * static_cast<size_t>(t) + 1] = static_cast<int32_t>(L.unit_lo.size());
  }
  if (L.halo.size() >= static_cast<size_t>(INT32_MAX)) {
    *code = RACE_EUNSUPPORTED;
    return "halo lists exceed 2^31 entries";
  }

  const int32_t n_units = static_cast<int32_t>(L.unit_lo.size());
  L.row_flags.assign((static_cast<size_t>(n) + 15) / 16, 0u);
  // shared indices: touched by two or more units of one leaf
  if (shared_atomics) {
    std::vector<int32_t> cnt(static_cast<size_t>(n), 0), stamp(static_cast<size_t>(n), -1);
    for (int32_t t = 0; t < n_leaves; ++t) {
      const int32_t u0 = L.leaf_units[2 * static_cast<size_t>(t)], u1 = L.leaf_units[2 * static_cast<size_t>(t) + 1];
      if (u1 - u0 < 2) continue;
      auto count = [&](int32_t g) {
        if (stamp[g] != t) {
          stamp[g] = t;
          cnt[g] = 0;
        }
        ++cnt[g];
      };
      for (int32_t u = u0; u < u1; ++u) {
        for (int32_t g = L.unit_lo[u]; g < L.unit_hi[u]; ++g) count(g);
        for (int32_t j = L.unit_halo_ptr[u]; j < L.unit_halo_ptr[u + 1]; ++j) count(static_cast<int32_t>(L.halo[j]));
      }
      for (int32_t u = u0; u < u1; ++u) {
        for (int32_t g = L.unit_lo[u]; g < L.unit_hi[u]; ++g)
          if (cnt[g] > 1) L.row_flags[static_cast<size_t>(g) >> 4] |= 2u << (2 * (g & 15));
        for (int32_t j = L.unit_halo_ptr[u]; j < L.unit_halo_ptr[u + 1]; ++j)
          if (cnt[static_cast<int32_t>(L.halo[j])] > 1) L.halo[j] |= kSharedBit;
      }
    }
  }

  // first writer of every y entry, and the independence check: units of
  // different leaves in one phase must never touch the same index.  A first
  // touch that is shared is replaced by clearing y[g] before the product.
  std::vector<int32_t> last_phase(static_cast<size_t>(n), -1), last_leaf(static_cast<size_t>(n), -1);
  for (int32_t u = 0; u < n_units; ++u) {
    const int32_t t = L.unit_leaf[u];
    const int32_t ph = tree.leaf_phase[t];
    auto touch = [&](int32_t g) -> int {
      if (last_phase[g] < 0) {
        last_phase[g] = ph;
        last_leaf[g] = t;
        return 1;
      }
      if (last_phase[g] == ph && last_leaf[g] != t) return -1;
      last_phase[g] = ph;
      last_leaf[g] = t;
      return 0;
    };
    for (int32_t g = L.unit_lo[u]; g < L.unit_hi[u]; ++g) {
      const int f = touch(g);
      if (f < 0) {
        *code = RACE_EINTERNAL;
        return "phase " + std::to_string(ph) + ": row " + std::to_string(g) + " is touched by two leaves";
      }
      const bool shared = row_flag(L.row_flags, g) & 2u;
      if (shared) {
        ++L.shared_touches;
        if (f) L.zero_idx.push_back(g);
      } else if (f) {
        L.row_flags[static_cast<size_t>(g) >> 4] |= 1u << (2 * (g & 15));
      } else {
        ++L.rows_rmw;
      }
    }
    for (int32_t j = L.unit_halo_ptr[u]; j < L.unit_halo_ptr[u + 1]; ++j) {
      const int32_t g = static_cast<int32_t>(L.halo[j] & kIndexMask);
      const int f = touch(g);
      if (f < 0) {
        *code = RACE_EINTERNAL;
        return "phase " + std::to_string(ph) + ": index " + std::to_string(g) + " is touched by two leaves";
      }
      if (L.halo[j] & kSharedBit) {
        ++L.shared_touches;
        if (f) L.zero_idx.push_back(g);
      } else if (f) {
        L.halo[j] |= kFirstBit;
      } else {
        ++L.halo_rmw;
      }
    }
  }
  std::sort(L.zero_idx.begin(), L.zero_idx.end());
  L.n_zero_tasks = static_cast<int32_t>((L.zero_idx.size() + kZeroChunk - 1) / kZeroChunk);
  std::vector<int32_t> zero_task(static_cast<size_t>(n), -1);
  for (size_t i = 0; i < L.zero_idx.size(); ++i) zero_task[L.zero_idx[i]] = static_cast<int32_t>(i / kZeroChunk);
  // conflict edges: a plain touch of y[g] waits for the last plain toucher and
  // every shared toucher since; a shared touch waits for the last plain
  // toucher only (atomic adds of shared touches commute)
  {
    std::vector<int32_t> last_plain(static_cast<size_t>(n), -1), deps, pool_unit;
    std::vector<int64_t> shared_head(static_cast<size_t>(n), -1), pool_next;
    L.dep_ptr.assign(1, 0);
    for (int32_t u = 0; u < n_units; ++u) {
      deps.clear();
      auto touch = [&](int32_t g, bool shared) {
        if (last_plain[g] >= 0) deps.push_back(last_plain[g]);
        if (shared && zero_task[g] >= 0) deps.push_back(n_units + zero_task[g]);
        if (shared) {
          pool_unit.push_back(u);
          pool_next.push_back(shared_head[g]);
          shared_head[g] = static_cast<int64_t>(pool_unit.size()) - 1;
        } else {
          for (int64_t q = shared_head[g]; q >= 0; q = pool_next[q]) deps.push_back(pool_unit[q]);
          shared_head[g] = -1;
          last_plain[g] = u;
        }
      };
      for (int32_t g = L.unit_lo[u]; g < L.unit_hi[u]; ++g) touch(g, row_flag(L.row_flags, g) & 2u);
      for (int32_t j = L.unit_halo_ptr[u]; j < L.unit_halo_ptr[u + 1]; ++j)
        touch(static_cast<int32_t>(L.halo[j] & kIndexMask), L.halo[j] & kSharedBit);
      std::sort(deps.begin(), deps.end());
      deps.erase(std::unique(deps.begin(), deps.end()), deps.end());
      for (int32_t v : deps) {
        if (v >= u && v < n_units) {
          *code = RACE_EINTERNAL;
          return "conflict edge does not point to an earlier unit";
        }
        L.dep_idx.push_back(v);
      }
      L.dep_ptr.push_back(static_cast<int32_t>(L.dep_idx.size()));
    }
  }
  L.halo_total = static_cast<int64_t>(L.halo.size());
  L.phase_unit_ptr.assign(static_cast<size_t>(tree.n_phases) + 1, 0);
  for (int32_t u = 0; u < n_units; ++u) ++L.phase_unit_ptr[tree.leaf_phase[L.unit_leaf[u]] + 1];
  for (int32_t p = 0; p < tree.n_phases; ++p) L.phase_unit_ptr[p + 1] += L.phase_unit_ptr[p];
  L.phase_max_window.assign(static_cast<size_t>(tree.n_phases), 0);
  for (int32_t u = 0; u < n_units; ++u) {
    const int32_t ph = tree.leaf_phase[L.unit_leaf[u]];
    const int32_t w = (L.unit_hi[u] - L.unit_lo[u]) + (L.unit_halo_ptr[u + 1] - L.unit_halo_ptr[u]);
    L.phase_max_window[ph] = std::max(L.phase_max_window[ph], w);
  }
  return std::string();
}

void mpk_ticket_order(const Layout& L, const std::vector<int32_t>& ticket_unit, const std::vector<int32_t>& rdep_ptr,
                      const std::vector<int32_t>& rdep_idx, int32_t powers, int32_t n_static, int64_t lag_rows,
                      std::vector<int32_t>& order) {
  const int32_t nu = static_cast<int32_t>(L.unit_lo.size());
  const int32_t nz = L.n_zero_tasks;
  const int32_t per = nu + nz;
  const int64_t total = static_cast<int64_t>(per) * powers;
  // position of each unit within a power (after the clearing tasks)
  std::vector<int32_t> pos(static_cast<size_t>(nu));
  for (int32_t i = 0; i < nu; ++i) pos[static_cast<size_t>(ticket_unit[static_cast<size_t>(i)])] = nz + i;
  auto flag_pos = [&](int32_t v) { return v < nu ? pos[static_cast<size_t>(v)] : v - nu; };
  // dependency counts and successor lists over power-major indices
  std::vector<int32_t> indeg(static_cast<size_t>(total), 0);
  std::vector<int64_t> succ_ptr(static_cast<size_t>(total) + 1, 0);
  auto for_deps = [&](int64_t node, auto&& fn) {
    const int32_t p = static_cast<int32_t>(node / per), r = static_cast<int32_t>(node % per);
    if (r < nz) return;
    const int32_t u = ticket_unit[static_cast<size_t>(r - nz)];
    for (int32_t d = L.dep_ptr[static_cast<size_t>(u)]; d < L.dep_ptr[static_cast<size_t>(u) + 1]; ++d)
      fn(static_cast<int64_t>(p) * per + flag_pos(L.dep_idx[static_cast<size_t>(d)]));
    if (p > 0)
      for (int32_t d = rdep_ptr[static_cast<size_t>(u)]; d < rdep_ptr[static_cast<size_t>(u) + 1]; ++d)
        fn(static_cast<int64_t>(p - 1) * per + pos[static_cast<size_t>(rdep_idx[static_cast<size_t>(d)])]);
  };
  for (int64_t v = 0; v < total; ++v)
    for_deps(v, [&](int64_t w) {
      ++indeg[static_cast<size_t>(v)];
      ++succ_ptr[static_cast<size_t>(w) + 1];
    });
  for (int64_t v = 0; v < total; ++v) succ_ptr[static_cast<size_t>(v) + 1] += succ_ptr[static_cast<size_t>(v)];
  std::vector<int64_t> succ(static_cast<size_t>(succ_ptr.back()));
  {
    std::vector<int64_t> fill(succ_ptr.begin(), succ_ptr.end() - 1);
    for (int64_t v = 0; v < total; ++v)
      for_deps(v, [&](int64_t w) { succ[static_cast<size_t>(fill[static_cast<size_t>(w)]++)] = v; });
  }
  auto key = [&](int64_t v) {
    const int32_t p = static_cast<int32_t>(v / per), r = static_cast<int32_t>(v % per);
    const int64_t row = r < nz ? 0 : L.unit_lo[static_cast<size_t>(ticket_unit[static_cast<size_t>(r - nz)])];
    return row + static_cast<int64_t>(p) * lag_rows;
  };
  using Item = std::pair<int64_t, int64_t>;  // (key, power-major index), smallest first
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> ready;
  std::vector<char> done(static_cast<size_t>(total), 0);
  order.clear();
  order.reserve(static_cast<size_t>(total));
  auto emit = [&](int64_t v) {
    done[static_cast<size_t>(v)] = 1;
    order.push_back(static_cast<int32_t>(v));
    for (int64_t i = succ_ptr[static_cast<size_t>(v)]; i < succ_ptr[static_cast<size_t>(v) + 1]; ++i) {
      const int64_t w = succ[static_cast<size_t>(i)];
      if (--indeg[static_cast<size_t>(w)] == 0 && !(w < n_static)) ready.push({key(w), w});
    }
  };
  // the static prefix: power 0 in its own order, a closed set (its waits
  // point to smaller positions of power 0)
  for (int64_t v = 0; v < n_static && v < total; ++v) {
    if (indeg[static_cast<size_t>(v)] != 0) throw std::logic_error("static ticket waits outside the static prefix");
    emit(v);
  }
  // everything else that waits for nothing (successors of the prefix that
  // became ready are already queued; a repeat is skipped when popped)
  for (int64_t v = n_static; v < total; ++v)
    if (indeg[static_cast<size_t>(v)] == 0) ready.push({key(v), v});
  while (!ready.empty()) {
    const int64_t v = ready.top().second;
    ready.pop();
    if (!done[static_cast<size_t>(v)]) emit(v);
  }
  if (static_cast<int64_t>(order.size()) != total) throw std::logic_error("matrix-power waits form a cycle");
}

void build_read_deps(const Layout& L, std::vector<int32_t>& ptr, std::vector<int32_t>& idx) {
  const int32_t n = L.n;
  const int32_t n_units = static_cast<int32_t>(L.unit_lo.size());
  // touchers of every index: the unit owning the row, then the units holding it in their halo
  std::vector<int64_t> tptr(static_cast<size_t>(n) + 1, 0);
  for (int32_t u = 0; u < n_units; ++u) {
    for (int32_t g = L.unit_lo[u]; g < L.unit_hi[u]; ++g) ++tptr[g + 1];
    for (int32_t j = L.unit_halo_ptr[u]; j < L.unit_halo_ptr[u + 1]; ++j) ++tptr[(L.halo[j] & kIndexMask) + 1];
  }
  for (int32_t g = 0; g < n; ++g) tptr[g + 1] += tptr[g];
  std::vector<int32_t> touchers(static_cast<size_t>(tptr[n]));
  {
    std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
    for (int32_t u = 0; u < n_units; ++u) {
      for (int32_t g = L.unit_lo[u]; g < L.unit_hi[u]; ++g) touchers[fill[g]++] = u;
      for (int32_t j = L.unit_halo_ptr[u]; j < L.unit_halo_ptr[u + 1]; ++j)
        touchers[fill[L.halo[j] & kIndexMask]++] = u;
    }
  }
  ptr.assign(1, 0);
  idx.clear();
  std::vector<int32_t> stamp(static_cast<size_t>(n_units), -1), mine;
  auto add = [&](int32_t u, int32_t g) {
    for (int64_t q = tptr[g]; q < tptr[g + 1]; ++q)
      if (stamp[touchers[q]] != u) {
        stamp[touchers[q]] = u;
        mine.push_back(touchers[q]);
      }
  };
  for (int32_t u = 0; u < n_units; ++u) {
    mine.clear();
    for (int32_t g = L.unit_lo[u]; g < L.unit_hi[u]; ++g) add(u, g);
    for (int32_t j = L.unit_halo_ptr[u]; j < L.unit_halo_ptr[u + 1]; ++j) add(u, static_cast<int32_t>(L.halo[j] & kIndexMask));
    std::sort(mine.begin(), mine.end());
    idx.insert(idx.end(), mine.begin(), mine.end());
    ptr.push_back(static_cast<int32_t>(idx.size()));
  }
}

}  // namespace race
