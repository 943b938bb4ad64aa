// Host construction of the Gauss-Seidel layout (see gauss_seidel.hpp).
#include "gauss_seidel.hpp"

#include <algorithm>
#include <stdexcept>
#include <string>

#include "../../include/race.h"

namespace race {

std::string build_gs_layout(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                            const Tree& tree, GsLayout& L, int* code, bool kaczmarz) {
  L = GsLayout();
  L.n = n;
  *code = RACE_OK;
  std::vector<int32_t> inv(static_cast<size_t>(n));
  for (int32_t i = 0; i < n; ++i) inv[tree.perm[i]] = i;
  // full permuted rows: every stored off-diagonal (r, c) appears in the rows
  // of both ends
  const int64_t nnz_u = n > 0 ? row_ptr[n] : 0;
  std::vector<int64_t> cnt(static_cast<size_t>(n) + 1, 0);
  L.diag.assign(static_cast<size_t>(n), 0.0);
  std::vector<char> has_diag(static_cast<size_t>(n), 0);
  for (int32_t r = 0; r < n; ++r)
    for (int32_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
      if (col[k] == r) {
        L.diag[inv[r]] = val[k];
        has_diag[inv[r]] = 1;
      } else {
        ++cnt[inv[r] + 1];
        ++cnt[inv[col[k]] + 1];
      }
    }
  for (int32_t i = 0; i < n && !kaczmarz; ++i)
    if (!has_diag[i] || L.diag[i] == 0.0) {
      *code = RACE_EINVAL;
      return "Gauss-Seidel needs a nonzero stored diagonal in every row (row " + std::to_string(tree.perm[i]) +
             " of the input)";
    }
  for (int32_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  if (cnt[n] >= (int64_t(1) << 31)) {
    *code = RACE_EUNSUPPORTED;
    return "the full matrix has 2^31 or more off-diagonal entries";
  }
  (void)nnz_u;
  std::vector<int32_t> pcol(static_cast<size_t>(cnt[n]));
  std::vector<double> pval(static_cast<size_t>(cnt[n]));
  {
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int32_t r = 0; r < n; ++r)
      for (int32_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
        const int32_t c = col[k];
        if (c == r) continue;
        const int32_t a = inv[r], b = inv[c];
        pcol[fill[a]] = b;
        pval[fill[a]++] = val[k];
        pcol[fill[b]] = a;
        pval[fill[b]++] = val[k];
      }
  }
  // columns ascending within every row
  {
    std::vector<std::pair<int32_t, double>> tmp;
    for (int32_t i = 0; i < n; ++i) {
      tmp.clear();
      for (int64_t k = cnt[i]; k < cnt[i + 1]; ++k) tmp.emplace_back(pcol[k], pval[k]);
      std::sort(tmp.begin(), tmp.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
      for (size_t t = 0; t < tmp.size(); ++t) {
        pcol[cnt[i] + static_cast<int64_t>(t)] = tmp[t].first;
        pval[cnt[i] + static_cast<int64_t>(t)] = tmp[t].second;
      }
      L.max_row = std::max<int32_t>(L.max_row, static_cast<int32_t>(tmp.size()));
    }
  }
  L.row_ptr.assign(cnt.begin(), cnt.end());
  L.val = std::move(pval);
  L.slot.assign(L.val.size(), 0);
  // leaves in execution order, their halos and window slots
  const size_t nl = tree.leaves.size();
  L.phase_leaf_ptr.assign(static_cast<size_t>(tree.n_phases) + 1, 0);
  L.phase_max_window.assign(static_cast<size_t>(tree.n_phases), 0);
  L.halo_ptr.assign(nl + 1, 0);
  std::vector<int32_t> hl;
  for (size_t t = 0; t < nl; ++t) {
    const TreeNode& nd = tree.nodes[tree.leaves[t]];
    const int32_t lo = nd.lo, hi = nd.hi, R = hi - lo;
    L.leaf_lo.push_back(lo);
    L.leaf_hi.push_back(hi);
    ++L.phase_leaf_ptr[tree.leaf_phase[t] + 1];
    hl.clear();
    for (int64_t k = cnt[lo]; k < cnt[hi]; ++k)
      if (pcol[k] < lo || pcol[k] >= hi) hl.push_back(pcol[k]);
    std::sort(hl.begin(), hl.end());
    hl.erase(std::unique(hl.begin(), hl.end()), hl.end());
    const int64_t window = static_cast<int64_t>(R) + static_cast<int64_t>(hl.size());
    if (window > kGsMaxWindow) {
      *code = RACE_EUNSUPPORTED;
      return "a leaf of " + std::to_string(R) + " rows reads " + std::to_string(hl.size()) +
             " rows outside it: its window exceeds " + std::to_string(kGsMaxWindow) +
             " entries; rebuild with more n_workers or more stages";
    }
    for (int64_t k = cnt[lo]; k < cnt[hi]; ++k) {
      const int32_t c = pcol[k];
      L.slot[k] = static_cast<uint16_t>(
          c >= lo && c < hi ? c - lo : R + (std::lower_bound(hl.begin(), hl.end(), c) - hl.begin()));
    }
    L.halo.insert(L.halo.end(), hl.begin(), hl.end());
    L.halo_ptr[t + 1] = static_cast<int32_t>(L.halo.size());
    L.max_window = std::max<int32_t>(L.max_window, static_cast<int32_t>(window));
    int32_t& pm = L.phase_max_window[tree.leaf_phase[t]];
    pm = std::max<int32_t>(pm, static_cast<int32_t>(window));
  }
  for (int32_t p = 0; p < tree.n_phases; ++p) L.phase_leaf_ptr[p + 1] += L.phase_leaf_ptr[p];
  L.halo_total = static_cast<int64_t>(L.halo.size());
  if (kaczmarz) {
    L.nrm.assign(static_cast<size_t>(n), 0.0);
    for (int32_t i = 0; i < n; ++i) {
      double q = 0.0;
      bool diag_done = !has_diag[i];
      for (int64_t k = cnt[i]; k < cnt[i + 1]; ++k) {
        if (!diag_done && pcol[k] > i) {
          q += L.diag[i] * L.diag[i];
          diag_done = true;
        }
        q += L.val[k] * L.val[k];
      }
      if (!diag_done) q += L.diag[i] * L.diag[i];
      L.nrm[i] = q;
    }
    // windows of one phase must not overlap (leaves are sorted by phase)
    std::vector<int32_t> owner(static_cast<size_t>(n), -1);
    for (int32_t p = 0; p < tree.n_phases; ++p) {
      const int32_t l0 = L.phase_leaf_ptr[p], l1 = L.phase_leaf_ptr[p + 1];
      auto claim = [&](int32_t r, int32_t t) {
        if (owner[r] >= l0 && owner[r] != t) return false;
        owner[r] = t;
        return true;
      };
      for (int32_t t = l0; t < l1; ++t) {
        bool ok = true;
        for (int32_t r = L.leaf_lo[t]; r < L.leaf_hi[t] && ok; ++r) ok = claim(r, t);
        for (int32_t h = L.halo_ptr[t]; h < L.halo_ptr[t + 1] && ok; ++h) ok = claim(L.halo[h], t);
        if (!ok) {
          *code = RACE_EINTERNAL;
          return "two leaves of phase " + std::to_string(p) +
                 " share a row of their windows: the schedule is not distance-2 independent";
        }
      }
    }
  }
  return "";
}

void build_gs_flow(const GsLayout& G, int32_t direction, GsFlow& f) {
  const int32_t nl = static_cast<int32_t>(G.leaf_lo.size());
  const int32_t np = static_cast<int32_t>(G.phase_leaf_ptr.size()) - 1;
  f = GsFlow{};
  f.direction = direction;
  // phase of every leaf; items of up to kGsFlowLeaves leaves inside a phase
  std::vector<int32_t> leaf_phase(static_cast<size_t>(nl)), leaf_item(static_cast<size_t>(nl));
  std::vector<int32_t> phase_item_ptr(static_cast<size_t>(np) + 1, 0);
  for (int32_t p = 0; p < np; ++p) {
    phase_item_ptr[static_cast<size_t>(p)] = static_cast<int32_t>(f.item_leaf0.size());
    for (int32_t l = G.phase_leaf_ptr[static_cast<size_t>(p)]; l < G.phase_leaf_ptr[static_cast<size_t>(p) + 1];
         l += kGsFlowLeaves) {
      const int32_t cnt = std::min(kGsFlowLeaves, G.phase_leaf_ptr[static_cast<size_t>(p) + 1] - l);
      for (int32_t i = 0; i < cnt; ++i) {
        leaf_phase[static_cast<size_t>(l + i)] = p;
        leaf_item[static_cast<size_t>(l + i)] = static_cast<int32_t>(f.item_leaf0.size());
      }
      f.item_leaf0.push_back(l);
      f.item_count.push_back(cnt);
    }
  }
  phase_item_ptr[static_cast<size_t>(np)] = static_cast<int32_t>(f.item_leaf0.size());
  const int32_t ni = static_cast<int32_t>(f.item_leaf0.size());
  // leaf of every row (leaves cover the rows as disjoint ranges)
  std::vector<int32_t> row_leaf(static_cast<size_t>(G.n), -1);
  for (int32_t l = 0; l < nl; ++l)
    for (int32_t r = G.leaf_lo[static_cast<size_t>(l)]; r < G.leaf_hi[static_cast<size_t>(l)]; ++r)
      row_leaf[static_cast<size_t>(r)] = l;
  // tickets
  std::vector<int32_t> fwd_ticket(static_cast<size_t>(ni), -1), bwd_ticket(static_cast<size_t>(ni), -1);
  if (direction != 1)
    for (int32_t i = 0; i < ni; ++i) {
      fwd_ticket[static_cast<size_t>(i)] = static_cast<int32_t>(f.ticket_item.size());
      f.ticket_item.push_back(i);
      f.ticket_back.push_back(0);
    }
  if (direction != 0)
    for (int32_t p = np - 1; p >= 0; --p)
      for (int32_t i = phase_item_ptr[static_cast<size_t>(p)]; i < phase_item_ptr[static_cast<size_t>(p) + 1]; ++i) {
        bwd_ticket[static_cast<size_t>(i)] = static_cast<int32_t>(f.ticket_item.size());
        f.ticket_item.push_back(i);
        f.ticket_back.push_back(1);
      }
  // waits
  const int32_t nt = static_cast<int32_t>(f.ticket_item.size());
  f.dep_ptr.assign(static_cast<size_t>(nt) + 1, 0);
  std::vector<int32_t> deps;
  for (int32_t t = 0; t < nt; ++t) {
    const int32_t i = f.ticket_item[static_cast<size_t>(t)];
    const bool back = f.ticket_back[static_cast<size_t>(t)] != 0;
    deps.clear();
    if (back && direction == 2) deps.push_back(fwd_ticket[static_cast<size_t>(i)]);
    for (int32_t l = f.item_leaf0[static_cast<size_t>(i)];
         l < f.item_leaf0[static_cast<size_t>(i)] + f.item_count[static_cast<size_t>(i)]; ++l) {
      const int32_t p = leaf_phase[static_cast<size_t>(l)];
      for (int32_t h = G.halo_ptr[static_cast<size_t>(l)]; h < G.halo_ptr[static_cast<size_t>(l) + 1]; ++h) {
        const int32_t m = row_leaf[static_cast<size_t>(G.halo[static_cast<size_t>(h)])];
        const int32_t q = leaf_phase[static_cast<size_t>(m)];
        if (q == p) throw std::logic_error("Gauss-Seidel dataflow: two leaves of one phase share an edge");
        if (!back && q < p) deps.push_back(fwd_ticket[static_cast<size_t>(leaf_item[static_cast<size_t>(m)])]);
        if (back && q > p) deps.push_back(bwd_ticket[static_cast<size_t>(leaf_item[static_cast<size_t>(m)])]);
      }
    }
    std::sort(deps.begin(), deps.end());
    deps.erase(std::unique(deps.begin(), deps.end()), deps.end());
    for (const int32_t d : deps)
      if (d < 0 || d >= t) throw std::logic_error("Gauss-Seidel dataflow: a wait that does not point backwards");
    f.dep_idx.insert(f.dep_idx.end(), deps.begin(), deps.end());
    f.dep_ptr[static_cast<size_t>(t) + 1] = static_cast<int32_t>(f.dep_idx.size());
  }
}

void build_kacz_flow(const GsLayout& K, int32_t direction, GsFlow& f) {
  const int32_t nl = static_cast<int32_t>(K.leaf_lo.size());
  const int32_t np = static_cast<int32_t>(K.phase_leaf_ptr.size()) - 1;
  f = GsFlow{};
  f.direction = direction;
  for (int32_t l = 0; l < nl; ++l) {
    f.item_leaf0.push_back(l);
    f.item_count.push_back(1);
  }
  if (direction != 1)
    for (int32_t l = 0; l < nl; ++l) {
      f.ticket_item.push_back(l);
      f.ticket_back.push_back(0);
    }
  if (direction != 0)
    for (int32_t p = np - 1; p >= 0; --p)
      for (int32_t l = K.phase_leaf_ptr[static_cast<size_t>(p)]; l < K.phase_leaf_ptr[static_cast<size_t>(p) + 1]; ++l) {
        f.ticket_item.push_back(l);
        f.ticket_back.push_back(1);
      }
  const int32_t nt = static_cast<int32_t>(f.ticket_item.size());
  f.dep_ptr.assign(static_cast<size_t>(nt) + 1, 0);
  std::vector<int32_t> last(static_cast<size_t>(K.n), -1), deps;
  for (int32_t t = 0; t < nt; ++t) {
    const int32_t l = f.ticket_item[static_cast<size_t>(t)];
    deps.clear();
    auto touch = [&](int32_t r) {
      int32_t& w = last[static_cast<size_t>(r)];
      if (w >= 0) deps.push_back(w);
      w = t;
    };
    for (int32_t r = K.leaf_lo[static_cast<size_t>(l)]; r < K.leaf_hi[static_cast<size_t>(l)]; ++r) touch(r);
    for (int32_t h = K.halo_ptr[static_cast<size_t>(l)]; h < K.halo_ptr[static_cast<size_t>(l) + 1]; ++h)
      touch(K.halo[static_cast<size_t>(h)]);
    std::sort(deps.begin(), deps.end());
    deps.erase(std::unique(deps.begin(), deps.end()), deps.end());
    for (const int32_t d : deps)
      if (d >= t) throw std::logic_error("Kaczmarz dataflow: a wait that does not point backwards");
    f.dep_idx.insert(f.dep_idx.end(), deps.begin(), deps.end());
    f.dep_ptr[static_cast<size_t>(t) + 1] = static_cast<int32_t>(f.dep_idx.size());
  }
}

}  // namespace race
