// Learned cost model: host side (see costmodel.hpp).
#include "costmodel.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <queue>

namespace race {

void mlp_forward_host(const float* theta, const float* X, int64_t n, float* y) {
  const float* W1 = theta;
  const float* b1 = W1 + kMlpHid * kMlpIn;
  const float* W2 = b1 + kMlpHid;
  const float* b2 = W2 + kMlpHid * kMlpHid;
  const float* w3 = b2 + kMlpHid;
  const float b3 = w3[kMlpHid];
  float h1[kMlpHid];
  for (int64_t s = 0; s < n; ++s) {
    const float* x = X + s * kMlpIn;
    for (int j = 0; j < kMlpHid; ++j) {
      float z = b1[j];
      for (int i = 0; i < kMlpIn; ++i) z = std::fma(W1[j * kMlpIn + i], x[i], z);
      h1[j] = z > 0.0f ? z : 0.0f;
    }
    float f = b3;
    for (int o = 0; o < kMlpHid; ++o) {
      float z = b2[o];
      for (int j = 0; j < kMlpHid; ++j) z = std::fma(W2[o * kMlpHid + j], h1[j], z);
      if (z > 0.0f) f = std::fma(w3[o], z, f);
    }
    y[s] = f;
  }
}

namespace {

struct RowStats {
  double sum = 0, sum2 = 0;
  int32_t max = 0;
  void add(int32_t v) {
    sum += v;
    sum2 += static_cast<double>(v) * v;
    max = std::max(max, v);
  }
  double mean(int32_t rows) const { return rows ? sum / rows : 0.0; }
  double cv(int32_t rows) const {
    if (rows == 0 || sum == 0) return 0.0;
    const double m = sum / rows;
    return std::sqrt(std::max(0.0, sum2 / rows - m * m)) / m;
  }
};

void fill_features(float* f, int32_t rows, int64_t nnz, const RowStats& st, int64_t halo, int64_t offd_out,
                   int64_t window, int64_t rmw, int64_t shared, int64_t phase_units, double phase_frac, int32_t k) {
  f[0] = static_cast<float>(std::log2(1.0 + rows));
  f[1] = static_cast<float>(std::log2(1.0 + static_cast<double>(nnz)));
  f[2] = static_cast<float>(st.mean(rows));
  f[3] = static_cast<float>(st.max);
  f[4] = static_cast<float>(st.cv(rows));
  f[5] = rows ? static_cast<float>(static_cast<double>(halo) / rows) : 0.0f;
  f[6] = st.sum > 0 ? static_cast<float>(static_cast<double>(offd_out) / st.sum) : 0.0f;
  f[7] = window ? static_cast<float>(static_cast<double>(rmw) / window) : 0.0f;
  f[8] = window ? static_cast<float>(static_cast<double>(shared) / window) : 0.0f;
  f[9] = static_cast<float>(std::log2(1.0 + static_cast<double>(phase_units)));
  f[10] = static_cast<float>(phase_frac);
  f[11] = static_cast<float>(std::log2(static_cast<double>(k)));
}

}  // namespace

void unit_features(const Layout& L, const Tree& t, int32_t k, std::vector<float>& out) {
  const int32_t n_units = static_cast<int32_t>(L.unit_lo.size());
  out.assign(static_cast<size_t>(n_units) * kMlpIn, 0.0f);
  const std::vector<int32_t>& rp = L.prow_ptr;
  const std::vector<int32_t>& pc = L.pcol;
  for (int32_t u = 0; u < n_units; ++u) {
    const int32_t a = L.unit_lo[u], b = L.unit_hi[u];
    RowStats st;
    int64_t offd_out = 0, rmw = 0, shared = 0;
    for (int32_t r = a; r < b; ++r) {
      int32_t i = rp[r];
      if (i < rp[r + 1] && pc[i] == r) ++i;
      st.add(rp[r + 1] - i);
      for (; i < rp[r + 1]; ++i)
        if (pc[i] >= b) ++offd_out;
      const uint32_t fl = row_flag(L.row_flags, r);
      if (fl & 2u) ++shared;
      else if (!(fl & 1u)) ++rmw;
    }
    const int32_t h0 = L.unit_halo_ptr[u], h1 = L.unit_halo_ptr[u + 1];
    for (int32_t j = h0; j < h1; ++j) {
      if (L.halo[j] & kSharedBit) ++shared;
      else if (!(L.halo[j] & kFirstBit)) ++rmw;
    }
    const int32_t ph = t.leaf_phase[L.unit_leaf[u]];
    fill_features(&out[static_cast<size_t>(u) * kMlpIn], b - a, static_cast<int64_t>(rp[b]) - rp[a], st, h1 - h0,
                  offd_out, static_cast<int64_t>(b - a) + (h1 - h0), rmw, shared,
                  L.phase_unit_ptr[ph + 1] - L.phase_unit_ptr[ph], static_cast<double>(ph) / t.n_phases, k);
  }
}

double simulate(const Layout& L, const float* cost, double flush_frac, int32_t workers,
                const std::vector<int32_t>& order) {
  const int32_t n_units = static_cast<int32_t>(L.unit_lo.size());
  std::vector<double> finish(static_cast<size_t>(n_units), 0.0);
  std::priority_queue<double, std::vector<double>, std::greater<double>> free_at;
  for (int32_t w = 0; w < std::max(1, workers); ++w) free_at.push(0.0);
  double end = 0.0;
  for (int32_t i = 0; i < n_units; ++i) {
    const int32_t u = order.empty() ? i : order[static_cast<size_t>(i)];
    const double start = free_at.top();
    free_at.pop();
    double ready = start + (1.0 - flush_frac) * cost[u];
    // edges to clearing tasks (index >= n_units) count as met at the start:
    // the tasks hold the first tickets and clear a few KB each
    for (int32_t i = L.dep_ptr[u]; i < L.dep_ptr[u + 1]; ++i)
      if (L.dep_idx[i] < n_units) ready = std::max(ready, finish[L.dep_idx[i]]);
    finish[u] = ready + flush_frac * cost[u];
    free_at.push(finish[u]);
    end = std::max(end, finish[u]);
  }
  return end;
}

void learned_row_loads(const Graph& g, int32_t n, const int32_t* row_ptr, const int32_t* col, const float* theta,
                       int32_t window_max, int32_t root_mode, int32_t level_order, std::vector<int64_t>& m) {
  m.assign(static_cast<size_t>(n), 1);
  if (n == 0) return;
  // stage-0 levels and order, as the tree builder finds them
  std::vector<int32_t> lev, order, pos(static_cast<size_t>(n));
  stage0_order(g, root_mode, level_order, lev, order);
  int32_t nl = 0;
  for (int32_t v = 0; v < n; ++v) nl = std::max(nl, lev[v] + 1);
  std::vector<int32_t> level_ptr(static_cast<size_t>(nl) + 1, 0);
  for (int32_t v = 0; v < n; ++v) ++level_ptr[lev[v] + 1];
  for (int32_t l = 0; l < nl; ++l) level_ptr[l + 1] += level_ptr[l];
  for (int32_t p = 0; p < n; ++p) pos[order[p]] = p;
  std::vector<uint8_t> has_diag(static_cast<size_t>(n), 0);
  for (int32_t r = 0; r < n; ++r)
    if (row_ptr[r] < row_ptr[r + 1] && col[row_ptr[r]] == r) has_diag[r] = 1;
  // pieces: greedy position ranges of one level whose window fits
  struct Piece {
    int32_t a, b;
  };
  std::vector<Piece> pieces;
  std::vector<float> feats;
  std::vector<uint8_t> marked(static_cast<size_t>(n), 0);
  std::vector<int32_t> mark_list;
  auto upper_offd = [&](int32_t v) {
    int32_t c = 0;
    for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) c += pos[g.adj[e]] > pos[v];
    return c;
  };
  for (int32_t l = 0; l < nl; ++l) {
    int32_t a = level_ptr[l];
    while (a < level_ptr[l + 1]) {
      int64_t w = 0;
      int32_t b = a;
      while (b < level_ptr[l + 1]) {
        const int32_t v = order[b];
        int64_t new_h = 0;
        for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
          const int32_t u = g.adj[e];
          if (pos[u] > b && !marked[pos[u]]) ++new_h;
        }
        const int64_t w_new = w + (marked[b] ? 0 : 1) + new_h;
        if (w_new > window_max && b > a) break;
        if (!marked[b]) {
          marked[b] = 1;
          mark_list.push_back(b);
        }
        for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
          const int32_t q = pos[g.adj[e]];
          if (q > b && !marked[q]) {
            marked[q] = 1;
            mark_list.push_back(q);
          }
        }
        w = w_new;
        ++b;
      }
      for (int32_t q : mark_list) marked[q] = 0;
      mark_list.clear();
      pieces.push_back({a, b});
      a = b;
    }
  }
  const int64_t n_pieces = static_cast<int64_t>(pieces.size());
  feats.assign(static_cast<size_t>(n_pieces) * kMlpIn, 0.0f);
  for (int64_t i = 0; i < n_pieces; ++i) {
    const int32_t a = pieces[i].a, b = pieces[i].b;
    RowStats st;
    int64_t nnz = 0, offd_out = 0;
    for (int32_t p = a; p < b; ++p) {
      const int32_t v = order[p];
      const int32_t c = upper_offd(v);
      st.add(c);
      nnz += c + has_diag[v];
      for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
        const int32_t q = pos[g.adj[e]];
        if (q >= b) {
          ++offd_out;
          if (!marked[q]) {
            marked[q] = 1;
            mark_list.push_back(q);
          }
        }
      }
    }
    const int64_t halo = static_cast<int64_t>(mark_list.size());
    for (int32_t q : mark_list) marked[q] = 0;
    mark_list.clear();
    // schedule-dependent features at neutral values: no read-modify-write
    // or shared flushes, half of the pieces concurrent, first phase, k = 1
    fill_features(&feats[static_cast<size_t>(i) * kMlpIn], b - a, nnz, st, halo, offd_out, (b - a) + halo, 0, 0,
                  n_pieces / 2, 0.0, 1);
  }
  std::vector<float> pred(static_cast<size_t>(n_pieces));
  mlp_forward_host(theta, feats.data(), n_pieces, pred.data());
  for (int64_t i = 0; i < n_pieces; ++i) {
    const int32_t a = pieces[i].a, b = pieces[i].b;
    const double cost_ns = 1000.0 * std::exp(std::min(30.0, static_cast<double>(pred[i])));
    double wsum = 0;
    for (int32_t p = a; p < b; ++p) wsum += 1.0 + upper_offd(order[p]);
    for (int32_t p = a; p < b; ++p) {
      const double share = cost_ns * (1.0 + upper_offd(order[p])) / wsum;
      m[order[p]] = std::max<int64_t>(1, std::llround(share));
    }
  }
}

void critical_path_order(const Layout& L, const float* cost, std::vector<int32_t>& order) {
  const int32_t n_units = static_cast<int32_t>(L.unit_lo.size());
  // successors: the units whose edges point to u (edges to clearing tasks
  // carry no order among units)
  std::vector<int32_t> succ_ptr(static_cast<size_t>(n_units) + 1, 0), indeg(static_cast<size_t>(n_units), 0);
  for (int32_t u = 0; u < n_units; ++u)
    for (int32_t i = L.dep_ptr[u]; i < L.dep_ptr[u + 1]; ++i)
      if (L.dep_idx[i] < n_units) {
        ++succ_ptr[L.dep_idx[i] + 1];
        ++indeg[u];
      }
  for (int32_t u = 0; u < n_units; ++u) succ_ptr[u + 1] += succ_ptr[u];
  std::vector<int32_t> succ(static_cast<size_t>(succ_ptr[n_units]));
  {
    std::vector<int32_t> fill(succ_ptr.begin(), succ_ptr.end() - 1);
    for (int32_t u = 0; u < n_units; ++u)
      for (int32_t i = L.dep_ptr[u]; i < L.dep_ptr[u + 1]; ++i)
        if (L.dep_idx[i] < n_units) succ[fill[L.dep_idx[i]]++] = u;
  }
  // edges point to smaller units, so successors have larger indices
  std::vector<double> bl(static_cast<size_t>(n_units), 0.0);
  for (int32_t u = n_units - 1; u >= 0; --u) {
    double m = 0.0;
    for (int32_t i = succ_ptr[u]; i < succ_ptr[u + 1]; ++i) m = std::max(m, bl[succ[i]]);
    bl[u] = static_cast<double>(cost[u]) + m;
  }
  auto lower = [&](int32_t a, int32_t b) { return bl[a] < bl[b] || (bl[a] == bl[b] && a > b); };
  std::priority_queue<int32_t, std::vector<int32_t>, decltype(lower)> ready(lower);
  for (int32_t u = 0; u < n_units; ++u)
    if (indeg[u] == 0) ready.push(u);
  order.clear();
  order.reserve(static_cast<size_t>(n_units));
  while (!ready.empty()) {
    const int32_t u = ready.top();
    ready.pop();
    order.push_back(u);
    for (int32_t i = succ_ptr[u]; i < succ_ptr[u + 1]; ++i)
      if (--indeg[succ[i]] == 0) ready.push(succ[i]);
  }
}

}  // namespace race
