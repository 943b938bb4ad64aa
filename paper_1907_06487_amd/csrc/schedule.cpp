// RACE schedule construction (Section 4): BFS levels, permutation, distance-2
// level groups, epsilon aggregation with worker counts, load balancing,
// recursion on T + N(T), phases, effective rows and eta (Section 5).
//
// Built without floating-point contraction: every double below is rounded
// in the order written, so the schedule is reproducible bit for bit.
#include "schedule.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <numeric>

namespace race {

void build_graph(int32_t n, const int32_t* row_ptr, const int32_t* col, Graph& g) {
  g.n = n;
  std::vector<int64_t> deg(static_cast<size_t>(n) + 1, 0);
  for (int32_t r = 0; r < n; ++r)
    for (int32_t i = row_ptr[r]; i < row_ptr[r + 1]; ++i) {
      const int32_t c = col[i];
      if (c == r) continue;
      ++deg[r];
      ++deg[c];
    }
  g.ptr.assign(static_cast<size_t>(n) + 1, 0);
  for (int32_t v = 0; v < n; ++v) g.ptr[v + 1] = g.ptr[v] + deg[v];
  g.adj.resize(static_cast<size_t>(g.ptr[n]));
  std::vector<int64_t> fill(g.ptr.begin(), g.ptr.end() - 1);
  for (int32_t r = 0; r < n; ++r)
    for (int32_t i = row_ptr[r]; i < row_ptr[r + 1]; ++i) {
      const int32_t c = col[i];
      if (c == r) continue;
      g.adj[fill[r]++] = c;
      g.adj[fill[c]++] = r;
    }
}

void row_loads(int32_t n, const int32_t* row_ptr, const int32_t* col, bool by_rows, std::vector<int64_t>& m) {
  m.assign(static_cast<size_t>(n), by_rows ? 1 : 0);
  if (by_rows) return;
  for (int32_t r = 0; r < n; ++r) {
    m[r] += row_ptr[r + 1] - row_ptr[r];
    for (int32_t i = row_ptr[r]; i < row_ptr[r + 1]; ++i)
      if (col[i] != r) ++m[col[i]];
  }
}

// ---------------------------------------------------------------------------
// Section 4.4.3 steps 1-3

std::vector<Pair> aggregate_pairs(const std::vector<int64_t>& m_levels, int64_t n_t, double eps_s, int32_t k) {
  const int32_t nl = static_cast<int32_t>(m_levels.size());
  int64_t m_total = 0;
  for (int64_t m : m_levels) m_total += m;
  std::vector<Pair> pairs;
  if (m_total == 0) return pairs;
  const double mt = static_cast<double>(m_total);
  std::vector<double> w(static_cast<size_t>(nl));
  for (int32_t i = 0; i < nl; ++i) w[i] = (static_cast<double>(m_levels[i]) * static_cast<double>(n_t)) / mt;
  int32_t start = 0;
  while (start < nl) {
    double a = 0.0;
    int32_t i = start;
    int64_t b = 0;
    bool qualified = false;
    while (i < nl) {
      a += w[i];
      ++i;
      if (i - start >= 2 * k) {
        b = std::max<int64_t>(1, static_cast<int64_t>(std::floor(a + 0.5)));
        const double eps = 1.0 - std::fabs(a - static_cast<double>(b));
        if (eps > eps_s) {
          qualified = true;
          break;
        }
      }
    }
    if (qualified) {
      const double bd = static_cast<double>(b);
      while (i < nl) {
        const double a2 = a + w[i];
        if (a2 > bd) break;
        if (!((1.0 - std::fabs(a2 - bd)) > (1.0 - std::fabs(a - bd)))) break;
        a = a2;
        ++i;
      }
      pairs.push_back({start, i, b});
      start = i;
    } else {
      if (nl - start >= 2 * k) {
        pairs.push_back({start, nl, std::max<int64_t>(1, static_cast<int64_t>(std::floor(a + 0.5)))});
      } else if (!pairs.empty()) {
        pairs.back().end = nl;
      } else {
        return {};
      }
      start = nl;
    }
  }
  if (pairs.size() < 2) return {};
  return pairs;
}

// Section 4.4.3 step 4: the two groups of a pair share their workers and are
// balanced against each other by single-level moves that strictly lower
// |load(red) - load(blue)|, starting from red = first ceil(n/2) levels.
void split_pairs(const std::vector<Pair>& pairs, const std::vector<int64_t>& m_levels, int32_t k,
                 std::vector<int32_t>& t_ptr, std::vector<int64_t>& worker) {
  t_ptr.clear();
  worker.clear();
  t_ptr.push_back(pairs.front().start);
  for (const Pair& p : pairs) {
    int32_t r = p.start + (p.end - p.start + 1) / 2;
    int64_t red = 0, blue = 0;
    for (int32_t l = p.start; l < r; ++l) red += m_levels[l];
    for (int32_t l = r; l < p.end; ++l) blue += m_levels[l];
    for (;;) {
      if (red > blue && r - p.start > k) {
        const int64_t x = m_levels[r - 1];
        if (std::llabs((red - x) - (blue + x)) < std::llabs(red - blue)) {
          red -= x;
          blue += x;
          --r;
          continue;
        }
      } else if (blue > red && p.end - r > k) {
        const int64_t x = m_levels[r];
        if (std::llabs((red + x) - (blue - x)) < std::llabs(red - blue)) {
          red += x;
          blue -= x;
          ++r;
          continue;
        }
      }
      break;
    }
    t_ptr.push_back(r);
    t_ptr.push_back(p.end);
    worker.push_back(p.b);
    worker.push_back(p.b);
  }
}

// Section 4.3, Algorithm "Load Balancing" with worker counts.
static double lb_variance(const std::vector<int32_t>& t_ptr, const std::vector<int64_t>& worker,
                          const std::vector<int64_t>& prefix, std::vector<double>& diff) {
  const size_t ng = worker.size();
  std::vector<double> per(ng);
  for (size_t i = 0; i < ng; ++i) {
    const int64_t load = prefix[t_ptr[i + 1]] - prefix[t_ptr[i]];
    per[i] = static_cast<double>(load) / static_cast<double>(worker[i]);
  }
  double s_r = 0.0, s_b = 0.0;
  int64_t n_r = 0, n_b = 0;
  for (size_t i = 0; i < ng; ++i) {
    if (i % 2 == 0) {
      s_r += per[i];
      ++n_r;
    } else {
      s_b += per[i];
      ++n_b;
    }
  }
  const double mean_r = s_r / static_cast<double>(n_r);
  const double mean_b = s_b / static_cast<double>(n_b);
  diff.resize(ng);
  for (size_t i = 0; i < ng; ++i) diff[i] = per[i] - (i % 2 == 0 ? mean_r : mean_b);
  double var = 0.0;
  for (size_t i = 0; i < ng; ++i) {
    const double d2 = diff[i] * diff[i];
    var += d2;
  }
  return var / static_cast<double>(ng);
}

static void shift_levels(std::vector<int32_t>& t, int32_t donor, int32_t receiver) {
  if (receiver < donor) {
    for (int32_t j = receiver + 1; j <= donor; ++j) t[j] += 1;
  } else {
    for (int32_t j = donor + 1; j <= receiver; ++j) t[j] -= 1;
  }
}

void load_balance(std::vector<int32_t>& t_ptr, const std::vector<int64_t>& worker, const std::vector<int64_t>& m_levels,
                  int32_t k) {
  std::vector<int64_t> prefix(m_levels.size() + 1, 0);
  for (size_t i = 0; i < m_levels.size(); ++i) prefix[i + 1] = prefix[i] + m_levels[i];
  const int32_t ng = static_cast<int32_t>(worker.size());
  std::vector<double> diff, diff2;
  std::vector<int32_t> abs_rank(ng), rank(ng), cand;
  for (;;) {
    const double var = lb_variance(t_ptr, worker, prefix, diff);
    std::vector<double> negabs(ng);
    for (int32_t i = 0; i < ng; ++i) negabs[i] = -std::fabs(diff[i]);
    std::iota(abs_rank.begin(), abs_rank.end(), 0);
    std::stable_sort(abs_rank.begin(), abs_rank.end(), [&](int32_t a, int32_t b) { return negabs[a] < negabs[b]; });
    std::iota(rank.begin(), rank.end(), 0);
    std::stable_sort(rank.begin(), rank.end(), [&](int32_t a, int32_t b) { return diff[a] < diff[b]; });
    bool improved = false;
    for (int32_t cr = 0; cr < ng; ++cr) {
      const int32_t g = abs_rank[cr];
      int32_t donor = -1, receiver = -1;
      if (diff[g] < 0) {
        for (int32_t t = ng - 1; t >= 0; --t) {
          const int32_t el = rank[t];
          if (t_ptr[el + 1] - t_ptr[el] > k) {
            donor = el;
            break;
          }
        }
        receiver = g;
      } else if (t_ptr[g + 1] - t_ptr[g] > k) {
        donor = g;
        receiver = rank[0];
      }
      if (donor < 0 || donor == receiver) continue;
      cand = t_ptr;
      shift_levels(cand, donor, receiver);
      const double new_var = lb_variance(cand, worker, prefix, diff2);
      if (new_var < var) {
        t_ptr = cand;
        improved = true;
        break;
      }
    }
    if (!improved) return;
  }
}

// ---------------------------------------------------------------------------
// recursion

// Rooted level structure of the component of `root` (Section 4.1): fills
// dist, records the visited vertices in `seen` and the last level in `last`
// (ascending); returns the eccentricity of the root.
static int32_t level_structure(const Graph& g, int32_t root, std::vector<int32_t>& dist, std::vector<int32_t>& seen,
                               std::vector<int32_t>& last) {
  std::vector<int32_t> frontier(1, root), next;
  dist[root] = 0;
  seen.push_back(root);
  int32_t d = 0;
  last = frontier;
  while (!frontier.empty()) {
    last = frontier;
    next.clear();
    for (int32_t v : frontier)
      for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
        const int32_t u = g.adj[e];
        if (dist[u] < 0) {
          dist[u] = d + 1;
          seen.push_back(u);
          next.push_back(u);
        }
      }
    ++d;
    frontier.swap(next);
  }
  std::sort(last.begin(), last.end());
  return d - 1;
}

// George and Liu's pseudo-peripheral node finder: from the current vertex
// r, take a vertex x of minimum degree in the last level of r's rooted
// level structure (the lowest index among equals); while x's eccentricity
// exceeds r's, continue from x.  Returns the last x.
int32_t pseudo_peripheral(const Graph& g, int32_t start, std::vector<int32_t>& dist) {
  std::vector<int32_t> seen, last, last_x;
  auto reset = [&]() {
    for (int32_t v : seen) dist[v] = -1;
    seen.clear();
  };
  int32_t ecc_r = level_structure(g, start, dist, seen, last);
  reset();
  for (;;) {
    int32_t x = last[0];
    int64_t best = g.ptr[x + 1] - g.ptr[x];
    for (int32_t v : last) {
      const int64_t dv = g.ptr[v + 1] - g.ptr[v];
      if (dv < best) {
        best = dv;
        x = v;
      }
    }
    const int32_t ecc_x = level_structure(g, x, dist, seen, last_x);
    reset();
    if (ecc_x <= ecc_r) return x;
    ecc_r = ecc_x;
    last.swap(last_x);
  }
}

void stage0_order(const Graph& g, int32_t root_mode, int32_t level_order, std::vector<int32_t>& lev,
                  std::vector<int32_t>& order) {
  const int32_t n = g.n;
  lev.assign(static_cast<size_t>(n), -1);
  order.clear();
  order.reserve(static_cast<size_t>(n));
  std::vector<int32_t> pp_dist, frontier, next, grp;
  if (root_mode == 1) pp_dist.assign(static_cast<size_t>(n), -1);
  int32_t cur_max = -1;
  for (int32_t first = 0; first < n; ++first) {
    if (lev[first] >= 0) continue;
    const int32_t root = root_mode == 1 ? pseudo_peripheral(g, first, pp_dist) : first;
    int32_t lvl = cur_max < 0 ? 0 : cur_max + 2;
    lev[root] = lvl;
    order.push_back(root);
    frontier.assign(1, root);
    while (!frontier.empty()) {
      cur_max = std::max(cur_max, lvl);
      next.clear();
      for (int32_t v : frontier) {
        grp.clear();
        for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
          const int32_t u = g.adj[e];
          if (lev[u] < 0) {
            lev[u] = lvl + 1;
            grp.push_back(u);
          }
        }
        // Cuthill-McKee: a vertex's new neighbours by increasing degree
        if (level_order == 1)
          std::stable_sort(grp.begin(), grp.end(), [&](int32_t a, int32_t b) {
            return g.ptr[a + 1] - g.ptr[a] < g.ptr[b + 1] - g.ptr[b];
          });
        next.insert(next.end(), grp.begin(), grp.end());
      }
      order.insert(order.end(), next.begin(), next.end());
      ++lvl;
      frontier.swap(next);
    }
  }
  if (level_order == 0) {
    // keep the input order inside every level: stable sort by level
    std::vector<int32_t> cnt(static_cast<size_t>(cur_max) + 2, 0);
    for (int32_t v = 0; v < n; ++v) ++cnt[lev[v] + 1];
    for (size_t l = 1; l < cnt.size(); ++l) cnt[l] += cnt[l - 1];
    for (int32_t v = 0; v < n; ++v) order[cnt[lev[v]]++] = v;
  }
}

namespace {

struct Builder {
  const Graph& g;
  const std::vector<int64_t>& m_row;
  const TreeParams& p;
  std::vector<int32_t> perm;
  std::vector<TreeNode> nodes;
  std::vector<int32_t> scratch;   // BFS level per vertex, -1 = unvisited
  std::vector<uint8_t> in_sub;    // membership of the current subgraph
  std::vector<int32_t> touched, frontier, next, sub_list;
  int32_t n_levels0 = 0;

  Builder(const Graph& g_, const std::vector<int64_t>& m_, const TreeParams& p_)
      : g(g_), m_row(m_), p(p_), perm(static_cast<size_t>(g_.n)), scratch(static_cast<size_t>(g_.n), -1),
        in_sub(static_cast<size_t>(g_.n), 0) {
    std::iota(perm.begin(), perm.end(), 0);
  }

  double eps_for(int32_t stage) const { return p.eps[stage < 8 ? stage : 7]; }

  // BFS distances inside the subgraph (all vertices when `all`), roots taken
  // from `members` in order, islands two levels above the largest so far.
  void bfs(const int32_t* members, int32_t nm, bool all, std::vector<int32_t>& lev) {
    int32_t cur_max = -1;
    int32_t q = 0;
    for (;;) {
      while (q < nm && scratch[members[q]] >= 0) ++q;
      if (q >= nm) break;
      const int32_t root = members[q];
      int32_t lvl = cur_max < 0 ? 0 : cur_max + 2;
      scratch[root] = lvl;
      touched.push_back(root);
      frontier.assign(1, root);
      while (!frontier.empty()) {
        cur_max = std::max(cur_max, lvl);
        next.clear();
        for (int32_t v : frontier)
          for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
            const int32_t u = g.adj[e];
            if ((all || in_sub[u]) && scratch[u] < 0) {
              scratch[u] = lvl + 1;
              touched.push_back(u);
              next.push_back(u);
            }
          }
        ++lvl;
        frontier.swap(next);
      }
    }
    lev.resize(static_cast<size_t>(nm));
    for (int32_t i = 0; i < nm; ++i) lev[i] = scratch[members[i]];
    for (int32_t t : touched) scratch[t] = -1;
    touched.clear();
  }

  void refine(int32_t nid) {
    const int32_t lo = nodes[nid].lo, hi = nodes[nid].hi, stage = nodes[nid].stage;
    const int64_t b = nodes[nid].workers;
    const int32_t nm = hi - lo;
    if (nm == 0) return;
    std::vector<int32_t> members(perm.begin() + lo, perm.begin() + hi);
    std::vector<int32_t> lev;
    const bool all = stage < 0;
    if (!all) {
      // the recursion subgraph: T and every vertex within distance k - 1 of
      // it, so no outside vertex can join two of T's vertices at distance k
      sub_list.clear();
      for (int32_t v : members)
        if (!in_sub[v]) { in_sub[v] = 1; sub_list.push_back(v); }
      size_t f0 = 0;
      for (int32_t d = 1; d < p.dist_k; ++d) {
        const size_t f1 = sub_list.size();
        for (size_t q = f0; q < f1; ++q) {
          const int32_t v = sub_list[q];
          for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
            const int32_t u = g.adj[e];
            if (!in_sub[u]) { in_sub[u] = 1; sub_list.push_back(u); }
          }
        }
        f0 = f1;
      }
    }
    if (all) {
      // stage 0: the whole graph, its island roots and in-level order by the
      // parameters; members follow the level order found
      std::vector<int32_t> lev_v;
      stage0_order(g, p.root_mode, p.level_order, lev_v, members);
      lev.resize(static_cast<size_t>(nm));
      for (int32_t i = 0; i < nm; ++i) lev[i] = lev_v[members[i]];
    } else {
      bfs(members.data(), nm, all, lev);
      for (int32_t v : sub_list) in_sub[v] = 0;
    }
    int32_t nl = 0;
    for (int32_t l : lev) nl = std::max(nl, l + 1);
    std::vector<int64_t> m_levels(static_cast<size_t>(nl), 0);
    std::vector<int32_t> counts(static_cast<size_t>(nl), 0);
    for (int32_t i = 0; i < nm; ++i) {
      m_levels[lev[i]] += m_row[members[i]];
      ++counts[lev[i]];
    }
    if (all) n_levels0 = nl;
    const std::vector<Pair> pairs = aggregate_pairs(m_levels, b, eps_for(stage + 1), p.dist_k);
    if (pairs.empty()) return;
    // stable counting sort of the members by level
    std::vector<int32_t> level_ptr(static_cast<size_t>(nl) + 1, 0);
    for (int32_t l = 0; l < nl; ++l) level_ptr[l + 1] = level_ptr[l] + counts[l];
    std::vector<int32_t> fill(level_ptr.begin(), level_ptr.end() - 1);
    for (int32_t i = 0; i < nm; ++i) perm[lo + fill[lev[i]]++] = members[i];
    std::vector<int32_t> t_ptr;
    std::vector<int64_t> worker;
    split_pairs(pairs, m_levels, p.dist_k, t_ptr, worker);
    if (p.global_lb) load_balance(t_ptr, worker, m_levels, p.dist_k);
    nodes[nid].n_levels = nl;
    std::vector<int32_t> kids;
    for (size_t gi = 0; gi < worker.size(); ++gi) {
      TreeNode c;
      c.stage = stage + 1;
      c.color = static_cast<int32_t>(gi % 2);
      c.lo = lo + level_ptr[t_ptr[gi]];
      c.hi = lo + level_ptr[t_ptr[gi + 1]];
      c.workers = static_cast<int32_t>(std::min<int64_t>(worker[gi], INT32_MAX));
      c.parent = nid;
      nodes.push_back(c);
      kids.push_back(static_cast<int32_t>(nodes.size()) - 1);
    }
    nodes[nid].children = kids;
    for (int32_t cid : kids)
      if (nodes[cid].workers > 1 && nodes[cid].stage + 1 < p.max_stages) refine(cid);
  }
};

}  // namespace

std::string build_tree(const Graph& g, const std::vector<int64_t>& row_load, const TreeParams& p, Tree& out) {
  if (p.dist_k < 1 || p.dist_k > 8) return "dist_k must be in 1..8";
  if (p.n_workers < 1) return "n_workers must be >= 1";
  if (p.max_stages < 1 || p.max_stages > 16) return "max_stages must be in 1..16";
  Builder bld(g, row_load, p);
  TreeNode root;
  root.stage = -1;
  root.lo = 0;
  root.hi = g.n;
  root.workers = p.n_workers;
  bld.nodes.push_back(root);
  bld.refine(0);

  // preorder renumbering
  std::vector<int32_t> order;
  std::function<void(int32_t)> visit = [&](int32_t i) {
    order.push_back(i);
    for (int32_t c : bld.nodes[i].children) visit(c);
  };
  visit(0);
  std::vector<int32_t> remap(bld.nodes.size());
  for (size_t i = 0; i < order.size(); ++i) remap[order[i]] = static_cast<int32_t>(i);
  out = Tree();
  out.n = g.n;
  out.n_workers = p.n_workers;
  out.perm = std::move(bld.perm);
  out.n_levels0 = bld.n_levels0;
  out.nodes.resize(order.size());
  for (size_t i = 0; i < order.size(); ++i) {
    TreeNode nd = bld.nodes[order[i]];
    nd.parent = nd.parent >= 0 ? remap[nd.parent] : -1;
    for (int32_t& c : nd.children) c = remap[c];
    out.nodes[i] = std::move(nd);
  }
  std::vector<int32_t> leaves;
  int32_t depth = -1;
  for (size_t i = 0; i < out.nodes.size(); ++i)
    if (out.nodes[i].children.empty()) {
      leaves.push_back(static_cast<int32_t>(i));
      depth = std::max(depth, out.nodes[i].stage);
    }
  std::vector<int32_t> phase(leaves.size());
  std::vector<int32_t> bits;
  for (size_t t = 0; t < leaves.size(); ++t) {
    bits.clear();
    for (int32_t j = leaves[t]; out.nodes[j].parent >= 0; j = out.nodes[j].parent) bits.push_back(out.nodes[j].color);
    std::reverse(bits.begin(), bits.end());
    int32_t ph = 0;
    for (int32_t s = 0; s <= depth; ++s) ph = ph * 2 + (s < static_cast<int32_t>(bits.size()) ? bits[s] : 0);
    phase[t] = ph;
  }
  std::vector<int32_t> idx(leaves.size());
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) {
    if (phase[a] != phase[b]) return phase[a] < phase[b];
    if (out.nodes[leaves[a]].lo != out.nodes[leaves[b]].lo) return out.nodes[leaves[a]].lo < out.nodes[leaves[b]].lo;
    return leaves[a] < leaves[b];
  });
  for (int32_t t : idx) {
    out.leaves.push_back(leaves[t]);
    out.leaf_phase.push_back(phase[t]);
  }
  out.depth = depth;
  out.n_phases = depth >= 0 ? (1 << (depth + 1)) : 1;

  std::function<int32_t(int32_t)> n_eff = [&](int32_t i) -> int32_t {
    const TreeNode& nd = out.nodes[i];
    if (nd.children.empty()) return nd.hi - nd.lo;
    int32_t r = 0, bl = 0;
    for (int32_t c : nd.children) {
      const int32_t e = n_eff(c);
      if (out.nodes[c].color == 0) r = std::max(r, e);
      else bl = std::max(bl, e);
    }
    return r + bl;
  };
  out.n_eff_root = n_eff(0);
  out.eta = out.n_eff_root > 0
                ? static_cast<double>(g.n) / (static_cast<double>(out.n_eff_root) * static_cast<double>(p.n_workers))
                : 1.0;
  return std::string();
}

}  // namespace race
