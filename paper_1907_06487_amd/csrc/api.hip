// C ABI of librace.so (declared in include/race.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/race.h"
#include "costmodel.hpp"
#include "errors.hpp"
#include "gauss_seidel.hpp"
#include "gs_kernels.hpp"
#include "kernels.hpp"
#include "layout.hpp"
#include "schedule.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return RACE_EHIP;
}

// Upper-triangle CRS: row_ptr[0] == 0, non-decreasing, columns strictly
// ascending inside a row and in [row, n).  `upper` false: any column in [0, n).
int validate_crs(int32_t n, const int32_t* row_ptr, const int32_t* col, bool upper) {
  if (n < 0) return fail(RACE_EINVAL, "n must be >= 0");
  if (!row_ptr) return fail(RACE_EINVAL, "row_ptr is NULL");
  if (row_ptr[0] != 0) return fail(RACE_EINVAL, "row_ptr[0] must be 0");
  for (int32_t r = 0; r < n; ++r)
    if (row_ptr[r + 1] < row_ptr[r]) return fail(RACE_EINVAL, "row_ptr decreases at row " + std::to_string(r));
  if (n > 0 && row_ptr[n] > 0 && !col) return fail(RACE_EINVAL, "col is NULL");
  for (int32_t r = 0; r < n; ++r) {
    for (int32_t i = row_ptr[r]; i < row_ptr[r + 1]; ++i) {
      const int32_t c = col[i];
      if (c < (upper ? r : 0) || c >= n)
        return fail(RACE_EINVAL, "column " + std::to_string(c) + " of row " + std::to_string(r) +
                                     (upper ? " is not in [row, n)" : " is out of range"));
      if (i > row_ptr[r] && c <= col[i - 1])
        return fail(RACE_EINVAL, "columns of row " + std::to_string(r) + " are not strictly ascending");
    }
  }
  return RACE_OK;
}

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t count = 0;
};

template <typename T>
hipError_t upload(DevBuf<T>& b, const T* host, size_t count, int64_t* total) {
  b.count = count;
  if (count == 0) return hipSuccess;
  hipError_t e = hipMalloc(&b.p, count * sizeof(T));
  if (e != hipSuccess) return e;
  *total += static_cast<int64_t>(count * sizeof(T));
  return hipMemcpy(b.p, host, count * sizeof(T), hipMemcpyHostToDevice);
}

template <typename T>
void release(DevBuf<T>& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.count = 0;
}

}  // namespace

namespace race {
int set_error(int code, const std::string& msg) { return fail(code, msg); }
int set_hip_error(hipError_t e, const char* what) { return hip_fail(e, what); }
}  // namespace race

// Claim words per CU for the dataflow launch's static tickets: at least the
// workgroups one CU can hold (32 wavefronts).
constexpr int32_t kClaimsPerCu = 32;

struct race_schedule {
  race_params params{};
  race::Tree tree;
  race::Layout L;
  race_stats stats{};
  bool has_values = false;
  bool uploaded = false;
  int device = -1;
  DevBuf<int32_t> leaf_units, chunk_len, new2old, dep_idx;
  DevBuf<race::UnitDesc> unit_desc;
  // ticket order of the dataflow product (units by ticket; empty: the
  // layout's execution order) and its device copies with the inverse
  std::vector<int32_t> ticket_unit;
  DevBuf<int32_t> ticket_unit_d, unit_ticket_d;
  DevBuf<uint32_t> flow_state;  // done[n_units + n_zero_tasks], status, padding, counter (64-bit, 8-byte aligned)
  DevBuf<uint32_t> claims;      // claim words of static tickets (32 per CU), then the takeover count
  int32_t late_stride = 0;      // tests only (race_schedule_flow_test_late)
  uint32_t epoch = 0;
  uint64_t ticket_next = 0;
  int32_t n_cus = 0;
  // Gauss-Seidel phases with at least this many leaves run four leaves per
  // wavefront: -1 the default (32 x CUs), -2 never, >= 0 that count
  int32_t gs_quad_min = -1;
  // Gauss-Seidel execution: 0 one launch per phase, 1 one dataflow launch
  // per sweep (plans per direction, built on first use); flags of the
  // tickets (set to the launch's epoch), then the status word
  int32_t gs_exec = 0;
  race::GsFlow gs_flow_h[3];
  DevBuf<int32_t> gsf_item[3], gsf_back[3], gsf_leaf0[3], gsf_count[3], gsf_dptr[3], gsf_didx[3];
  DevBuf<uint32_t> gsf_flags;
  uint32_t gs_epoch = 0;
  // distance-2 schedules built with race_params.kaczmarz: the Kaczmarz
  // sweep layout and its device copies
  bool kz = false;
  race::GsLayout KG;
  DevBuf<int32_t> kz_leaf_lo, kz_leaf_hi, kz_halo_ptr, kz_halo, kz_row_ptr;
  DevBuf<uint16_t> kz_slot;
  DevBuf<double> kz_val, kz_diag, kz_nrm;
  DevBuf<uint32_t> halo, row_flags, chunk_off;
  DevBuf<int32_t> zero_idx;
  DevBuf<uint16_t> lane_slot, sell_slot;
  DevBuf<double> lane_diag64, sell_val64;
  DevBuf<float> lane_diag32, sell_val32;
  DevBuf<race::Cplx<false>> lane_diagc, sell_valc;  // complex values (value_type 2 or 3)
  DevBuf<double> tiles_x, tiles_y;  // column tiles of X and Y for products with many passes (grown on demand)
  // matrix powers: read dependencies (host and device, built on first use)
  // and the launch state (P * flags + counter), grown on demand
  std::vector<int32_t> rdep_ptr_h, rdep_idx_h;
  DevBuf<int32_t> rdep_ptr, rdep_idx;
  DevBuf<uint32_t> mpk_state;
  uint64_t mpk_ticket_next = 0;
  // matrix-power ticket order (race_schedule_set_mpk_order): lag < 0 is
  // power-major; else the diagonal order, cached for one (powers, static
  // tickets) pair
  int64_t mpk_lag = -1;
  int32_t mpk_cache = 0;
  std::vector<int32_t> mpk_order_h;
  int32_t mpk_order_P = 0, mpk_order_static = -1;
  DevBuf<int32_t> mpk_order_d;
  // the full permuted matrix in CRS, when single-vector products run as a
  // CRS product (race_params.low_locality)
  bool expanded = false;
  int32_t exp_per = 0;   // entries per thread of its row blocks
  int32_t exp_nblk = 0;  // row blocks
  int32_t exp_nblk2 = 0; // row blocks of the SpMM with 2..4 columns
  int32_t exp_nblk3 = 0; // row blocks of the SpMM with 5..16 columns
  DevBuf<int32_t> exp_rp, exp_col, exp_blk, exp_blk2, exp_blk3;
  DevBuf<double> exp_val64;
  DevBuf<float> exp_val32;
  // distance-1 schedules: the Gauss-Seidel layout and its device copies
  bool gs = false;
  race::GsLayout G;
  DevBuf<int32_t> gs_leaf_lo, gs_leaf_hi, gs_halo_ptr, gs_halo, gs_row_ptr;
  DevBuf<uint16_t> gs_slot;
  DevBuf<double> gs_val, gs_diag;

  void free_device() {
    release(gs_leaf_lo); release(gs_leaf_hi); release(gs_halo_ptr); release(gs_halo); release(gs_row_ptr);
    release(gs_slot); release(gs_val); release(gs_diag);
    release(kz_leaf_lo); release(kz_leaf_hi); release(kz_halo_ptr); release(kz_halo); release(kz_row_ptr);
    release(kz_slot); release(kz_val); release(kz_diag); release(kz_nrm);
    for (int d = 0; d < 3; ++d) {
      release(gsf_item[d]); release(gsf_back[d]); release(gsf_leaf0[d]); release(gsf_count[d]);
      release(gsf_dptr[d]); release(gsf_didx[d]);
      gs_flow_h[d].direction = -1;
    }
    release(gsf_flags);
    release(leaf_units); release(unit_desc); release(ticket_unit_d); release(unit_ticket_d);
    release(chunk_len); release(new2old); release(halo); release(row_flags); release(chunk_off);
    release(zero_idx);
    release(lane_slot); release(sell_slot); release(lane_diag64); release(sell_val64); release(lane_diag32);
    release(sell_val32); release(lane_diagc); release(sell_valc); release(dep_idx); release(flow_state); release(claims); release(tiles_x); release(tiles_y);
    release(exp_rp); release(exp_col); release(exp_blk); release(exp_blk2); release(exp_blk3); release(exp_val64); release(exp_val32);
    release(rdep_ptr); release(rdep_idx); release(mpk_state); release(mpk_order_d);
    uploaded = false;
  }
};

struct race_csr {
  int32_t n = 0;
  int32_t lpr = 8;     // lanes per row, or (negative) row blocks of -lpr entries per thread
  int32_t n_blk = 0;   // row blocks (lpr < 0)
  bool atomic = false;
  int device = -1;
  DevBuf<int32_t> rp, col, blk;
  DevBuf<double> val;
};

struct race_batch {
  int32_t count = 0;
  int32_t k = 1;
  int32_t kt = 1;  // right-hand sides per pass
  bool tiled = false;  // four or more passes: through contiguous column tiles
  int32_t value_type = 0;
  int32_t threads = 256;
  int32_t grid = 0;
  int32_t wmax = 1;
  int32_t n_tickets = 0;
  int device = -1;
  std::vector<race_schedule_t> mats;
  std::vector<int64_t> unit_base;  // offset of each matrix's done flags in the state
  DevBuf<int32_t> ticket_mat, ticket_unit;
  DevBuf<uint32_t> state;
  DevBuf<double> tiles_x, tiles_y;  // every matrix's column tiles (tiled runs), matrix m at tile_base[m]
  std::vector<int64_t> tile_base;
  void* d_mats = nullptr;          // BatchMat<ValT>[count]
  // members whose product is the expanded one: no tickets; with k = 1 one
  // row-block launch over all their blocks, with k > 1 a CRS SpMM each
  std::vector<int32_t> exp_members;
  std::vector<const double*> exp_x;  // their X and Y (bound)
  std::vector<double*> exp_y;
  int32_t n_exp_blocks = 0;
  DevBuf<int32_t> blk_mat;
  void* d_bmats = nullptr;         // BlockMat<ValT>[exp_members.size()]
  bool bound = false;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

const char* race_last_error(void) { return g_err.c_str(); }

int race_params_default(race_params* p) {
  if (!p) return fail(RACE_EINVAL, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->dist_k = 2;
  p->n_workers = 1024;
  p->max_stages = 4;
  p->balance_by = 0;
  p->global_lb = 0;
  p->value_type = 0;
  p->window_max = 3840;
  p->block_threads = 256;
  const double eps[8] = {0.8, 0.8, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5};
  for (int i = 0; i < 8; ++i) p->eps[i] = eps[i];
  p->cost_model = nullptr;
  p->cost_model_len = 0;
  p->exec_mode = 1;
  p->shared_atomics = 1;
  p->rhs_tile = 0;
  p->root_mode = 0;
  p->level_order = 0;
  p->low_locality = 0;
  p->kaczmarz = 0;
  return RACE_OK;
}

int race_build_schedule(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                        const race_params* p, race_schedule_t* out) {
  if (!out) return fail(RACE_EINVAL, "out is NULL");
  *out = nullptr;
  race_params prm;
  if (p) prm = *p;
  else race_params_default(&prm);
  if (prm.dist_k < 1 || prm.dist_k > 8) return fail(RACE_EINVAL, "dist_k must be in 1..8");
  if (prm.dist_k == 1 && prm.value_type != 0)
    return fail(RACE_EUNSUPPORTED, "distance-1 schedules (Gauss-Seidel sweeps) take float64 values only");
  if (prm.n_workers < 1) return fail(RACE_EINVAL, "n_workers must be >= 1");
  if (prm.max_stages < 1 || prm.max_stages > 16) return fail(RACE_EINVAL, "max_stages must be in 1..16");
  if (prm.balance_by < 0 || prm.balance_by > 2)
    return fail(RACE_EINVAL, "balance_by must be 0 (nonzeros), 1 (rows) or 2 (cost model)");
  if (prm.balance_by == 2 && (!prm.cost_model || prm.cost_model_len != race::kMlpParams))
    return fail(RACE_EINVAL, "balance_by 2 needs cost_model with RACE_MLP_PARAMS floats");
  if (prm.value_type < 0 || prm.value_type > 3) return fail(RACE_EINVAL, "value_type must be in 0..3");
  const bool cplx = prm.value_type >= 2;
  if (cplx && prm.exec_mode != 1)
    return fail(RACE_EUNSUPPORTED, "complex values run in the dataflow mode (exec_mode 1) only");
  if (prm.exec_mode < 0 || prm.exec_mode > 1) return fail(RACE_EINVAL, "exec_mode must be 0 or 1");
  if (prm.shared_atomics < 0 || prm.shared_atomics > 1) return fail(RACE_EINVAL, "shared_atomics must be 0 or 1");
  if (prm.rhs_tile < 0 || prm.rhs_tile > 16) return fail(RACE_EINVAL, "rhs_tile must be in 0..16");
  if (prm.root_mode < 0 || prm.root_mode > 1) return fail(RACE_EINVAL, "root_mode must be 0 or 1");
  if (prm.level_order < 0 || prm.level_order > 1) return fail(RACE_EINVAL, "level_order must be 0 or 1");
  if (prm.low_locality < 0 || prm.low_locality > 2) return fail(RACE_EINVAL, "low_locality must be 0, 1 or 2");
  if (prm.kaczmarz < 0 || prm.kaczmarz > 1) return fail(RACE_EINVAL, "kaczmarz must be 0 or 1");
  if (prm.kaczmarz && (prm.dist_k < 2 || prm.value_type > 1))
    return fail(RACE_EUNSUPPORTED, "Kaczmarz sweeps need a distance-2 (or wider) schedule of real values");
  if (prm.window_max == 0) prm.window_max = 3840;
  if (prm.window_max < 2 || prm.window_max > 8000) return fail(RACE_EINVAL, "window_max must be in 2..8000");
  if (prm.block_threads == 0) prm.block_threads = 256;
  if (prm.block_threads != 64 && prm.block_threads != 128 && prm.block_threads != 256 && prm.block_threads != 512 &&
      prm.block_threads != 1024)
    return fail(RACE_EINVAL, "block_threads must be 64, 128, 256, 512 or 1024");
  for (int i = 0; i < 8; ++i)
    if (!(prm.eps[i] >= 0.0 && prm.eps[i] < 1.0)) return fail(RACE_EINVAL, "eps values must be in [0, 1)");
  int rc = validate_crs(n, row_ptr, col, true);
  if (rc) return rc;
  race_schedule* s = new (std::nothrow) race_schedule();
  if (!s) return fail(RACE_ENOMEM, "out of host memory");
  try {
    s->params = prm;
    race::Graph g;
    race::build_graph(n, row_ptr, col, g);
    std::vector<int64_t> m;
    if (prm.balance_by == 2)
      race::learned_row_loads(g, n, row_ptr, col, prm.cost_model, prm.window_max, prm.root_mode, prm.level_order, m);
    else
      race::row_loads(n, row_ptr, col, prm.balance_by == 1, m);
    race::TreeParams tp;
    tp.n_workers = prm.n_workers;
    tp.max_stages = prm.max_stages;
    tp.dist_k = prm.dist_k;
    tp.global_lb = prm.global_lb != 0;
    tp.root_mode = prm.root_mode;
    tp.level_order = prm.level_order;
    for (int i = 0; i < 8; ++i) tp.eps[i] = prm.eps[i];
    std::string err = race::build_tree(g, m, tp, s->tree);
    if (!err.empty()) {
      delete s;
      return fail(RACE_EINVAL, err);
    }
    int code = RACE_OK;
    if (prm.dist_k == 1) {
      // a distance-1 coloring serves Gauss-Seidel sweeps; its leaves may
      // share scatter targets, so no SymmSpMV layout is built
      s->gs = true;
      if (val) {
        err = race::build_gs_layout(n, row_ptr, col, val, s->tree, s->G, &code);
        if (!err.empty()) {
          delete s;
          return fail(code, err);
        }
      }
    }
    // complex values arrive as interleaved (re, im) pairs
    std::vector<double> v_re, v_im;
    if (cplx && val) {
      const int64_t nnz = row_ptr[n];
      v_re.resize(static_cast<size_t>(nnz));
      v_im.resize(static_cast<size_t>(nnz));
      for (int64_t i = 0; i < nnz; ++i) {
        v_re[i] = val[2 * i];
        v_im[i] = val[2 * i + 1];
      }
    }
    if (!s->gs)
      err = race::build_layout(n, row_ptr, col, cplx ? (val ? v_re.data() : nullptr) : val,
                               cplx ? (val ? v_im.data() : nullptr) : nullptr, s->tree, prm.window_max,
                               prm.value_type, prm.shared_atomics != 0, s->L, &code);
    if (!err.empty()) {
      delete s;
      return fail(code, err);
    }
    if (prm.kaczmarz && val) {
      // rows of one distance-2 phase share no column, so their Kaczmarz
      // projections commute
      err = race::build_gs_layout(n, row_ptr, col, val, s->tree, s->KG, &code, true);
      if (!err.empty()) {
        delete s;
        return fail(code, err);
      }
      s->kz = true;
      s->stats.kacz_max_window = s->KG.max_window;
    }
    s->has_values = val != nullptr;
    s->params.cost_model = nullptr;  // borrowed for the build only
    s->params.cost_model_len = 0;
    race_stats& st = s->stats;
    const race::Tree& t = s->tree;
    const race::Layout& L = s->L;
    st.n = n;
    st.n_levels0 = t.n_levels0;
    st.depth = t.depth;
    st.n_nodes = static_cast<int32_t>(t.nodes.size());
    st.n_leaves = static_cast<int32_t>(t.leaves.size());
    st.n_phases = t.n_phases;
    int32_t used = 0;
    {
      // phases holding a leaf (the leaves are sorted by phase)
      int32_t last = -1;
      for (const int32_t ph : t.leaf_phase)
        if (ph != last) {
          ++used;
          last = ph;
        }
    }
    st.n_phases_used = used;
    st.n_units = static_cast<int32_t>(L.unit_lo.size());
    st.max_window = s->gs ? s->G.max_window : L.max_window;
    st.n_chunks = static_cast<int32_t>(L.chunk_len.size());
    st.n_eff_root = t.n_eff_root;
    st.n_workers = prm.n_workers;
    st.eta = t.eta;
    st.nnz_upper = n > 0 ? row_ptr[n] : 0;
    if (s->gs) {
      int64_t nd = 0;
      for (int32_t r = 0; r < n; ++r) nd += row_ptr[r + 1] > row_ptr[r] && col[row_ptr[r]] == r;
      st.n_diag = nd;
    } else {
      st.n_diag = L.n_diag;
    }
    st.nnz_full = 2 * st.nnz_upper - st.n_diag;
    st.sell_elems = static_cast<int64_t>(L.sell_val.size());
    st.halo_total = s->gs ? s->G.halo_total : L.halo_total;
    st.rows_rmw = L.rows_rmw;
    st.halo_rmw = L.halo_rmw;
    st.bytes_min = 12 * st.nnz_upper + 20 * static_cast<int64_t>(n) + 4;
    const int64_t vb = prm.value_type == 1 ? 4 : (cplx ? 16 : 8);
    // slices: value + 2-byte slot per element; per lane: slot + diagonal;
    // per slice: offset + length; per unit: 4 ints; halo: index;
    // unit descriptors (32 B), conflict edges (index and flag), x: own rows
    // + halo read once; y: own rows + halo written, RMW and atomic touches
    // read; cleared entries: index read, zero written.
    st.shared_touches = L.shared_touches;
    st.n_zeroed = static_cast<int64_t>(L.zero_idx.size());
    st.bytes_kernel = st.sell_elems * (vb + 2) + static_cast<int64_t>(st.n_chunks) * (8 + race::kSlice * (2 + vb)) +
                      static_cast<int64_t>(st.n_units) * 32 + static_cast<int64_t>(L.dep_idx.size()) * 8 +
                      st.halo_total * 4 +
                      (static_cast<int64_t>(n) + 15) / 16 * 4 +
                      8 * (static_cast<int64_t>(n) + st.halo_total) + 8 * (static_cast<int64_t>(n) + st.halo_total) +
                      8 * (st.rows_rmw + st.halo_rmw + st.shared_touches) + 12 * st.n_zeroed;
    st.device_bytes = 0;
    st.n_deps = static_cast<int64_t>(L.dep_idx.size());
    st.flow_grid = 0;
    st.exec_mode = prm.exec_mode;
    // no reuse in the windows: most touches of y are shared entries, added
    // with global atomics; a CRS product of the expanded matrix needs none
    const int64_t touches = static_cast<int64_t>(n) + st.halo_total;
    s->expanded = !s->gs && prm.value_type <= 1 && n > 0 &&
                  (prm.low_locality == 2 || (prm.low_locality == 1 && 2 * st.shared_touches > touches));
    st.product_path = s->expanded ? 1 : 0;
    st.expanded_per_thread = s->expanded ? race::kExpandedPerThread : 0;
    st.n_zero_tasks = L.n_zero_tasks;
    s->exp_per = st.expanded_per_thread;
  } catch (const std::bad_alloc&) {
    delete s;
    return fail(RACE_ENOMEM, "out of host memory while building the schedule");
  } catch (const std::exception& ex) {
    delete s;
    return fail(RACE_EINTERNAL, ex.what());
  }
  *out = s;
  return RACE_OK;
}

}  // extern "C"


// The full permuted matrix in CRS from the permuted upper triangle: every
// off-diagonal entry (r, c) also appears as (c, r); columns ascending.
static void expand_permuted(const race::Layout& L, std::vector<int32_t>& rp, std::vector<int32_t>& col,
                            std::vector<double>& val) {
  const int32_t n = L.n;
  rp.assign(static_cast<size_t>(n) + 1, 0);
  for (int32_t r = 0; r < n; ++r)
    for (int32_t i = L.prow_ptr[r]; i < L.prow_ptr[r + 1]; ++i) {
      ++rp[r + 1];
      if (L.pcol[i] != r) ++rp[L.pcol[i] + 1];
    }
  for (int32_t r = 0; r < n; ++r) rp[r + 1] += rp[r];
  col.resize(static_cast<size_t>(rp[n]));
  val.resize(static_cast<size_t>(rp[n]));
  std::vector<int32_t> fill(rp.begin(), rp.end() - 1);
  // rows in ascending order, so each row's lower entries arrive before its
  // own (upper) ones, both ascending: the row ends up sorted
  for (int32_t r = 0; r < n; ++r)
    for (int32_t i = L.prow_ptr[r]; i < L.prow_ptr[r + 1]; ++i) {
      const int32_t c = L.pcol[i];
      col[fill[r]] = c;
      val[fill[r]++] = L.pval[i];
      if (c != r) {
        col[fill[c]] = r;
        val[fill[c]++] = L.pval[i];
      }
    }
}

// The ticket order's device arrays: unit of each ticket and its inverse.
static void ticket_arrays(race_schedule_t s, std::vector<int32_t>& tu, std::vector<int32_t>& ut) {
  const size_t n_units = s->L.unit_lo.size();
  tu.resize(n_units);
  ut.resize(n_units);
  for (size_t i = 0; i < n_units; ++i) tu[i] = s->ticket_unit.empty() ? static_cast<int32_t>(i) : s->ticket_unit[i];
  for (size_t i = 0; i < n_units; ++i) ut[static_cast<size_t>(tu[i])] = static_cast<int32_t>(i);
}

extern "C" {

int race_schedule_upload(race_schedule_t s) {
  if (!s) return fail(RACE_EINVAL, "schedule is NULL");
  if (s->uploaded) return RACE_OK;
  if (!s->has_values) return fail(RACE_ESTATE, "schedule was built from a pattern without values");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  const race::Layout& L = s->L;
  int64_t total = 0;
#define UP(buf, vec)                                               \
  e = upload(s->buf, (vec).data(), (vec).size(), &total);          \
  if (e != hipSuccess) {                                           \
    s->free_device();                                              \
    return hip_fail(e, "upload of " #buf);                         \
  }
  if (s->gs) {
    const race::GsLayout& G = s->G;
    UP(gs_leaf_lo, G.leaf_lo)
    UP(gs_leaf_hi, G.leaf_hi)
    UP(gs_halo_ptr, G.halo_ptr)
    UP(gs_halo, G.halo)
    UP(gs_row_ptr, G.row_ptr)
    UP(gs_slot, G.slot)
    UP(gs_val, G.val)
    {
      // the sweep multiplies by the reciprocal diagonal
      std::vector<double> inv(G.diag.size());
      for (size_t i = 0; i < inv.size(); ++i) inv[i] = 1.0 / G.diag[i];
      UP(gs_diag, inv)
    }
    UP(new2old, s->tree.perm)
    e = hipDeviceGetAttribute(&s->n_cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) {
      s->free_device();
      return hip_fail(e, "hipDeviceGetAttribute");
    }
    s->device = dev;
    s->uploaded = true;
    s->stats.device_bytes = total;
    return RACE_OK;
  }
  if (s->kz) {
    const race::GsLayout& K = s->KG;
    UP(kz_leaf_lo, K.leaf_lo)
    UP(kz_leaf_hi, K.leaf_hi)
    UP(kz_halo_ptr, K.halo_ptr)
    UP(kz_halo, K.halo)
    UP(kz_row_ptr, K.row_ptr)
    UP(kz_slot, K.slot)
    UP(kz_val, K.val)
    UP(kz_diag, K.diag)
    {
      std::vector<double> inv(K.nrm.size());
      for (size_t i = 0; i < inv.size(); ++i) inv[i] = K.nrm[i] > 0.0 ? 1.0 / K.nrm[i] : 0.0;
      UP(kz_nrm, inv)
    }
  }
  UP(leaf_units, L.leaf_units)
  {
    std::vector<race::UnitDesc> desc(L.unit_lo.size());
    for (size_t u = 0; u < desc.size(); ++u)
      desc[u] = race::UnitDesc{L.unit_lo[u],         L.unit_hi[u],         L.unit_halo_ptr[u], L.unit_halo_ptr[u + 1],
                               L.unit_chunk_ptr[u], L.unit_chunk_ptr[u + 1], L.dep_ptr[u],       L.dep_ptr[u + 1]};
    UP(unit_desc, desc)
  }
  UP(chunk_len, L.chunk_len)
  UP(new2old, s->tree.perm)
  UP(halo, L.halo)
  UP(row_flags, L.row_flags)
  UP(zero_idx, L.zero_idx)
  UP(chunk_off, L.chunk_off)
  UP(lane_slot, L.lane_slot)
  UP(sell_slot, L.sell_slot)
  UP(dep_idx, L.dep_idx)
  {
    std::vector<int32_t> tu, ut;
    ticket_arrays(s, tu, ut);
    UP(ticket_unit_d, tu)
    UP(unit_ticket_d, ut)
  }
  {
    // done[] per unit and clearing task, then status, then an aligned 64-bit counter
    const size_t words = (L.unit_lo.size() + static_cast<size_t>(L.n_zero_tasks) + 2 + 1) / 2 * 2 + 2;
    std::vector<uint32_t> zeros(words, 0u);
    UP(flow_state, zeros)
  }
  if (s->expanded) {
    std::vector<int32_t> erp, ecol;
    std::vector<double> eval;
    try {
      expand_permuted(L, erp, ecol, eval);
    } catch (const std::bad_alloc&) {
      s->free_device();
      return fail(RACE_ENOMEM, "out of host memory while expanding the matrix");
    }
    {
      std::vector<int32_t> blk;
      race::csr_row_blocks(static_cast<int32_t>(erp.size()) - 1, erp.data(), s->exp_per, blk);
      s->exp_nblk = static_cast<int32_t>(blk.size()) - 1;
      UP(exp_blk, blk)
      race::csr_row_blocks(static_cast<int32_t>(erp.size()) - 1, erp.data(), race::csr_spmm_block_per(2), blk);
      s->exp_nblk2 = static_cast<int32_t>(blk.size()) - 1;
      UP(exp_blk2, blk)
      race::csr_row_blocks(static_cast<int32_t>(erp.size()) - 1, erp.data(), race::csr_spmm_block_per(16), blk);
      s->exp_nblk3 = static_cast<int32_t>(blk.size()) - 1;
      UP(exp_blk3, blk)
    }
    UP(exp_rp, erp)
    UP(exp_col, ecol)
    if (s->params.value_type == 0) {
      UP(exp_val64, eval)
    } else {
      std::vector<float> e32(eval.begin(), eval.end());
      UP(exp_val32, e32)
    }
  }
  e = hipDeviceGetAttribute(&s->n_cus, hipDeviceAttributeMultiprocessorCount, dev);
  int clock_khz = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) {
    s->free_device();
    return hip_fail(e, "hipDeviceGetAttribute");
  }
  s->stats.wall_clock_hz = static_cast<int64_t>(clock_khz) * 1000;
  {
    std::vector<uint32_t> zeros(static_cast<size_t>(kClaimsPerCu) * s->n_cus + 1, 0u);
    UP(claims, zeros)
  }
  if (s->params.value_type == 0) {
    UP(lane_diag64, L.lane_diag)
    UP(sell_val64, L.sell_val)
  } else if (s->params.value_type >= 2) {
    std::vector<race::Cplx<false>> dc(L.lane_diag.size()), vc(L.sell_val.size());
    for (size_t i = 0; i < dc.size(); ++i) dc[i] = {L.lane_diag[i], L.lane_diag_im[i]};
    for (size_t i = 0; i < vc.size(); ++i) vc[i] = {L.sell_val[i], L.sell_val_im[i]};
    UP(lane_diagc, dc)
    UP(sell_valc, vc)
  } else {
    std::vector<float> d32(L.lane_diag.begin(), L.lane_diag.end());
    std::vector<float> v32(L.sell_val.begin(), L.sell_val.end());
    UP(lane_diag32, d32)
    UP(sell_val32, v32)
  }
#undef UP
  s->device = dev;
  s->uploaded = true;
  s->stats.device_bytes = total;
  return RACE_OK;
}

void race_schedule_destroy(race_schedule_t s) {
  if (!s) return;
  if (s->uploaded) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(s->device);
    s->free_device();
    (void)hipSetDevice(cur);
  }
  delete s;
}

int race_schedule_stats(race_schedule_t s, race_stats* out) {
  if (!s || !out) return fail(RACE_EINVAL, "NULL argument");
  *out = s->stats;
  return RACE_OK;
}

int race_schedule_perm(race_schedule_t s, int32_t* new2old) {
  if (!s || !new2old) return fail(RACE_EINVAL, "NULL argument");
  std::copy(s->tree.perm.begin(), s->tree.perm.end(), new2old);
  return RACE_OK;
}

int race_schedule_tree(race_schedule_t s, int32_t* n_nodes, int32_t* stage, int32_t* color, int32_t* parent,
                       int32_t* lo, int32_t* hi, int32_t* workers) {
  if (!s || !n_nodes) return fail(RACE_EINVAL, "NULL argument");
  const auto& nodes = s->tree.nodes;
  *n_nodes = static_cast<int32_t>(nodes.size());
  for (size_t i = 0; i < nodes.size(); ++i) {
    if (stage) stage[i] = nodes[i].stage;
    if (color) color[i] = nodes[i].color;
    if (parent) parent[i] = nodes[i].parent;
    if (lo) lo[i] = nodes[i].lo;
    if (hi) hi[i] = nodes[i].hi;
    if (workers) workers[i] = nodes[i].workers;
  }
  return RACE_OK;
}

int race_schedule_leaves(race_schedule_t s, int32_t* n_leaves, int32_t* node, int32_t* phase) {
  if (!s || !n_leaves) return fail(RACE_EINVAL, "NULL argument");
  *n_leaves = static_cast<int32_t>(s->tree.leaves.size());
  if (node) std::copy(s->tree.leaves.begin(), s->tree.leaves.end(), node);
  if (phase) std::copy(s->tree.leaf_phase.begin(), s->tree.leaf_phase.end(), phase);
  return RACE_OK;
}

int race_schedule_units(race_schedule_t s, int32_t* n_units, int64_t* n_halo, int32_t* unit_leaf, int32_t* row_lo,
                        int32_t* row_hi, int64_t* halo_ptr, int32_t* halo, uint8_t* halo_flags, uint8_t* row_flags) {
  if (!s || !n_units || !n_halo) return fail(RACE_EINVAL, "NULL argument");
  const race::Layout& L = s->L;
  *n_units = static_cast<int32_t>(L.unit_lo.size());
  *n_halo = static_cast<int64_t>(L.halo.size());
  for (size_t u = 0; u < L.unit_lo.size(); ++u) {
    if (unit_leaf) unit_leaf[u] = L.unit_leaf[u];
    if (row_lo) row_lo[u] = L.unit_lo[u];
    if (row_hi) row_hi[u] = L.unit_hi[u];
  }
  if (halo_ptr)
    for (size_t u = 0; u < L.unit_halo_ptr.size(); ++u) halo_ptr[u] = L.unit_halo_ptr[u];
  for (size_t j = 0; j < L.halo.size(); ++j) {
    if (halo) halo[j] = static_cast<int32_t>(L.halo[j] & race::kIndexMask);
    if (halo_flags)
      halo_flags[j] = static_cast<uint8_t>(((L.halo[j] & race::kFirstBit) ? 1 : 0) | ((L.halo[j] & race::kSharedBit) ? 2 : 0));
  }
  if (row_flags)
    for (int32_t r = 0; r < L.n; ++r) row_flags[r] = static_cast<uint8_t>(race::row_flag(L.row_flags, r));
  return RACE_OK;
}

int race_schedule_zero_list(race_schedule_t s, int64_t* count, int32_t* idx) {
  if (!s || !count) return fail(RACE_EINVAL, "NULL argument");
  *count = static_cast<int64_t>(s->L.zero_idx.size());
  if (idx) std::copy(s->L.zero_idx.begin(), s->L.zero_idx.end(), idx);
  return RACE_OK;
}

int race_schedule_features(race_schedule_t s, int32_t k, float* out) {
  if (!s || !out) return fail(RACE_EINVAL, "NULL argument");
  if (k < 1 || k > 16) return fail(RACE_EINVAL, "k must be in 1..16");
  try {
    std::vector<float> f;
    race::unit_features(s->L, s->tree, k, f);
    std::copy(f.begin(), f.end(), out);
  } catch (const std::bad_alloc&) {
    return fail(RACE_ENOMEM, "out of host memory");
  }
  return RACE_OK;
}

int race_schedule_simulate(race_schedule_t s, const float* cost, double flush_frac, int32_t workers,
                           double* makespan) {
  if (!s || !makespan || (!cost && !s->L.unit_lo.empty())) return fail(RACE_EINVAL, "NULL argument");
  if (!(flush_frac >= 0.0 && flush_frac <= 1.0)) return fail(RACE_EINVAL, "flush_frac must be in [0, 1]");
  if (workers < 1) return fail(RACE_EINVAL, "workers must be >= 1");
  try {
    *makespan = race::simulate(s->L, cost, flush_frac, workers, s->ticket_unit);
  } catch (const std::bad_alloc&) {
    return fail(RACE_ENOMEM, "out of host memory");
  }
  return RACE_OK;
}

int race_schedule_set_ticket_order(race_schedule_t s, const int32_t* ticket_unit) {
  if (!s) return fail(RACE_EINVAL, "schedule is NULL");
  if (s->gs) return fail(RACE_EUNSUPPORTED, "a distance-1 schedule has no dataflow tickets");
  const race::Layout& L = s->L;
  const int32_t n_units = static_cast<int32_t>(L.unit_lo.size());
  std::vector<int32_t> order;
  try {
    if (ticket_unit) {
      // a permutation of the units in which every conflict edge points to an earlier ticket
      std::vector<int32_t> pos(static_cast<size_t>(n_units), -1);
      for (int32_t i = 0; i < n_units; ++i) {
        const int32_t u = ticket_unit[i];
        if (u < 0 || u >= n_units || pos[u] >= 0) return fail(RACE_EINVAL, "ticket_unit is not a permutation of the units");
        pos[u] = i;
      }
      for (int32_t u = 0; u < n_units; ++u)
        for (int32_t i = L.dep_ptr[u]; i < L.dep_ptr[u + 1]; ++i)
          if (L.dep_idx[i] < n_units && pos[L.dep_idx[i]] > pos[u])
            return fail(RACE_EINVAL, "unit " + std::to_string(u) + " would take its ticket before unit " +
                                         std::to_string(L.dep_idx[i]) + ", which it waits for");
      order.assign(ticket_unit, ticket_unit + n_units);
    }
    if (s->uploaded && n_units > 0) {
      std::vector<int32_t> keep;
      keep.swap(s->ticket_unit);
      s->ticket_unit = order;
      std::vector<int32_t> tu, ut;
      ticket_arrays(s, tu, ut);
      hipError_t e = hipDeviceSynchronize();
      if (e == hipSuccess) e = hipMemcpy(s->ticket_unit_d.p, tu.data(), sizeof(int32_t) * tu.size(), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(s->unit_ticket_d.p, ut.data(), sizeof(int32_t) * ut.size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        s->ticket_unit.swap(keep);
        return hip_fail(e, "upload of the ticket order");
      }
    } else {
      s->ticket_unit = order;
    }
  } catch (const std::bad_alloc&) {
    return fail(RACE_ENOMEM, "out of host memory");
  }
  s->mpk_order_P = 0;  // a cached matrix-power order follows the old ticket order
  return RACE_OK;
}

int race_schedule_order_tickets(race_schedule_t s, const float* cost) {
  if (!s) return fail(RACE_EINVAL, "schedule is NULL");
  if (!cost) return race_schedule_set_ticket_order(s, nullptr);
  const int32_t n_units = static_cast<int32_t>(s->L.unit_lo.size());
  for (int32_t u = 0; u < n_units; ++u)
    if (!(cost[u] >= 0.0f) || std::isinf(cost[u])) return fail(RACE_EINVAL, "unit costs must be finite and >= 0");
  std::vector<int32_t> order;
  try {
    race::critical_path_order(s->L, cost, order);
  } catch (const std::bad_alloc&) {
    return fail(RACE_ENOMEM, "out of host memory");
  }
  if (static_cast<int32_t>(order.size()) != n_units) return fail(RACE_EINTERNAL, "conflict edges form a cycle");
  return race_schedule_set_ticket_order(s, order.data());
}

int race_schedule_ticket_order(race_schedule_t s, int32_t* ticket_unit) {
  if (!s || !ticket_unit) return fail(RACE_EINVAL, "NULL argument");
  const size_t n_units = s->L.unit_lo.size();
  for (size_t i = 0; i < n_units; ++i)
    ticket_unit[i] = s->ticket_unit.empty() ? static_cast<int32_t>(i) : s->ticket_unit[i];
  return RACE_OK;
}

int race_schedule_flow_grid(race_schedule_t s, int32_t k, int32_t* grid) {
  if (!s || !grid) return fail(RACE_EINVAL, "NULL argument");
  if (k < 1 || k > 16) return fail(RACE_EINVAL, "k must be in 1..16");
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "device query");
  const int32_t wmax = std::max(1, s->L.max_window);
  int32_t per_cu = 0;
  if (s->params.value_type >= 2)  // a complex product: one vector, two columns
    e = k == 1 ? race::race_flow_occupancy<race::Cplx<false>>(2, s->params.block_threads, wmax, &per_cu)
               : hipErrorInvalidValue;
  else
    e = s->params.value_type == 0 ? race::race_flow_occupancy<double>(k, s->params.block_threads, wmax, &per_cu)
                                  : race::race_flow_occupancy<float>(k, s->params.block_threads, wmax, &per_cu);
  if (e != hipSuccess) return hip_fail(e, "occupancy query");
  const int32_t n_units = static_cast<int32_t>(s->L.unit_lo.size());
  *grid = std::max(1, std::min(n_units, per_cu * cus));
  return RACE_OK;
}

int race_mlp_forward_host(const float* theta, const float* X, int64_t n, float* y) {
  if (n < 0) return fail(RACE_EINVAL, "n must be >= 0");
  if (n > 0 && (!theta || !X || !y)) return fail(RACE_EINVAL, "NULL argument");
  race::mlp_forward_host(theta, X, n, y);
  return RACE_OK;
}

int race_mlp_forward(const float* theta, const float* X, int64_t n, float* y, void* stream) {
  if (n < 0) return fail(RACE_EINVAL, "n must be >= 0");
  if (n == 0) return RACE_OK;
  if (!theta || !X || !y) return fail(RACE_EINVAL, "NULL argument");
  if (n > (int64_t(1) << 31) * 255) return fail(RACE_EUNSUPPORTED, "too many samples for one launch");
  hipError_t e = race::launch_mlp_forward(theta, X, n, y, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "network forward launch");
  return RACE_OK;
}

int race_mlp_workspace(int64_t n, int64_t* floats) {
  if (!floats || n < 1) return fail(RACE_EINVAL, "need n >= 1 and an output");
  *floats = race::mlp_workspace_floats(n);
  return RACE_OK;
}

int race_mlp_loss_grad(const float* theta, const float* X, const float* t, int64_t n, float* workspace, float* grad,
                       float* loss, void* stream) {
  if (n < 1) return fail(RACE_EINVAL, "n must be >= 1");
  if (!theta || !X || !t || !workspace || !grad) return fail(RACE_EINVAL, "NULL argument");
  if (n > (int64_t(1) << 30)) return fail(RACE_EUNSUPPORTED, "at most 2^30 samples per call");
  hipError_t e = race::launch_mlp_loss_grad(theta, X, t, n, workspace, grad, loss, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "network gradient launch");
  return RACE_OK;
}

int race_mlp_adam(float* theta, const float* grad, float* m, float* v, int32_t step, float lr, float beta1, float beta2,
                  float eps, void* stream) {
  if (!theta || !grad || !m || !v) return fail(RACE_EINVAL, "NULL argument");
  if (step < 1) return fail(RACE_EINVAL, "step counts from 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f && lr >= 0.0f))
    return fail(RACE_EINVAL, "need 0 <= beta < 1, eps > 0, lr >= 0");
  const double c1 = 1.0 / (1.0 - std::pow(static_cast<double>(beta1), step));
  const double c2 = 1.0 / (1.0 - std::pow(static_cast<double>(beta2), step));
  hipError_t e = race::launch_mlp_adam(theta, grad, m, v, lr, beta1, beta2, eps, static_cast<float>(c1),
                                       static_cast<float>(c2), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "Adam launch");
  return RACE_OK;
}

}  // extern "C"

template <typename ValT>
static race::UnitArgs<ValT> unit_args(race_schedule_t s, const ValT* diag, const ValT* vals) {
  return race::UnitArgs<ValT>{s->leaf_units.p, s->unit_desc.p, s->halo.p, s->row_flags.p, s->chunk_off.p,
                              s->chunk_len.p,  s->lane_slot.p, diag,      vals,          s->sell_slot.p};
}

// Advances the schedule's launch epoch (shared by products and matrix
// powers, whose claim words are the same); on wrap-around every done flag
// and claim is cleared, so none equals the new epoch.
static hipError_t next_epoch(race_schedule_t s, hipStream_t st) {
  s->epoch += 1;
  if (s->epoch != 0) return hipSuccess;
  const size_t n_flags = s->L.unit_lo.size() + static_cast<size_t>(s->L.n_zero_tasks);
  hipError_t e = hipMemsetAsync(s->flow_state.p, 0, sizeof(uint32_t) * n_flags, st);
  if (e == hipSuccess) e = hipMemsetAsync(s->claims.p, 0, sizeof(uint32_t) * (s->claims.count - 1), st);
  if (e == hipSuccess && s->mpk_state.p) {
    e = hipMemsetAsync(s->mpk_state.p, 0, sizeof(uint32_t) * s->mpk_state.count, st);
    s->mpk_ticket_next = 0;  // the counter lives in that state
  }
  s->epoch = 1;
  return e;
}

template <typename ValT>
static int run_flow(race_schedule_t s, const race::UnitArgs<ValT>& a, int32_t k, const double* x, double* y,
                    int32_t ld, uint64_t* trace, hipStream_t st) {
  const race::Layout& L = s->L;
  const int32_t n_units = static_cast<int32_t>(L.unit_lo.size());
  if (n_units == 0) return RACE_OK;
  // the launch identifies itself by an epoch and a ticket base passed as
  // arguments, against state that lives on the device: a captured launch
  // would replay the same epoch and find every ticket already taken
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(st, &cap);
  if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
  if (cap != hipStreamCaptureStatusNone)
    return fail(RACE_EUNSUPPORTED,
                "the dataflow product cannot be captured into a graph; use race_symm_spmv_noalloc, which resets its "
                "state inside the stream");
  const int32_t wmax = std::max(1, L.max_window);
  int32_t per_cu = 0;
  e = race::race_flow_occupancy<ValT>(k, s->params.block_threads, wmax, &per_cu);
  if (e != hipSuccess) return hip_fail(e, "occupancy query");
  if (per_cu < 1) return fail(RACE_EUNSUPPORTED, "dataflow kernel does not fit a CU with this window and block size");
  // the first tickets clear the y entries whose first touch is a shared atomic add
  const int32_t n_flags = n_units + L.n_zero_tasks;
  const int32_t n_tickets = n_flags;
  const int32_t grid = std::max(1, std::min(n_tickets, per_cu * s->n_cus));
  uint32_t* base = s->flow_state.p;
  const size_t counter_word = s->flow_state.count - 2;
  // static tickets: workgroup b starts on ticket b; the counter serves the rest
  const int32_t n_static = std::min(grid, n_tickets);
  const size_t claim_cap = s->claims.count - 1;
  if (static_cast<size_t>(n_static) > claim_cap) return fail(RACE_EINTERNAL, "more workgroups than claim words");
  race::FlowArgs f{s->dep_idx.p, base, reinterpret_cast<uint64_t*>(base + counter_word), base + n_flags,
                   s->claims.p, s->claims.p + claim_cap, n_static, s->late_stride, trace, n_tickets, n_units,
                   L.n_zero_tasks, race::kZeroChunk, s->zero_idx.p, static_cast<int64_t>(L.zero_idx.size()),
                   s->ticket_unit_d.p, s->unit_ticket_d.p};
  e = next_epoch(s, st);
  if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
  // the counter moves once per counter ticket and once more per workgroup
  // (its last, empty request)
  const uint64_t ticket_base = s->ticket_next;
  s->ticket_next += static_cast<uint64_t>(n_tickets - n_static) + static_cast<uint64_t>(grid);
  s->stats.flow_grid = grid;
  e = race::launch_race_flow<ValT>(a, f, k, x, y, ld, wmax, s->params.block_threads, grid, s->epoch, ticket_base, st);
  if (e != hipSuccess) return hip_fail(e, "RACE dataflow launch");
  return RACE_OK;
}

template <typename ValT>
static int run_phases(race_schedule_t s, const race::UnitArgs<ValT>& a, int32_t k, const double* x, double* y,
                      int32_t ld, uint64_t* trace, hipStream_t st) {
  const race::Layout& L = s->L;
  // a leaf's units run on one workgroup in order, or each on its own
  // workgroup when they combine their shared entries atomically
  const int32_t per_unit = s->params.shared_atomics;
  for (int32_t ph = 0; ph < s->tree.n_phases; ++ph) {
    const std::vector<int32_t>& ptr = per_unit ? L.phase_unit_ptr : L.phase_leaf_ptr;
    const int32_t i0 = ptr[ph], i1 = ptr[ph + 1];
    if (i1 == i0) continue;
    const int32_t wmax = std::max(1, L.phase_max_window[ph]);
    hipError_t e =
        race::launch_race_phase<ValT>(a, i0, i1 - i0, per_unit, k, x, y, ld, wmax, s->params.block_threads, trace, st);
    if (e != hipSuccess) return hip_fail(e, "RACE phase launch");
  }
  return RACE_OK;
}

// Right-hand sides per pass: all k when the unit windows of that many fit
// the LDS (or rhs_tile asks for fewer), else the widest tile that fits.
static int32_t rhs_tile(race_schedule_t s, int32_t k) {
  const size_t lds_limit = 159 * 1024;  // dynamic windows plus the kernels' own few bytes
  const int32_t wmax = std::max(1, s->L.max_window);
  int32_t kt = s->params.rhs_tile > 0 ? std::min(k, s->params.rhs_tile) : k;
  while (kt > 1 && race::window_lds_bytes(wmax, kt) > lds_limit) --kt;
  return race::window_lds_bytes(wmax, kt) > lds_limit ? 0 : kt;
}

static const char* kDist1Product =
    "a distance-1 schedule serves Gauss-Seidel sweeps (race_symm_gs); SymmSpMV needs dist_k >= 2";

// y = A x as a CRS product of the expanded permuted matrix over row blocks
// (schedules whose windows predict no reuse, race_params.low_locality).
static int run_expanded(race_schedule_t s, const double* x, double* y, hipStream_t st) {
  const hipError_t e =
      s->params.value_type == 0
          ? race::launch_csr_block<double>(s->exp_nblk, s->exp_blk.p, s->exp_rp.p, s->exp_col.p, s->exp_val64.p, x, y,
                                           s->exp_per, st)
          : race::launch_csr_block<float>(s->exp_nblk, s->exp_blk.p, s->exp_rp.p, s->exp_col.p, s->exp_val32.p, x, y,
                                          s->exp_per, st);
  if (e != hipSuccess) return hip_fail(e, "expanded CRS product launch");
  return RACE_OK;
}

// Y = A X (k >= 2 columns, row-major) as a CRS SpMM of the expanded
// permuted matrix.
static hipError_t expanded_spmm(race_schedule_t s, int32_t k, const double* x, double* y, hipStream_t st) {
  // row blocks, k products per entry in LDS: blocks of 512 entries up to 4
  // columns, of 256 above
  const int32_t nb = k <= 4 ? s->exp_nblk2 : s->exp_nblk3;
  const int32_t* blk = k <= 4 ? s->exp_blk2.p : s->exp_blk3.p;
  return s->params.value_type == 0
             ? race::launch_csr_block_spmm<double>(nb, blk, s->exp_rp.p, s->exp_col.p, s->exp_val64.p, x, y, k, st)
             : race::launch_csr_block_spmm<float>(nb, blk, s->exp_rp.p, s->exp_col.p, s->exp_val32.p, x, y, k, st);
}

static int run_expanded_spmm(race_schedule_t s, int32_t k, const double* x, double* y, hipStream_t st) {
  const hipError_t e = expanded_spmm(s, k, x, y, st);
  if (e != hipSuccess) return hip_fail(e, "expanded CRS SpMM launch");
  return RACE_OK;
}

static int run_products(race_schedule_t s, int32_t k, const double* x, double* y, uint64_t* trace, void* stream) {
  if (!s) return fail(RACE_EINVAL, "schedule is NULL");
  if (s->gs) return fail(RACE_EUNSUPPORTED, kDist1Product);
  if (!s->uploaded) return fail(RACE_ESTATE, "race_schedule_upload has not been called");
  if (k < 1 || k > 16) return fail(RACE_EUNSUPPORTED, "k must be in 1..16");
  if (s->tree.n == 0) return RACE_OK;
  if (!x || !y) return fail(RACE_EINVAL, "x or y is NULL");
  if (s->expanded && !trace)
    return k == 1 ? run_expanded(s, x, y, static_cast<hipStream_t>(stream))
                  : run_expanded_spmm(s, k, x, y, static_cast<hipStream_t>(stream));
  if (s->params.value_type >= 2) {
    // complex: one vector of n interleaved (re, im) pairs, run as two columns
    if (k != 1) return fail(RACE_EUNSUPPORTED, "complex values take one right-hand side");
    if (rhs_tile(s, 2) < 2)
      return fail(RACE_EUNSUPPORTED, "a complex unit window does not fit the LDS; rebuild with a smaller window_max");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (s->params.value_type == 2) {
      const auto a = unit_args<race::Cplx<false>>(s, s->lane_diagc.p, s->sell_valc.p);
      return run_flow<race::Cplx<false>>(s, a, 2, x, y, 2, trace, st);
    }
    const auto a = unit_args<race::Cplx<true>>(s, reinterpret_cast<const race::Cplx<true>*>(s->lane_diagc.p),
                                               reinterpret_cast<const race::Cplx<true>*>(s->sell_valc.p));
    return run_flow<race::Cplx<true>>(s, a, 2, x, y, 2, trace, st);
  }
  const int32_t kt = rhs_tile(s, k);
  if (kt < 1) return fail(RACE_EUNSUPPORTED, "a unit window does not fit the LDS; rebuild with a smaller window_max");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int32_t n = s->tree.n;
  // with four or more passes, strided columns would waste most of every
  // cache line: copy X into contiguous column tiles, run the passes on
  // them, and copy Y back
  const int32_t passes = (k + kt - 1) / kt;
  const bool tiled = passes >= 4;
  const double* xp = x;
  double* yp = y;
  if (tiled) {
    const size_t need = static_cast<size_t>(n) * k;
    for (DevBuf<double>* b : {&s->tiles_x, &s->tiles_y}) {
      if (b->count < need) {
        release(*b);
        hipError_t e = hipMalloc(&b->p, need * sizeof(double));
        if (e != hipSuccess) return hip_fail(e, "hipMalloc of the column tiles");
        b->count = need;
      }
    }
    hipError_t e = race::launch_tile(n, k, kt, const_cast<double*>(x), s->tiles_x.p, 1, st);
    if (e != hipSuccess) return hip_fail(e, "tiling X");
    xp = s->tiles_x.p;
    yp = s->tiles_y.p;
  }
  // one pass per tile of right-hand sides: columns c0 .. c0 + kc, either in
  // place (rows k doubles apart) or in their contiguous tile (rows kc apart)
  for (int32_t c0 = 0; c0 < k; c0 += kt) {
    const int32_t kc = std::min(kt, k - c0);
    const size_t off = tiled ? static_cast<size_t>(n) * c0 : static_cast<size_t>(c0);
    const int32_t ld = tiled ? kc : k;
    int rc = RACE_OK;
    if (s->params.exec_mode == 0) {  // (the dataflow launch clears them itself, in its first tickets)
      hipError_t ze = race::launch_zero_entries(yp + off, ld, kc, s->zero_idx.p,
                                                static_cast<int64_t>(s->L.zero_idx.size()), st);
      if (ze != hipSuccess) return hip_fail(ze, "clearing shared entries");
    }
    if (s->params.value_type == 0) {
      const auto a = unit_args<double>(s, s->lane_diag64.p, s->sell_val64.p);
      rc = s->params.exec_mode == 1 ? run_flow<double>(s, a, kc, xp + off, yp + off, ld, trace, st)
                                    : run_phases<double>(s, a, kc, xp + off, yp + off, ld, trace, st);
    } else {
      const auto a = unit_args<float>(s, s->lane_diag32.p, s->sell_val32.p);
      rc = s->params.exec_mode == 1 ? run_flow<float>(s, a, kc, xp + off, yp + off, ld, trace, st)
                                    : run_phases<float>(s, a, kc, xp + off, yp + off, ld, trace, st);
    }
    if (rc != RACE_OK) return rc;
  }
  if (tiled) {
    hipError_t e = race::launch_tile(n, k, kt, y, s->tiles_y.p, 0, st);
    if (e != hipSuccess) return hip_fail(e, "untiling Y");
  }
  return RACE_OK;
}

extern "C" {

int race_schedule_check(race_schedule_t s) {
  if (!s) return fail(RACE_EINVAL, "schedule is NULL");
  if (!s->uploaded) return RACE_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  // the status words: after the dataflow state of a product, and after the
  // ticket flags of a dataflow sweep (Gauss-Seidel or Kaczmarz; phase
  // launches have no bounded waits)
  uint32_t* words[2] = {nullptr, nullptr};
  if (!s->gs && s->flow_state.p)
    words[0] = s->flow_state.p + static_cast<int32_t>(s->L.unit_lo.size()) + s->L.n_zero_tasks;
  if (s->gsf_flags.p) words[1] = s->gsf_flags.p + s->gsf_flags.count - 1;
  bool gave_up = false;
  for (uint32_t* status_at : words) {
    if (!status_at) continue;
    uint32_t status = 0;
    e = hipMemcpy(&status, status_at, sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    if (status) {
      const uint32_t zero = 0;
      e = hipMemcpy(status_at, &zero, sizeof(uint32_t), hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
      gave_up = true;
    }
  }
  if (gave_up) return fail(RACE_EINTERNAL, "a dataflow wait gave up (bounded spin exceeded)");
  return RACE_OK;
}

int race_schedule_flow_takeovers(race_schedule_t s, int64_t* count) {
  if (!s || !count) return fail(RACE_EINVAL, "NULL argument");
  *count = 0;
  if (!s->uploaded || s->gs) return RACE_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  uint32_t v = 0;
  e = hipMemcpy(&v, s->claims.p + (s->claims.count - 1), sizeof(uint32_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  *count = v;
  return RACE_OK;
}

int race_schedule_flow_test_late(race_schedule_t s, int32_t stride) {
  if (!s) return fail(RACE_EINVAL, "schedule is NULL");
  if (stride < 0) return fail(RACE_EINVAL, "stride must be >= 0");
  s->late_stride = stride;
  return RACE_OK;
}

int race_symm_spmv(race_schedule_t s, const double* x, double* y, void* stream) {
  return run_products(s, 1, x, y, nullptr, stream);
}

}  // extern "C"

// Dataflow state of race_symm_spmv_noalloc: completion flags, the ticket
// counter, the static-ticket claims and the takeover count of one product,
// in a fixed array that every device holds once for the life of the
// process.  Host code never uses the array's name as an address: each
// device's copy is reached through the address hipGetSymbolAddress returns
// with that device current.
constexpr int64_t kNoallocWords = int64_t(1) << 20;  // 4 MiB
static __device__ __align__(256) uint32_t scratch[kNoallocWords];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch[kMaxDevices] = {};

// Address of the current device's copy of `scratch` (looked up once per device).
int noalloc_scratch(int dev, uint32_t** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(RACE_EUNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the no-allocation state");
    g_scratch[dev] = static_cast<uint32_t*>(p);
  }
  *out = g_scratch[dev];
  return RACE_OK;
}

template <typename ValT>
int run_flow_noalloc(race_schedule_t s, const race::UnitArgs<ValT>& a, const double* x, double* y, uint32_t* scr,
                     hipStream_t st) {
  const race::Layout& L = s->L;
  const int32_t n_units = static_cast<int32_t>(L.unit_lo.size());
  if (n_units == 0) return RACE_OK;
  const int32_t wmax = std::max(1, L.max_window);
  int32_t per_cu = 0;
  hipError_t e = race::race_flow_occupancy<ValT>(1, s->params.block_threads, wmax, &per_cu);
  if (e != hipSuccess) return hip_fail(e, "occupancy query");
  if (per_cu < 1) return fail(RACE_EUNSUPPORTED, "dataflow kernel does not fit a CU with this window and block size");
  const int32_t n_flags = n_units + L.n_zero_tasks;
  const int32_t grid = std::max(1, std::min(n_flags, per_cu * s->n_cus));
  const int32_t n_static = grid;
  // [done flags][pad to 8 bytes][64-bit counter][claims][takeover count]
  const int64_t counter_word = (static_cast<int64_t>(n_flags) + 1) / 2 * 2;
  const int64_t claim_word = counter_word + 2;
  const int64_t words = claim_word + n_static + 1;
  if (words > kNoallocWords)
    return fail(RACE_EUNSUPPORTED, "schedule needs " + std::to_string(words) +
                                       " words of dataflow state; race_symm_spmv_noalloc holds at most " +
                                       std::to_string(kNoallocWords) + " (units + clearing tasks + workgroups)");
  // every call starts from cleared state, so the launch can always use
  // epoch 1 and ticket base 0 (and a captured graph replays correctly)
  e = race::launch_clear_words(scr, words, st);
  if (e != hipSuccess) return hip_fail(e, "clearing the dataflow state");
  race::FlowArgs f{s->dep_idx.p, scr, reinterpret_cast<uint64_t*>(scr + counter_word),
                   s->flow_state.p + n_flags,  // the schedule's own status word (race_schedule_check)
                   scr + claim_word, scr + claim_word + n_static, n_static, 0, nullptr, n_flags, n_units,
                   L.n_zero_tasks, race::kZeroChunk, s->zero_idx.p, static_cast<int64_t>(L.zero_idx.size()),
                   s->ticket_unit_d.p, s->unit_ticket_d.p};
  e = race::launch_race_flow<ValT>(a, f, 1, x, y, 1, wmax, s->params.block_threads, grid, 1u, 0u, st);
  if (e != hipSuccess) return hip_fail(e, "RACE dataflow launch");
  return RACE_OK;
}

}  // namespace

extern "C" {

int race_symm_spmv_noalloc(race_schedule_t s, const double* x, double* y, void* stream) {
  if (!s) return fail(RACE_EINVAL, "schedule is NULL");
  if (s->gs) return fail(RACE_EUNSUPPORTED, kDist1Product);
  if (!s->uploaded) return fail(RACE_ESTATE, "race_schedule_upload has not been called");
  if (s->params.value_type > 1) return fail(RACE_EUNSUPPORTED, "race_symm_spmv_noalloc takes real values only");
  if (s->tree.n == 0) return RACE_OK;
  if (!x || !y) return fail(RACE_EINVAL, "x or y is NULL");
  // the expanded product uses no dataflow state
  if (s->expanded) return run_expanded(s, x, y, static_cast<hipStream_t>(stream));
  if (s->params.exec_mode != 1) return fail(RACE_EUNSUPPORTED, "race_symm_spmv_noalloc runs the dataflow mode only");
  if (rhs_tile(s, 1) < 1)
    return fail(RACE_EUNSUPPORTED, "a unit window does not fit the LDS; rebuild with a smaller window_max");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != s->device) return fail(RACE_EINVAL, "the schedule was uploaded to another device");
  uint32_t* scr = nullptr;
  int rc = noalloc_scratch(dev, &scr);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (s->params.value_type == 0)
    return run_flow_noalloc<double>(s, unit_args<double>(s, s->lane_diag64.p, s->sell_val64.p), x, y, scr, st);
  return run_flow_noalloc<float>(s, unit_args<float>(s, s->lane_diag32.p, s->sell_val32.p), x, y, scr, st);
}

int race_symm_spmm(race_schedule_t s, int32_t k, const double* X, double* Y, void* stream) {
  return run_products(s, k, X, Y, nullptr, stream);
}

int race_symm_spmm_traced(race_schedule_t s, int32_t k, const double* X, double* Y, uint64_t* trace, void* stream) {
  if (!trace) return fail(RACE_EINVAL, "trace is NULL");
  return run_products(s, k, X, Y, trace, stream);
}

}  // extern "C"

// Read dependencies of matrix powers (built once, uploaded when the schedule is).
static int ensure_read_deps(race_schedule_t s, bool device) {
  try {
    if (s->rdep_ptr_h.empty()) race::build_read_deps(s->L, s->rdep_ptr_h, s->rdep_idx_h);
  } catch (const std::bad_alloc&) {
    return fail(RACE_ENOMEM, "out of host memory while building the read dependencies");
  }
  if (device && !s->rdep_ptr.p) {
    int64_t total = 0;
    hipError_t e = upload(s->rdep_ptr, s->rdep_ptr_h.data(), s->rdep_ptr_h.size(), &total);
    if (e == hipSuccess) e = upload(s->rdep_idx, s->rdep_idx_h.data(), s->rdep_idx_h.size(), &total);
    if (e != hipSuccess) {
      release(s->rdep_ptr);
      release(s->rdep_idx);
      return hip_fail(e, "upload of the read dependencies");
    }
  }
  return RACE_OK;
}

// The diagonal matrix-power ticket order for P powers and n_static static
// tickets (host).
static int build_mpk_order(race_schedule_t s, int32_t P, int32_t n_static, std::vector<int32_t>& order) {
  int rc = ensure_read_deps(s, false);
  if (rc) return rc;
  std::vector<int32_t> tu, ut;
  ticket_arrays(s, tu, ut);
  try {
    race::mpk_ticket_order(s->L, tu, s->rdep_ptr_h, s->rdep_idx_h, P, n_static, std::max<int64_t>(0, s->mpk_lag),
                           order);
  } catch (const std::bad_alloc&) {
    return fail(RACE_ENOMEM, "out of host memory while ordering the matrix-power tickets");
  } catch (const std::exception& ex) {
    return fail(RACE_EINTERNAL, ex.what());
  }
  return RACE_OK;
}

template <typename ValT>
static int run_mpk(race_schedule_t s, const race::UnitArgs<ValT>& a, int32_t P, const double* x, double* Y,
                   hipStream_t st) {
  const race::Layout& L = s->L;
  const int32_t n_units = static_cast<int32_t>(L.unit_lo.size());
  if (n_units == 0) return RACE_OK;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(st, &cap);
  if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
  if (cap != hipStreamCaptureStatusNone)
    return fail(RACE_EUNSUPPORTED, "matrix powers cannot be captured into a graph (the launch epoch is an argument)");
  int rc = ensure_read_deps(s, true);
  if (rc) return rc;
  const int32_t wmax = std::max(1, L.max_window);
  int32_t per_cu = 0;
  e = race::race_mpk_occupancy<ValT>(s->params.block_threads, wmax, &per_cu);
  if (e != hipSuccess) return hip_fail(e, "occupancy query");
  if (per_cu < 1) return fail(RACE_EUNSUPPORTED, "matrix-power kernel does not fit a CU with this window and block size");
  const int32_t n_flags = n_units + L.n_zero_tasks;
  const int64_t n_tickets64 = static_cast<int64_t>(P) * n_flags;
  if (n_tickets64 >= (int64_t(1) << 31)) return fail(RACE_EUNSUPPORTED, "too many tickets (powers x units)");
  const int32_t n_tickets = static_cast<int32_t>(n_tickets64);
  const int32_t grid = std::max(1, std::min(n_tickets, per_cu * s->n_cus));
  // static tickets stay within the first power: a later power's ticket is
  // handed out only once every static ticket has a running owner
  const int32_t n_static = std::min(grid, n_flags);
  const size_t claim_cap = s->claims.count - 1;
  if (static_cast<size_t>(n_static) > claim_cap) return fail(RACE_EINTERNAL, "more workgroups than claim words");
  // [done flags of every power][pad to 8 bytes][64-bit counter]
  const size_t flag_words = static_cast<size_t>(n_tickets);
  const size_t counter_word = (flag_words + 1) / 2 * 2;
  const size_t words = counter_word + 2;
  if (s->mpk_state.count < words) {
    release(s->mpk_state);
    e = hipMalloc(&s->mpk_state.p, words * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemsetAsync(s->mpk_state.p, 0, words * sizeof(uint32_t), st);
    if (e != hipSuccess) {
      release(s->mpk_state);
      return hip_fail(e, "allocation of the matrix-power state");
    }
    s->mpk_state.count = words;
    s->mpk_ticket_next = 0;
  }
  e = next_epoch(s, st);
  if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
  uint32_t* state = s->mpk_state.p;
  const size_t counter_at = (s->mpk_state.count - 2) / 2 * 2;
  const uint64_t ticket_base = s->mpk_ticket_next;
  s->mpk_ticket_next += static_cast<uint64_t>(n_tickets - n_static) + static_cast<uint64_t>(grid);
  race::FlowArgs f{s->dep_idx.p, state, reinterpret_cast<uint64_t*>(state + counter_at),
                   s->flow_state.p + n_flags,  // the schedule's status word (race_schedule_check)
                   s->claims.p, s->claims.p + claim_cap, n_static, s->late_stride, nullptr, n_tickets, n_units,
                   L.n_zero_tasks, race::kZeroChunk, s->zero_idx.p, static_cast<int64_t>(L.zero_idx.size()),
                   s->ticket_unit_d.p, s->unit_ticket_d.p};
  const int32_t* order = nullptr;
  if (s->mpk_lag >= 0) {
    if (s->mpk_order_P != P || s->mpk_order_static != n_static) {
      rc = build_mpk_order(s, P, n_static, s->mpk_order_h);
      if (rc) return rc;
      // the buffer may still be read by an earlier launch on this stream
      e = hipStreamSynchronize(st);
      if (e == hipSuccess && s->mpk_order_d.count < s->mpk_order_h.size()) {
        release(s->mpk_order_d);
        int64_t total = 0;
        e = upload(s->mpk_order_d, s->mpk_order_h.data(), s->mpk_order_h.size(), &total);
      } else if (e == hipSuccess) {
        e = hipMemcpy(s->mpk_order_d.p, s->mpk_order_h.data(), sizeof(int32_t) * s->mpk_order_h.size(),
                      hipMemcpyHostToDevice);
      }
      if (e != hipSuccess) {
        s->mpk_order_P = 0;
        return hip_fail(e, "upload of the matrix-power ticket order");
      }
      s->mpk_order_P = P;
      s->mpk_order_static = n_static;
    }
    order = s->mpk_order_d.p;
  }
  race::MpkArgs m{s->rdep_ptr.p, s->rdep_idx.p, P, n_flags, static_cast<int64_t>(s->tree.n), order, s->mpk_cache};
  e = race::launch_race_mpk<ValT>(a, f, m, x, Y, wmax, s->params.block_threads, grid, s->epoch, ticket_base, st);
  if (e != hipSuccess) return hip_fail(e, "matrix-power launch");
  return RACE_OK;
}

extern "C" {

int race_symm_mpk(race_schedule_t s, int32_t powers, const double* x, double* Y, void* stream) {
  if (!s) return fail(RACE_EINVAL, "schedule is NULL");
  if (s->gs) return fail(RACE_EUNSUPPORTED, kDist1Product);
  if (!s->uploaded) return fail(RACE_ESTATE, "race_schedule_upload has not been called");
  if (powers < 1 || powers > 64) return fail(RACE_EINVAL, "powers must be in 1..64");
  if (s->params.value_type > 1) return fail(RACE_EUNSUPPORTED, "matrix powers take real values only");
  if (s->tree.n == 0) return RACE_OK;
  if (!x || !Y) return fail(RACE_EINVAL, "x or Y is NULL");
  if (rhs_tile(s, 1) < 1)
    return fail(RACE_EUNSUPPORTED, "a unit window does not fit the LDS; rebuild with a smaller window_max");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != s->device) return fail(RACE_EINVAL, "the schedule was uploaded to another device");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (s->params.value_type == 0)
    return run_mpk<double>(s, unit_args<double>(s, s->lane_diag64.p, s->sell_val64.p), powers, x, Y, st);
  return run_mpk<float>(s, unit_args<float>(s, s->lane_diag32.p, s->sell_val32.p), powers, x, Y, st);
}

int race_symm_poly(race_schedule_t s, int32_t degree, const double* coeffs, const double* x, double* work, double* z,
                   void* stream) {
  if (!s) return fail(RACE_EINVAL, "schedule is NULL");
  if (degree < 0 || degree > race::kMaxPolyDegree) return fail(RACE_EINVAL, "degree must be in 0..32");
  if (!coeffs) return fail(RACE_EINVAL, "coeffs is NULL");
  if (s->tree.n > 0 && (!x || !z || (degree > 0 && !work))) return fail(RACE_EINVAL, "x, work or z is NULL");
  if (degree > 0) {
    const int rc = race_symm_mpk(s, degree, x, work, stream);
    if (rc) return rc;
  } else if (!s->uploaded) {
    return fail(RACE_ESTATE, "race_schedule_upload has not been called");
  }
  race::PolyCoeffs c{};
  for (int32_t p = 0; p <= degree; ++p) c.c[p] = coeffs[p];
  const hipError_t e = race::launch_poly_combine(s->tree.n, degree, c, x, work, z, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "polynomial combination launch");
  return RACE_OK;
}

int race_schedule_set_mpk_order(race_schedule_t s, int64_t lag_rows, int32_t cache_matrix) {
  if (!s) return fail(RACE_EINVAL, "schedule is NULL");
  if (s->gs) return fail(RACE_EUNSUPPORTED, "a distance-1 schedule has no units");
  if (cache_matrix != 0 && cache_matrix != 1) return fail(RACE_EINVAL, "cache_matrix must be 0 or 1");
  s->mpk_lag = lag_rows < 0 ? -1 : lag_rows;
  s->mpk_cache = cache_matrix;
  s->mpk_order_P = 0;
  return RACE_OK;
}

int race_schedule_mpk_order(race_schedule_t s, int32_t powers, int32_t n_static, int32_t* order) {
  if (!s || !order) return fail(RACE_EINVAL, "NULL argument");
  if (s->gs) return fail(RACE_EUNSUPPORTED, "a distance-1 schedule has no units");
  if (powers < 1 || powers > 64) return fail(RACE_EINVAL, "powers must be in 1..64");
  const int32_t per = static_cast<int32_t>(s->L.unit_lo.size()) + s->L.n_zero_tasks;
  if (n_static < 0 || n_static > per) return fail(RACE_EINVAL, "n_static must be in 0..units + clearing tasks");
  const int64_t total = static_cast<int64_t>(powers) * per;
  if (s->mpk_lag < 0) {
    for (int64_t t = 0; t < total; ++t) order[t] = static_cast<int32_t>(t);
    return RACE_OK;
  }
  std::vector<int32_t> o;
  const int rc = build_mpk_order(s, powers, n_static, o);
  if (rc) return rc;
  std::copy(o.begin(), o.end(), order);
  return RACE_OK;
}

int race_schedule_read_deps(race_schedule_t s, int64_t* count, int32_t* ptr, int32_t* idx) {
  if (!s || !count) return fail(RACE_EINVAL, "NULL argument");
  if (s->gs) return fail(RACE_EUNSUPPORTED, "a distance-1 schedule has no units");
  const int rc = ensure_read_deps(s, false);
  if (rc) return rc;
  *count = static_cast<int64_t>(s->rdep_idx_h.size());
  if (ptr) std::copy(s->rdep_ptr_h.begin(), s->rdep_ptr_h.end(), ptr);
  if (idx) std::copy(s->rdep_idx_h.begin(), s->rdep_idx_h.end(), idx);
  return RACE_OK;
}

}  // extern "C"

// One dataflow launch for a whole sweep (race_schedule_set_gs_exec 1).
// kacz: a Kaczmarz sweep over the schedule's Kaczmarz layout (one leaf
// per ticket) with relaxation omega.  A schedule holds one of the two
// layouts, so both share the plan caches, flags and epoch.
static int run_gs_flow(race_schedule_t s, const race::GsArgs& a, int32_t direction, const double* b, double* x,
                       hipStream_t st, bool kacz = false, double omega = 1.0) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(st, &cap);
  if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
  if (cap != hipStreamCaptureStatusNone)
    return fail(RACE_EUNSUPPORTED, "a dataflow sweep cannot be captured into a graph (the launch epoch is an argument)");
  race::GsFlow& f = s->gs_flow_h[direction];
  if (f.direction != direction) {
    try {
      if (kacz)
        race::build_kacz_flow(s->KG, direction, f);
      else
        race::build_gs_flow(s->G, direction, f);
    } catch (const std::bad_alloc&) {
      f.direction = -1;
      return fail(RACE_ENOMEM, "out of host memory while planning the dataflow sweep");
    } catch (const std::exception& ex) {
      f.direction = -1;
      return fail(RACE_EINTERNAL, ex.what());
    }
    int64_t total = 0;
    for (DevBuf<int32_t>* bf : {&s->gsf_item[direction], &s->gsf_back[direction], &s->gsf_leaf0[direction],
                                &s->gsf_count[direction], &s->gsf_dptr[direction], &s->gsf_didx[direction]})
      release(*bf);
    e = upload(s->gsf_item[direction], f.ticket_item.data(), f.ticket_item.size(), &total);
    if (e == hipSuccess) e = upload(s->gsf_back[direction], f.ticket_back.data(), f.ticket_back.size(), &total);
    if (e == hipSuccess) e = upload(s->gsf_leaf0[direction], f.item_leaf0.data(), f.item_leaf0.size(), &total);
    if (e == hipSuccess) e = upload(s->gsf_count[direction], f.item_count.data(), f.item_count.size(), &total);
    if (e == hipSuccess) e = upload(s->gsf_dptr[direction], f.dep_ptr.data(), f.dep_ptr.size(), &total);
    if (e == hipSuccess && !f.dep_idx.empty()) e = upload(s->gsf_didx[direction], f.dep_idx.data(), f.dep_idx.size(), &total);
    if (e != hipSuccess) {
      f.direction = -1;
      return hip_fail(e, "upload of the dataflow sweep plan");
    }
  }
  const int32_t nt = static_cast<int32_t>(f.ticket_item.size());
  if (nt == 0) return RACE_OK;
  // flags of every ticket, the drain word, then the status word; a new
  // allocation starts at epoch 0 everywhere
  if (s->gsf_flags.count < static_cast<size_t>(nt) + 2) {
    release(s->gsf_flags);
    std::vector<uint32_t> zeros(static_cast<size_t>(nt) + 2, 0u);
    int64_t total = 0;
    e = upload(s->gsf_flags, zeros.data(), zeros.size(), &total);
    if (e != hipSuccess) return hip_fail(e, "allocation of the dataflow sweep flags");
    s->gs_epoch = 0;
  }
  if (++s->gs_epoch == 0) {
    // the epoch wrapped: clear the flags and the drain word (the status
    // word keeps its value)
    e = race::launch_clear_words(s->gsf_flags.p, static_cast<int64_t>(s->gsf_flags.count) - 1, st);
    if (e != hipSuccess) return hip_fail(e, "flag reset");
    s->gs_epoch = 1;
  }
  int32_t grid = 0;
  const int32_t wmax = kacz ? s->KG.max_window : s->G.max_window;
  e = kacz ? race::kacz_flow_grid(wmax, s->n_cus, &grid) : race::gs_flow_grid(wmax, s->n_cus, &grid);
  if (e != hipSuccess) return hip_fail(e, "occupancy query");
  if (grid < 1) return fail(RACE_EUNSUPPORTED, "the dataflow sweep does not fit a CU");
  grid = std::min(grid, nt);
  const race::GsFlowArgs fa{s->gsf_item[direction].p, s->gsf_back[direction].p, s->gsf_leaf0[direction].p,
                            s->gsf_count[direction].p, s->gsf_dptr[direction].p, s->gsf_didx[direction].p,
                            s->gsf_flags.p, s->gsf_flags.p + s->gsf_flags.count - 1,
                            s->gsf_flags.p + s->gsf_flags.count - 2, nt, s->gs_epoch};
  e = kacz ? race::launch_kacz_flow(a, fa, wmax, grid, omega, b, x, st) : race::launch_gs_flow(a, fa, wmax, grid, b, x, st);
  if (e != hipSuccess) return hip_fail(e, "dataflow sweep launch");
  return RACE_OK;
}

extern "C" {

int race_schedule_set_gs_exec(race_schedule_t s, int32_t mode) {
  if (!s) return fail(RACE_EINVAL, "schedule is NULL");
  if (!s->gs && !s->kz)
    return fail(RACE_EUNSUPPORTED, "sweeps need a distance-1 schedule or one built with race_params.kaczmarz");
  if (mode != 0 && mode != 1) return fail(RACE_EINVAL, "mode must be 0 (a launch per phase) or 1 (one dataflow launch)");
  s->gs_exec = mode;
  return RACE_OK;
}

int race_schedule_gs_flow_plan(race_schedule_t s, int32_t direction, int32_t* n_tickets, int64_t* n_deps,
                               int32_t* ticket_leaf0, int32_t* ticket_count, int32_t* ticket_back, int32_t* dep_ptr,
                               int32_t* dep_idx) {
  if (!s || !n_tickets || !n_deps) return fail(RACE_EINVAL, "NULL argument");
  if (!s->gs && !s->kz)
    return fail(RACE_EUNSUPPORTED, "sweeps need a distance-1 schedule or one built with race_params.kaczmarz");
  if (direction < 0 || direction > 2) return fail(RACE_EINVAL, "direction must be 0 (forward), 1 (backward) or 2 (both)");
  race::GsFlow f;
  try {
    if (s->gs)
      race::build_gs_flow(s->G, direction, f);
    else
      race::build_kacz_flow(s->KG, direction, f);
  } catch (const std::bad_alloc&) {
    return fail(RACE_ENOMEM, "out of host memory while planning the dataflow sweep");
  } catch (const std::exception& ex) {
    return fail(RACE_EINTERNAL, ex.what());
  }
  const int32_t nt = static_cast<int32_t>(f.ticket_item.size());
  *n_tickets = nt;
  *n_deps = static_cast<int64_t>(f.dep_idx.size());
  for (int32_t t = 0; t < nt; ++t) {
    const int32_t i = f.ticket_item[static_cast<size_t>(t)];
    if (ticket_leaf0) ticket_leaf0[t] = f.item_leaf0[static_cast<size_t>(i)];
    if (ticket_count) ticket_count[t] = f.item_count[static_cast<size_t>(i)];
    if (ticket_back) ticket_back[t] = f.ticket_back[static_cast<size_t>(t)];
  }
  if (dep_ptr) std::copy(f.dep_ptr.begin(), f.dep_ptr.end(), dep_ptr);
  if (dep_idx) std::copy(f.dep_idx.begin(), f.dep_idx.end(), dep_idx);
  return RACE_OK;
}

int race_schedule_set_gs_quad(race_schedule_t s, int32_t min_leaves) {
  if (!s) return fail(RACE_EINVAL, "schedule is NULL");
  if (!s->gs && !s->kz)
    return fail(RACE_EUNSUPPORTED, "sweeps need a distance-1 schedule or one built with race_params.kaczmarz");
  if (min_leaves < -2) return fail(RACE_EINVAL, "min_leaves must be -2 (never), -1 (default) or >= 0");
  s->gs_quad_min = min_leaves;
  return RACE_OK;
}

int race_symm_gs(race_schedule_t s, const double* b, double* x, int32_t direction, void* stream) {
  if (!s) return fail(RACE_EINVAL, "schedule is NULL");
  if (!s->gs) return fail(RACE_EUNSUPPORTED, "Gauss-Seidel sweeps need a distance-1 schedule (dist_k = 1)");
  if (!s->uploaded) return fail(RACE_ESTATE, "race_schedule_upload has not been called");
  if (direction < 0 || direction > 2) return fail(RACE_EINVAL, "direction must be 0 (forward), 1 (backward) or 2 (both)");
  if (s->tree.n == 0) return RACE_OK;
  if (!b || !x) return fail(RACE_EINVAL, "b or x is NULL");
  const race::GsLayout& G = s->G;
  const race::GsArgs a{s->gs_leaf_lo.p, s->gs_leaf_hi.p, s->gs_halo_ptr.p, s->gs_halo.p,
                       s->gs_row_ptr.p, s->gs_slot.p,    s->gs_val.p,      s->gs_diag.p};
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (s->gs_exec == 1 && G.max_window <= race::kGsQuadMaxWindow) return run_gs_flow(s, a, direction, b, x, st);
  const int32_t np = s->tree.n_phases;
  auto phase = [&](int32_t ph, bool backward) {
    const int32_t l0 = G.phase_leaf_ptr[ph], l1 = G.phase_leaf_ptr[ph + 1];
    // four leaves per wavefront once a phase has more leaves than the CUs
    // hold wavefronts (32 each)
    const int32_t quad_min = s->gs_quad_min >= 0 ? s->gs_quad_min : (s->gs_quad_min == -1 ? 32 * s->n_cus : INT32_MAX);
    return race::launch_gs_phase(a, l0, l1 - l0, G.phase_max_window[ph], backward, quad_min, b, x, st);
  };
  if (direction != 1)
    for (int32_t ph = 0; ph < np; ++ph) {
      hipError_t e = phase(ph, false);
      if (e != hipSuccess) return hip_fail(e, "Gauss-Seidel phase launch");
    }
  if (direction != 0)
    for (int32_t ph = np - 1; ph >= 0; --ph) {
      hipError_t e = phase(ph, true);
      if (e != hipSuccess) return hip_fail(e, "Gauss-Seidel phase launch");
    }
  return RACE_OK;
}

int race_symm_kacz(race_schedule_t s, const double* b, double* x, int32_t direction, double omega, void* stream) {
  if (!s) return fail(RACE_EINVAL, "schedule is NULL");
  if (s->gs) return fail(RACE_EUNSUPPORTED, "Kaczmarz sweeps need a distance-2 schedule (dist_k >= 2)");
  if (!s->kz) return fail(RACE_ESTATE, "the schedule was built without race_params.kaczmarz = 1");
  if (!s->uploaded) return fail(RACE_ESTATE, "race_schedule_upload has not been called");
  if (direction < 0 || direction > 2) return fail(RACE_EINVAL, "direction must be 0 (forward), 1 (backward) or 2 (both)");
  if (!(omega > 0.0 && omega < 2.0)) return fail(RACE_EINVAL, "omega must be in (0, 2)");
  if (s->tree.n == 0) return RACE_OK;
  if (!b || !x) return fail(RACE_EINVAL, "b or x is NULL");
  const race::GsLayout& K = s->KG;
  const race::GsArgs a{s->kz_leaf_lo.p, s->kz_leaf_hi.p, s->kz_halo_ptr.p, s->kz_halo.p, s->kz_row_ptr.p,
                       s->kz_slot.p,    s->kz_val.p,     s->kz_diag.p,     s->kz_nrm.p};
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (s->gs_exec == 1) return run_gs_flow(s, a, direction, b, x, st, true, omega);
  const int32_t np = s->tree.n_phases;
  // four leaves per wavefront once a phase has more leaves than the CUs
  // hold wavefronts (32 each)
  const int32_t quad_min = s->gs_quad_min >= 0 ? s->gs_quad_min : (s->gs_quad_min == -1 ? 32 * s->n_cus : INT32_MAX);
  auto phase = [&](int32_t ph, bool backward) {
    const int32_t l0 = K.phase_leaf_ptr[ph], l1 = K.phase_leaf_ptr[ph + 1];
    return race::launch_kacz_phase(a, l0, l1 - l0, K.phase_max_window[ph], backward, omega, quad_min, b, x, st);
  };
  if (direction != 1)
    for (int32_t ph = 0; ph < np; ++ph) {
      hipError_t e = phase(ph, false);
      if (e != hipSuccess) return hip_fail(e, "Kaczmarz phase launch");
    }
  if (direction != 0)
    for (int32_t ph = np - 1; ph >= 0; --ph) {
      hipError_t e = phase(ph, true);
      if (e != hipSuccess) return hip_fail(e, "Kaczmarz phase launch");
    }
  return RACE_OK;
}

int race_permute(race_schedule_t s, int32_t k, const double* in, double* out, int32_t to_permuted, void* stream) {
  if (!s) return fail(RACE_EINVAL, "schedule is NULL");
  if (!s->uploaded) return fail(RACE_ESTATE, "race_schedule_upload has not been called");
  if (k < 1) return fail(RACE_EINVAL, "k must be >= 1");
  if (s->tree.n == 0) return RACE_OK;
  if (!in || !out) return fail(RACE_EINVAL, "in or out is NULL");
  hipError_t e = race::launch_permute(s->tree.n, k, s->new2old.p, in, out, to_permuted, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "permute launch");
  return RACE_OK;
}

}  // extern "C"

template <typename ValT>
static race::BatchMat<ValT> batch_mat(race_schedule_t s, const ValT* diag, const ValT* vals, uint32_t* done,
                                      const double* x, double* y) {
  return race::BatchMat<ValT>{unit_args<ValT>(s, diag, vals),
                              s->dep_idx.p,
                              done,
                              x,
                              y,
                              s->zero_idx.p,
                              static_cast<int64_t>(s->L.zero_idx.size()),
                              static_cast<int32_t>(s->L.unit_lo.size()),
                              s->L.n_zero_tasks,
                              race::kZeroChunk,
                              s->tree.n,
                              nullptr,
                              nullptr};
}

static void batch_release(race_batch_t b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  b->exec = nullptr;
  b->graph = nullptr;
  b->cap = nullptr;
  if (b->d_mats) (void)hipFree(b->d_mats);
  b->d_mats = nullptr;
  if (b->d_bmats) (void)hipFree(b->d_bmats);
  b->d_bmats = nullptr;
  release(b->blk_mat);
  release(b->ticket_mat);
  release(b->ticket_unit);
  release(b->state);
  release(b->tiles_x);
  release(b->tiles_y);
}

// One pass per tile of right-hand sides, each a state reset and one
// persistent launch over all tickets.
static hipError_t batch_enqueue(race_batch_t b, hipStream_t st) {
  if (b->n_exp_blocks > 0) {
    hipError_t e = b->value_type == 0
                       ? race::launch_csr_block_batch<double>(static_cast<const race::BlockMat<double>*>(b->d_bmats),
                                                              b->blk_mat.p, b->n_exp_blocks, st)
                       : race::launch_csr_block_batch<float>(static_cast<const race::BlockMat<float>*>(b->d_bmats),
                                                             b->blk_mat.p, b->n_exp_blocks, st);
    if (e != hipSuccess) return e;
  }
  if (b->k > 1) {
    for (size_t i = 0; i < b->exp_members.size(); ++i) {
      hipError_t e = expanded_spmm(b->mats[b->exp_members[i]], b->k, b->exp_x[i], b->exp_y[i], st);
      if (e != hipSuccess) return e;
    }
  }
  if (b->n_tickets == 0) return hipSuccess;
  if (b->tiled) {
    hipError_t e = b->value_type == 0
                       ? race::launch_batch_tile<double>(static_cast<const race::BatchMat<double>*>(b->d_mats),
                                                         b->count, b->k, b->kt, 1, st)
                       : race::launch_batch_tile<float>(static_cast<const race::BatchMat<float>*>(b->d_mats),
                                                        b->count, b->k, b->kt, 1, st);
    if (e != hipSuccess) return e;
  }
  for (int32_t c0 = 0; c0 < b->k; c0 += b->kt) {
    const int32_t kc = std::min(b->kt, b->k - c0);
    race::BatchArgs a{b->ticket_mat.p, b->ticket_unit.p, b->state.p, static_cast<int64_t>(b->state.count),
                      b->n_tickets, c0, b->tiled ? kc : b->k, b->tiled ? 1 : 0};
    hipError_t e =
        b->value_type == 0
            ? race::launch_race_batch<double>(static_cast<const race::BatchMat<double>*>(b->d_mats), a, kc, b->wmax,
                                              b->threads, b->grid, st)
            : race::launch_race_batch<float>(static_cast<const race::BatchMat<float>*>(b->d_mats), a, kc, b->wmax,
                                             b->threads, b->grid, st);
    if (e != hipSuccess) return e;
  }
  if (b->tiled)
    return b->value_type == 0
               ? race::launch_batch_tile<double>(static_cast<const race::BatchMat<double>*>(b->d_mats), b->count,
                                                 b->k, b->kt, 0, st)
               : race::launch_batch_tile<float>(static_cast<const race::BatchMat<float>*>(b->d_mats), b->count, b->k,
                                                b->kt, 0, st);
  return hipSuccess;
}

extern "C" {

int race_batch_create(int32_t count, const race_schedule_t* s, int32_t k, int32_t threads_override,
                      race_batch_t* out) {
  if (!out || !s || count < 1) return fail(RACE_EINVAL, "need count >= 1 schedules and an output handle");
  *out = nullptr;
  if (k < 1 || k > 16) return fail(RACE_EUNSUPPORTED, "k must be in 1..16");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  int32_t wmax = 1, threads = 0, vt = -1;
  for (int32_t m = 0; m < count; ++m) {
    if (s[m] && s[m]->gs) return fail(RACE_EUNSUPPORTED, kDist1Product);
    if (!s[m] || !s[m]->uploaded) return fail(RACE_ESTATE, "every schedule must be uploaded");
    if (s[m]->device != dev) return fail(RACE_EINVAL, "schedules live on different devices");
    if (s[m]->params.value_type >= 2) return fail(RACE_EUNSUPPORTED, "batches take real values only");
    if (vt >= 0 && s[m]->params.value_type != vt) return fail(RACE_EINVAL, "schedules mix value types");
    vt = s[m]->params.value_type;
    threads = std::max(threads, s[m]->params.block_threads);
    if (!s[m]->expanded) wmax = std::max(wmax, s[m]->L.max_window);
  }
  // right-hand sides per pass: all k if the largest window allows, else the widest tile that fits
  int32_t kt = k;
  while (kt > 1 && race::window_lds_bytes(wmax, kt) > 159 * 1024) --kt;
  if (race::window_lds_bytes(wmax, kt) > 159 * 1024)
    return fail(RACE_EUNSUPPORTED, "largest window exceeds the LDS; rebuild with a smaller window_max");
  if (threads_override != 0) {
    if (threads_override != 64 && threads_override != 128 && threads_override != 256 && threads_override != 512 &&
        threads_override != 1024)
      return fail(RACE_EINVAL, "threads must be 0 (largest of the schedules) or 64, 128, 256, 512, 1024");
    threads = threads_override;
  }
  race_batch* b = new (std::nothrow) race_batch();
  if (!b) return fail(RACE_ENOMEM, "out of host memory");
  b->count = count;
  b->k = k;
  b->kt = kt;
  b->tiled = (k + kt - 1) / kt >= 4;
  b->value_type = vt;
  b->threads = threads;
  b->wmax = wmax;
  b->device = dev;
  b->mats.assign(s, s + count);
  // tickets: (key, matrix, ticket of the matrix): every matrix's clearing
  // tasks first (key -1), then its units keyed by their phase as a fraction
  // of the matrix's phases; every matrix keeps its own order, so all
  // conflict edges point backwards
  struct Tk {
    double key;
    int32_t m, u;
  };
  std::vector<Tk> tk;
  int64_t total_units = 0;
  b->unit_base.resize(count);
  std::vector<int32_t> blk_mat;
  for (int32_t m = 0; m < count; ++m) {
    const race::Layout& L = s[m]->L;
    const race::Tree& t = s[m]->tree;
    b->unit_base[m] = total_units;
    if (s[m]->expanded) {
      if (k == 1)
        blk_mat.insert(blk_mat.end(), static_cast<size_t>(s[m]->exp_nblk),
                       static_cast<int32_t>(b->exp_members.size()));
      b->exp_members.push_back(m);
      continue;
    }
    const int32_t nu = static_cast<int32_t>(L.unit_lo.size());
    for (int32_t z = 0; z < L.n_zero_tasks; ++z) tk.push_back({-1.0, m, z});
    for (int32_t u = 0; u < nu; ++u)
      tk.push_back({static_cast<double>(t.leaf_phase[L.unit_leaf[u]]) / static_cast<double>(t.n_phases), m,
                    L.n_zero_tasks + u});
    total_units += nu + L.n_zero_tasks;
  }
  std::stable_sort(tk.begin(), tk.end(), [](const Tk& a, const Tk& c) {
    if (a.key != c.key) return a.key < c.key;
    return a.m < c.m;
  });
  std::vector<int32_t> tm(tk.size()), tu(tk.size());
  for (size_t i = 0; i < tk.size(); ++i) {
    tm[i] = tk[i].m;
    tu[i] = tk[i].u;
  }
  b->n_tickets = static_cast<int32_t>(tk.size());
  int64_t total = 0;
  const size_t words = static_cast<size_t>((total_units + 4 + 1) / 2 * 2);
  std::vector<uint32_t> zeros(words, 0u);
  b->n_exp_blocks = static_cast<int32_t>(blk_mat.size());
  e = upload(b->ticket_mat, tm.data(), tm.size(), &total);
  if (e == hipSuccess) e = upload(b->ticket_unit, tu.data(), tu.size(), &total);
  if (e == hipSuccess && !blk_mat.empty()) e = upload(b->blk_mat, blk_mat.data(), blk_mat.size(), &total);
  if (e == hipSuccess) e = upload(b->state, zeros.data(), zeros.size(), &total);
  int32_t per_cu = 0;
  if (e == hipSuccess)
    e = vt == 0 ? race::race_flow_occupancy<double>(kt, threads, wmax, &per_cu)
                : race::race_flow_occupancy<float>(kt, threads, wmax, &per_cu);
  if (e != hipSuccess) {
    batch_release(b);
    delete b;
    return hip_fail(e, "batch setup");
  }
  b->grid = std::max(1, std::min(b->n_tickets, std::max(1, per_cu) * s[0]->n_cus));
  *out = b;
  return RACE_OK;
}

int race_batch_bind(race_batch_t b, const double* const* X, double* const* Y) {
  if (!b || !X || !Y) return fail(RACE_EINVAL, "NULL argument");
  for (int32_t m = 0; m < b->count; ++m)
    if (!X[m] || !Y[m]) return fail(RACE_EINVAL, "x/y pointer of matrix " + std::to_string(m) + " is NULL");
  hipError_t e = hipSuccess;
  const size_t bytes = b->value_type == 0 ? sizeof(race::BatchMat<double>) * b->count
                                          : sizeof(race::BatchMat<float>) * b->count;
  if (!b->d_mats) {
    e = hipMalloc(&b->d_mats, bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  }
  if (b->tiled && !b->tiles_x.p) {
    int64_t total = 0;
    b->tile_base.resize(b->count);
    for (int32_t m = 0; m < b->count; ++m) {
      b->tile_base[m] = total;
      total += static_cast<int64_t>(b->mats[m]->tree.n) * b->k;
    }
    for (DevBuf<double>* t : {&b->tiles_x, &b->tiles_y}) {
      e = hipMalloc(&t->p, std::max<int64_t>(1, total) * sizeof(double));
      if (e != hipSuccess) return hip_fail(e, "hipMalloc of the column tiles");
      t->count = static_cast<size_t>(total);
    }
  }
  auto tiles = [&](auto& bm, int32_t m) {
    bm.n = b->mats[m]->tree.n;
    bm.xt = b->tiled ? b->tiles_x.p + b->tile_base[m] : nullptr;
    bm.yt = b->tiled ? b->tiles_y.p + b->tile_base[m] : nullptr;
  };
  if (b->value_type == 0) {
    std::vector<race::BatchMat<double>> h(b->count);
    for (int32_t m = 0; m < b->count; ++m) {
      h[m] = batch_mat<double>(b->mats[m], b->mats[m]->lane_diag64.p, b->mats[m]->sell_val64.p,
                               b->state.p + b->unit_base[m], X[m], Y[m]);
      tiles(h[m], m);
      if (b->mats[m]->expanded) h[m].n = 0;  // not in the RACE passes (no tickets, no tile copies)
    }
    e = hipMemcpy(b->d_mats, h.data(), bytes, hipMemcpyHostToDevice);
  } else {
    std::vector<race::BatchMat<float>> h(b->count);
    for (int32_t m = 0; m < b->count; ++m) {
      h[m] = batch_mat<float>(b->mats[m], b->mats[m]->lane_diag32.p, b->mats[m]->sell_val32.p,
                              b->state.p + b->unit_base[m], X[m], Y[m]);
      tiles(h[m], m);
      if (b->mats[m]->expanded) h[m].n = 0;  // not in the RACE passes (no tickets, no tile copies)
    }
    e = hipMemcpy(b->d_mats, h.data(), bytes, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  b->exp_x.clear();
  b->exp_y.clear();
  for (const int32_t m : b->exp_members) {
    b->exp_x.push_back(X[m]);
    b->exp_y.push_back(Y[m]);
  }
  if (b->k == 1 && !b->exp_members.empty()) {
    const size_t ne = b->exp_members.size();
    const size_t bbytes = b->value_type == 0 ? sizeof(race::BlockMat<double>) * ne : sizeof(race::BlockMat<float>) * ne;
    if (!b->d_bmats) {
      e = hipMalloc(&b->d_bmats, bbytes);
      if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    }
    auto fill = [&](auto& h, auto val_of) {
      int32_t base = 0;
      for (size_t i = 0; i < ne; ++i) {
        const int32_t m = b->exp_members[i];
        const race_schedule_t sm = b->mats[m];
        h[i] = {sm->exp_blk.p, sm->exp_rp.p, sm->exp_col.p, val_of(sm), X[m], Y[m], base};
        base += sm->exp_nblk;
      }
      return hipMemcpy(b->d_bmats, h.data(), bbytes, hipMemcpyHostToDevice);
    };
    if (b->value_type == 0) {
      std::vector<race::BlockMat<double>> h(ne);
      e = fill(h, [](race_schedule_t sm) -> const double* { return sm->exp_val64.p; });
    } else {
      std::vector<race::BlockMat<float>> h(ne);
      e = fill(h, [](race_schedule_t sm) -> const float* { return sm->exp_val32.p; });
    }
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  }
  // capture reset + persistent kernel once; replays reuse it
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  if (!b->cap) {
    e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
  }
  // kernel attributes of every width a pass uses (the tile, and a narrower last tile)
  for (const int32_t kc : {b->kt, b->k % b->kt}) {
    if (kc == 0) continue;
    e = b->value_type == 0 ? race::prepare_race_batch<double>(kc) : race::prepare_race_batch<float>(kc);
    if (e != hipSuccess) break;
  }
  if (e != hipSuccess) return hip_fail(e, "batch kernel attributes");
  e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  hipError_t le = batch_enqueue(b, b->cap);
  e = hipStreamEndCapture(b->cap, &b->graph);
  if (le != hipSuccess) return hip_fail(le, "batch launch under capture");
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  b->bound = true;
  return RACE_OK;
}

int race_batch_run(race_batch_t b, int32_t use_graph, void* stream) {
  if (!b) return fail(RACE_EINVAL, "batch is NULL");
  if (!b->bound) return fail(RACE_ESTATE, "race_batch_bind has not been called");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = use_graph ? hipGraphLaunch(b->exec, st) : batch_enqueue(b, st);
  if (e != hipSuccess) return hip_fail(e, use_graph ? "hipGraphLaunch" : "batch launch");
  return RACE_OK;
}

int race_batch_check(race_batch_t b) {
  if (!b) return fail(RACE_EINVAL, "batch is NULL");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  uint32_t status = 0;
  e = hipMemcpy(&status, b->state.p + b->state.count - 4, sizeof(uint32_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  if (status) return fail(RACE_EINTERNAL, "a dataflow wait of the batch gave up (bounded spin exceeded)");
  return RACE_OK;
}

int race_batch_info(race_batch_t b, int32_t* n_tickets, int32_t* grid, int32_t* wmax) {
  if (!b) return fail(RACE_EINVAL, "batch is NULL");
  if (n_tickets) *n_tickets = b->n_tickets;
  if (grid) *grid = b->grid;
  if (wmax) *wmax = b->wmax;
  return RACE_OK;
}

void race_batch_destroy(race_batch_t b) {
  if (!b) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(b->device);
  batch_release(b);
  (void)hipSetDevice(cur);
  delete b;
}

static int pick_lpr(int32_t n, int64_t nnz) {
  const double mean = n > 0 ? static_cast<double>(nnz) / n : 1.0;
  int lpr = 1;
  while (lpr < 64 && lpr < mean / 2.0) lpr *= 2;
  return lpr;
}

static int csr_create(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val, int32_t lpr,
                      bool upper, race_csr_t* out) {
  if (!out) return fail(RACE_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_crs(n, row_ptr, col, upper);
  if (rc) return rc;
  const int64_t nnz = n > 0 ? row_ptr[n] : 0;
  if (nnz > 0 && !val) return fail(RACE_EINVAL, "val is NULL");
  if (lpr == 0) lpr = pick_lpr(n, nnz);
  if (lpr < 0 && (upper || (lpr != -4 && lpr != -8 && lpr != -16)))
    return fail(RACE_EINVAL, "row blocks take lanes_per_row -4, -8 or -16, full matrices only");
  if (lpr > 0 && lpr != 1 && lpr != 2 && lpr != 4 && lpr != 8 && lpr != 16 && lpr != 32 && lpr != 64)
    return fail(RACE_EINVAL, "lanes_per_row must be a power of two in 1..64");
  race_csr* h = new (std::nothrow) race_csr();
  if (!h) return fail(RACE_ENOMEM, "out of host memory");
  h->n = n;
  h->lpr = lpr;
  h->atomic = upper;
  hipError_t e = hipGetDevice(&h->device);
  int64_t total = 0;
  if (e == hipSuccess) e = upload(h->rp, row_ptr, static_cast<size_t>(n) + 1, &total);
  if (e == hipSuccess) e = upload(h->col, col, static_cast<size_t>(nnz), &total);
  if (e == hipSuccess) e = upload(h->val, val, static_cast<size_t>(nnz), &total);
  if (e == hipSuccess && lpr < 0) {
    std::vector<int32_t> blk;
    race::csr_row_blocks(n, row_ptr, -lpr, blk);
    h->n_blk = static_cast<int32_t>(blk.size()) - 1;
    e = upload(h->blk, blk.data(), blk.size(), &total);
  }
  if (e != hipSuccess) {
    race_csr_destroy(h);
    return hip_fail(e, "baseline upload");
  }
  *out = h;
  return RACE_OK;
}

int race_csr_create(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val, int32_t lanes_per_row,
                    race_csr_t* out) {
  return csr_create(n, row_ptr, col, val, lanes_per_row, false, out);
}

int race_atomic_create(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                       int32_t lanes_per_row, race_csr_t* out) {
  return csr_create(n, row_ptr, col, val, lanes_per_row, true, out);
}

int race_csr_spmv(race_csr_t h, const double* x, double* y, void* stream) {
  if (!h) return fail(RACE_EINVAL, "handle is NULL");
  if (h->atomic) return fail(RACE_ESTATE, "handle holds an upper triangle; use race_symm_spmv_atomic");
  if (h->n > 0 && (!x || !y)) return fail(RACE_EINVAL, "x or y is NULL");
  hipError_t e =
      h->lpr < 0 ? race::launch_csr_block<double>(h->n_blk, h->blk.p, h->rp.p, h->col.p, h->val.p, x, y, -h->lpr,
                                                  static_cast<hipStream_t>(stream))
                 : race::launch_csr_spmv<double>(h->n, h->rp.p, h->col.p, h->val.p, x, y, h->lpr,
                                                 static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "CSR SpMV launch");
  return RACE_OK;
}

int race_symm_spmv_atomic(race_csr_t h, const double* x, double* y, void* stream) {
  if (!h) return fail(RACE_EINVAL, "handle is NULL");
  if (!h->atomic) return fail(RACE_ESTATE, "handle holds a full matrix; use race_csr_spmv");
  if (h->n > 0 && (!x || !y)) return fail(RACE_EINVAL, "x or y is NULL");
  hipError_t e =
      race::launch_atomic_symm(h->n, h->rp.p, h->col.p, h->val.p, x, y, h->lpr, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "atomic SymmSpMV launch");
  return RACE_OK;
}

void race_csr_destroy(race_csr_t h) {
  if (!h) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (h->device >= 0) (void)hipSetDevice(h->device);
  release(h->rp);
  release(h->col);
  release(h->blk);
  release(h->val);
  (void)hipSetDevice(cur);
  delete h;
}

}  // extern "C"
