// gfx950 Gauss-Seidel sweep over a distance-1 RACE schedule: one launch per
// phase, one wavefront per leaf or (phases of more leaves than the CUs can
// hold wavefronts, windows up to kGsQuadMaxWindow entries) four leaves per
// wavefront (leaves of one phase share no edge, so they run at the same
// time), the rows of a leaf in order; or one dataflow launch per sweep.
// The Kaczmarz sweep over a distance-2 schedule runs the same ways (one or
// four leaves per wavefront in phase launches, one leaf per ticket in the
// dataflow launch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "gs_kernels.hpp"

namespace race {
namespace dev {

constexpr int kGsLanes = 64;
constexpr int kGsAhead = 8;  // rows whose entries are in flight ahead of the running row (divides 64)

// Load of a word no kernel writes, at an index that is the same in every
// lane: a scalar load through the constant address space.
template <typename T>
__device__ __forceinline__ T gs_uniform(const T* p, int64_t i) {
  using ConstT = const __attribute__((address_space(4))) T;
  return ((ConstT*)p)[i];
}

// Sum over the 64 lanes, returned in every lane: within each row of 16
// lanes by four DPP steps (quad swaps, half-row and row mirrors), then the
// four row sums through readlane.
template <int kCtrl>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), kCtrl, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);  // row_half_mirror
  v += dpp_mov<0x140>(v);  // row_mirror
  const double r0 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 0),
                                     __builtin_amdgcn_readlane(__double2loint(v), 0));
  const double r1 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 16),
                                     __builtin_amdgcn_readlane(__double2loint(v), 16));
  const double r2 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 32),
                                     __builtin_amdgcn_readlane(__double2loint(v), 32));
  const double r3 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 48),
                                     __builtin_amdgcn_readlane(__double2loint(v), 48));
  return (r0 + r1) + (r2 + r3);
}

// Per-row metadata of 64 consecutive rows of the sweep, one row per lane:
// the row's entry range, right-hand side and diagonal.  A row's values are
// then taken with readlane (scalar registers) at no memory wait: scalar
// loads inside the row loop would make every LDS wait (the same counter)
// wait for them as well.
struct GsMeta {
  int32_t e0 = 0, e1 = 0;
  double b = 0.0, d = 1.0;
};

// Rows t0 .. t0 + 63 of the sweep (row t of the sweep is lo + t, or hi - 1 - t backward).
template <bool kBackward>
__device__ __forceinline__ void gs_load_meta(const GsArgs& a, const double* __restrict__ bvec, int32_t lo, int32_t hi,
                                             int32_t t0, int32_t lane, GsMeta& m) {
  const int32_t t = t0 + lane;
  if (t < hi - lo) {
    const int32_t i = kBackward ? hi - 1 - t : lo + t;
    m.e0 = a.row_ptr[i];
    m.e1 = a.row_ptr[i + 1];
    m.b = bvec[i];
    m.d = a.diag[i];
  }
}

// x as the sweep reads and writes it: plain, or (kCoherent: several
// workgroups of one launch update x) agent-scope loads and stores, which are
// coherent across the XCDs.
template <bool kCoherent>
__device__ __forceinline__ double gs_x_load(const double* p) {
  if constexpr (kCoherent) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return *p;
}
template <bool kCoherent>
__device__ __forceinline__ void gs_x_store(double* p, double v) {
  if constexpr (kCoherent) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else *p = v;
}

// Stages a leaf's window in LDS: x of its own rows lo .. lo + R - 1 into
// slots 0 .. R - 1, x of its halo rows (halo[0 .. H - 1]) into slots R ..
// R + H - 1; kLanes lanes (lane j), kStage loads per lane in flight before
// their LDS writes (one HBM round trip per kLanes * kStage entries, two for
// the halo: indices, then values).  kCoherent: agent-scope loads (x is
// updated by other workgroups of the same launch).
template <int kLanes, bool kCoherent>
__device__ __forceinline__ void stage_window(const double* __restrict__ x, const int32_t* __restrict__ halo,
                                             int32_t lo, int32_t R, int32_t H, int32_t j, double* xw) {
  constexpr int kStage = 8;
  auto load = [](const double* p) { return gs_x_load<kCoherent>(p); };
  for (int32_t s0 = 0; s0 < R; s0 += kLanes * kStage) {
    double v[kStage];
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int32_t s = s0 + u * kLanes + j;
      v[u] = s < R ? load(x + lo + s) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int32_t s = s0 + u * kLanes + j;
      if (s < R) xw[s] = v[u];
    }
  }
  for (int32_t s0 = 0; s0 < H; s0 += kLanes * kStage) {
    int32_t r[kStage];
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int32_t s = s0 + u * kLanes + j;
      r[u] = s < H ? halo[s] : -1;
    }
    double v[kStage];
#pragma unroll
    for (int u = 0; u < kStage; ++u) v[u] = r[u] >= 0 ? load(x + r[u]) : 0.0;
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int32_t s = s0 + u * kLanes + j;
      if (s < H) xw[R + s] = v[u];
    }
  }
}

// Between two rows of a sweep inside a one-wavefront workgroup: the LDS
// runs a wavefront's instructions in the order they issue, so the next
// row's reads see this row's writes without a wait; the signal fence keeps
// the compiler from moving LDS accesses across the row boundary.
__device__ __forceinline__ void lds_row_order() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

__device__ __forceinline__ int32_t lane_value(int32_t v, int32_t l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ double lane_value(double v, int32_t l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// The first 64 off-diagonal entries of one row as the wavefront holds them
// (lane l takes entry l; lanes past the row hold slot 0 and value 0).
struct GsRow {
  double v = 0.0;
  uint32_t sl = 0;
};

__device__ __forceinline__ void gs_load_row(const GsArgs& a, const GsMeta& m, int32_t l, int32_t lane, GsRow& r) {
  const int32_t e = lane_value(m.e0, l) + lane;
  r.v = 0.0;
  r.sl = 0u;
  if (e < lane_value(m.e1, l)) {
    r.v = a.val[e];
    r.sl = a.slot[e];
  }
}

// One leaf: stage the window (own rows and halo) in LDS, update the rows in
// order (backward: last row first) with
//   x_i = (b_i - sum_j a_ij x_j) / a_ii
// reading every x_j from the window and writing x_i into it, then store the
// own rows back.  The entries of the next kGsAhead rows are in flight while
// a row is summed (they do not depend on x); the metadata of the current
// and the next 64 rows sits in lanes.
template <bool kBackward>
__global__ void __launch_bounds__(kGsLanes) gs_leaf_kernel(GsArgs a, int32_t leaf0, const double* __restrict__ bvec,
                                                          double* __restrict__ x) {
  extern __shared__ double xw[];
  const int32_t leaf = leaf0 + static_cast<int32_t>(blockIdx.x);
  const int32_t lane = static_cast<int32_t>(threadIdx.x);
  const int32_t lo = gs_uniform(a.leaf_lo, leaf), hi = gs_uniform(a.leaf_hi, leaf);
  const int32_t h0 = gs_uniform(a.halo_ptr, leaf), h1 = gs_uniform(a.halo_ptr, leaf + 1);
  const int32_t R = hi - lo, H = h1 - h0;
  stage_window<kGsLanes, false>(x, a.halo + h0, lo, R, H, lane, xw);
  GsMeta cur, next;
  gs_load_meta<kBackward>(a, bvec, lo, hi, 0, lane, cur);
  gs_load_meta<kBackward>(a, bvec, lo, hi, kGsLanes, lane, next);
  GsRow ring[kGsAhead];
#pragma unroll
  for (int p = 0; p < kGsAhead; ++p)
    if (p < R) gs_load_row(a, cur, p, lane, ring[p]);
  __syncthreads();
  for (int32_t t0 = 0; t0 < R; t0 += kGsAhead) {
#pragma unroll
    for (int p = 0; p < kGsAhead; ++p) {
      const int32_t t = t0 + p;
      if (t < R) {
        const int32_t i = kBackward ? hi - 1 - t : lo + t;
        const int32_t l = t & (kGsLanes - 1);
        double s = ring[p].v * xw[ring[p].sl];
        // entries past the first 64 (long rows) are loaded when the row runs
        const int32_t e1 = lane_value(cur.e1, l);
        for (int32_t e = lane_value(cur.e0, l) + kGsLanes + lane; e < e1; e += kGsLanes) s += a.val[e] * xw[a.slot[e]];
        const double bi = lane_value(cur.b, l), di = lane_value(cur.d, l);
        const int32_t tn = t + kGsAhead;
        // kGsAhead divides 64, so row tn is in the current or the next chunk
        if (tn < R) gs_load_row(a, (tn & (kGsLanes - 1)) >= l ? cur : next, tn & (kGsLanes - 1), lane, ring[p]);
        const double xi = (bi - wave_sum(s)) * di;
        if (lane == 0) xw[i - lo] = xi;
        lds_row_order();
        if (l == kGsLanes - 1) {
          // the chunk of rows t - 63 .. t is done: shift, fetch the one after next
          cur = next;
          gs_load_meta<kBackward>(a, bvec, lo, hi, t + 1 + kGsLanes, lane, next);
        }
      }
    }
  }
  for (int32_t s = lane; s < R; s += kGsLanes) x[lo + s] = xw[s];
}

// Kaczmarz sweep of one leaf (a distance-2 phase: the windows of its leaves
// are disjoint, so they run at the same time): stage the window in LDS,
// then for every row in order (backward: last row first)
//   c = omega (b_i - a_i . x) / |a_i|^2   (0 for a row with no value; the
//       layout holds the reciprocal squared norms),
//   x_j += c a_ij for every stored column j of the full row, x_i += c a_ii,
// and store the whole window back.  The dot product is summed across the
// lanes (one off-diagonal entry each, 64 at a time) plus the diagonal term;
// each lane then updates the slot of its own entry (the columns of a row
// are distinct, so no two lanes write one slot).  The entries of the next
// kGsAhead rows are in flight while a row runs, as in the Gauss-Seidel
// kernel.
struct KzMeta {
  int32_t e0 = 0, e1 = 0;
  double b = 0.0, d = 0.0, q = 0.0;
};

template <bool kBackward>
__device__ __forceinline__ void kz_load_meta(const GsArgs& a, const double* __restrict__ bvec, int32_t lo, int32_t hi,
                                             int32_t t0, int32_t lane, KzMeta& m) {
  const int32_t t = t0 + lane;
  if (t < hi - lo) {
    const int32_t i = kBackward ? hi - 1 - t : lo + t;
    m.e0 = a.row_ptr[i];
    m.e1 = a.row_ptr[i + 1];
    m.b = bvec[i];
    m.d = a.diag[i];
    m.q = a.nrm[i];
  }
}

__device__ __forceinline__ void kz_load_row(const GsArgs& a, const KzMeta& m, int32_t l, int32_t lane, GsRow& r) {
  const int32_t e = lane_value(m.e0, l) + lane;
  r.v = 0.0;
  r.sl = 0u;
  if (e < lane_value(m.e1, l)) {
    r.v = a.val[e];
    r.sl = a.slot[e];
  }
}

// One leaf on the wavefront (kCoherent: x through agent-scope loads and
// stores, for the dataflow launch).
template <bool kBackward, bool kCoherent>
__device__ __forceinline__ void kacz_leaf(const GsArgs& a, int32_t leaf, double omega, const double* __restrict__ bvec,
                                          double* __restrict__ x, double* xw) {
  const int32_t lane = static_cast<int32_t>(threadIdx.x);
  const int32_t lo = gs_uniform(a.leaf_lo, leaf), hi = gs_uniform(a.leaf_hi, leaf);
  const int32_t h0 = gs_uniform(a.halo_ptr, leaf), h1 = gs_uniform(a.halo_ptr, leaf + 1);
  const int32_t R = hi - lo, H = h1 - h0;
  stage_window<kGsLanes, kCoherent>(x, a.halo + h0, lo, R, H, lane, xw);
  KzMeta cur, next;
  kz_load_meta<kBackward>(a, bvec, lo, hi, 0, lane, cur);
  kz_load_meta<kBackward>(a, bvec, lo, hi, kGsLanes, lane, next);
  GsRow ring[kGsAhead];
#pragma unroll
  for (int p = 0; p < kGsAhead; ++p)
    if (p < R) kz_load_row(a, cur, p, lane, ring[p]);
  __syncthreads();
  for (int32_t t0 = 0; t0 < R; t0 += kGsAhead) {
#pragma unroll
    for (int p = 0; p < kGsAhead; ++p) {
      const int32_t t = t0 + p;
      if (t < R) {
        const int32_t i = kBackward ? hi - 1 - t : lo + t;
        const int32_t l = t & (kGsLanes - 1);
        const int32_t e0 = lane_value(cur.e0, l), e1 = lane_value(cur.e1, l);
        const GsRow row = ring[p];
        const double bi = lane_value(cur.b, l), di = lane_value(cur.d, l), qi = lane_value(cur.q, l);
        // the diagonal term rides in lane 0 of the sum
        const double xd = xw[i - lo];
        double s = row.v * xw[row.sl] + (lane == 0 ? di * xd : 0.0);
        // entries past the first 64 (long rows) are loaded when the row runs
        for (int32_t e = e0 + kGsLanes + lane; e < e1; e += kGsLanes) s += a.val[e] * xw[a.slot[e]];
        const int32_t tn = t + kGsAhead;
        // kGsAhead divides 64, so row tn is in the current or the next chunk
        if (tn < R) kz_load_row(a, (tn & (kGsLanes - 1)) >= l ? cur : next, tn & (kGsLanes - 1), lane, ring[p]);
        const double c = omega * (bi - wave_sum(s)) * qi;  // qi = 1 / |a_i|^2, 0 for a row with no value
        if (lane < e1 - e0) xw[row.sl] += c * row.v;
        for (int32_t e = e0 + kGsLanes + lane; e < e1; e += kGsLanes) xw[a.slot[e]] += c * a.val[e];
        if (lane == 0) xw[i - lo] = xd + c * di;
        lds_row_order();
        if (l == kGsLanes - 1) {
          cur = next;
          kz_load_meta<kBackward>(a, bvec, lo, hi, t + 1 + kGsLanes, lane, next);
        }
      }
    }
  }
  for (int32_t s = lane; s < R; s += kGsLanes) gs_x_store<kCoherent>(x + lo + s, xw[s]);
  for (int32_t s = lane; s < H; s += kGsLanes) gs_x_store<kCoherent>(x + a.halo[h0 + s], xw[R + s]);
}

template <bool kBackward>
__global__ void __launch_bounds__(kGsLanes) kacz_leaf_kernel(GsArgs a, int32_t leaf0, double omega,
                                                            const double* __restrict__ bvec, double* __restrict__ x) {
  extern __shared__ double xw[];
  kacz_leaf<kBackward, false>(a, leaf0 + static_cast<int32_t>(blockIdx.x), omega, bvec, x, xw);
}

// Four leaves per wavefront: lanes 16 g .. 16 g + 15 run leaf 4 b + g of
// the phase, so a phase of many small leaves needs a quarter of the
// wavefronts (the wave slots of a CU, not the LDS, bound how many leaves run
// at once with one leaf per wavefront).  The rows of the four leaves advance
// together; a group past its leaf's last row computes on empty rows and
// writes nothing.  A group's lanes take a row's entries 16 at a time (the
// first 32 are loaded ahead, kQAhead rows in advance), reduce within the
// group by four DPP steps (quad swaps, half-row and row mirrors, which stay
// inside a row of 16 lanes) and get the row's metadata from the lane that
// holds it (ds_bpermute).
// Bounded wait of the dataflow sweeps: about one second of the 100 MHz
// wall clock for one ticket's list (a chain of long leaves can legitimately
// take tens of milliseconds).
constexpr uint64_t kGsWaitTicks = 100000000ull;
constexpr int kQLanes = 16;
constexpr int kQAhead = 4;  // divides 16

__device__ __forceinline__ double group_sum(double v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);  // row_half_mirror
  v += dpp_mov<0x140>(v);  // row_mirror
  return v;
}

// Rows t0 .. t0 + 15 of the group's leaf, one per lane j of the group.
template <bool kBackward>
__device__ __forceinline__ void gsq_load_meta(const GsArgs& a, const double* __restrict__ bvec, int32_t lo, int32_t R,
                                              int32_t t0, int32_t j, GsMeta& m) {
  m = GsMeta{};
  const int32_t t = t0 + j;
  if (t < R) {
    const int32_t i = kBackward ? lo + R - 1 - t : lo + t;
    m.e0 = a.row_ptr[i];
    m.e1 = a.row_ptr[i + 1];
    m.b = bvec[i];
    m.d = a.diag[i];
  }
}

struct GsQRow {
  double v0 = 0.0, v1 = 0.0;
  uint32_t s0 = 0, s1 = 0;
};

__device__ __forceinline__ void gsq_load_row(const GsArgs& a, const GsMeta& m, int32_t src, int32_t j, GsQRow& r) {
  const int32_t e0 = __shfl(m.e0, src), e1 = __shfl(m.e1, src);
  r = GsQRow{};
  if (e0 + j < e1) {
    r.v0 = a.val[e0 + j];
    r.s0 = a.slot[e0 + j];
  }
  if (e0 + kQLanes + j < e1) {
    r.v1 = a.val[e0 + kQLanes + j];
    r.s1 = a.slot[e0 + kQLanes + j];
  }
}

// Leaves first .. first + cnt - 1 (cnt <= 4) on the wavefront, group g on
// leaf first + g; smem holds 4 windows of wmax entries.
template <bool kBackward, bool kCoherent>
__device__ __forceinline__ void gs_quad_leaves(const GsArgs& a, int32_t first, int32_t cnt, int32_t wmax,
                                               const double* __restrict__ bvec, double* __restrict__ x,
                                               double* smem) {
  const int32_t lane = static_cast<int32_t>(threadIdx.x);
  const int32_t g = lane / kQLanes, j = lane % kQLanes, base = lane - j;
  const bool live = g < cnt;
  const int32_t leaf = first + (live ? g : cnt - 1);
  double* xw = smem + static_cast<size_t>(g) * wmax;
  const int32_t lo = a.leaf_lo[leaf], h0 = a.halo_ptr[leaf];
  const int32_t R = live ? a.leaf_hi[leaf] - lo : 0, H = live ? a.halo_ptr[leaf + 1] - h0 : 0;
  stage_window<kQLanes, kCoherent>(x, a.halo + h0, lo, R, H, j, xw);
  int32_t rmax = R;
  rmax = max(rmax, __shfl_xor(rmax, 16));
  rmax = max(rmax, __shfl_xor(rmax, 32));
  rmax = __builtin_amdgcn_readfirstlane(rmax);
  GsMeta cur, next;
  gsq_load_meta<kBackward>(a, bvec, lo, R, 0, j, cur);
  gsq_load_meta<kBackward>(a, bvec, lo, R, kQLanes, j, next);
  GsQRow ring[kQAhead];
#pragma unroll
  for (int p = 0; p < kQAhead; ++p)
    if (p < rmax) gsq_load_row(a, cur, base + p, j, ring[p]);
  __syncthreads();
  for (int32_t t0 = 0; t0 < rmax; t0 += kQAhead) {
#pragma unroll
    for (int p = 0; p < kQAhead; ++p) {
      const int32_t t = t0 + p;
      if (t < rmax) {
        const int32_t l = t & (kQLanes - 1);
        const int32_t src = base + l;
        double s = ring[p].v0 * xw[ring[p].s0] + ring[p].v1 * xw[ring[p].s1];
        // entries past the first 32 (long rows) are loaded when the row runs
        const int32_t e1 = __shfl(cur.e1, src);
        for (int32_t e = __shfl(cur.e0, src) + 2 * kQLanes + j; e < e1; e += kQLanes) s += a.val[e] * xw[a.slot[e]];
        const double bi = __shfl(cur.b, src), di = __shfl(cur.d, src);
        const int32_t tn = t + kQAhead;
        // kQAhead divides 16, so row tn is in the current or the next chunk
        if (tn < rmax) {
          const int32_t ln = tn & (kQLanes - 1);
          gsq_load_row(a, ln >= l ? cur : next, base + ln, j, ring[p]);
        }
        const double xi = (bi - group_sum(s)) * di;
        if (t < R && j == 0) xw[kBackward ? R - 1 - t : t] = xi;
        lds_row_order();
        if (l == kQLanes - 1) {
          // the chunk of rows t - 15 .. t is done: shift, fetch the one after next
          cur = next;
          gsq_load_meta<kBackward>(a, bvec, lo, R, t + 1 + kQLanes, j, next);
        }
      }
    }
  }
  for (int32_t s = j; s < R; s += kQLanes) gs_x_store<kCoherent>(x + lo + s, xw[s]);
}

template <bool kBackward>
__global__ void __launch_bounds__(kGsLanes) gs_quad_kernel(GsArgs a, int32_t leaf0, int32_t count, int32_t wmax,
                                                          const double* __restrict__ bvec, double* __restrict__ x) {
  extern __shared__ double smem[];
  const int32_t first = static_cast<int32_t>(blockIdx.x) * 4;
  gs_quad_leaves<kBackward, false>(a, leaf0 + first, min(4, count - first), wmax, bvec, x, smem);
}

// Four Kaczmarz leaves per wavefront, as gs_quad_leaves: lanes 16 g .. 16 g
// + 15 run leaf first + g, rows advance together, a group past its leaf's
// last row computes on an empty row (coefficient 0) and writes nothing.
template <bool kBackward>
__global__ void __launch_bounds__(kGsLanes) kacz_quad_kernel(GsArgs a, int32_t leaf0, int32_t count, int32_t wmax,
                                                            double omega, const double* __restrict__ bvec,
                                                            double* __restrict__ x) {
  extern __shared__ double smem[];
  const int32_t first = leaf0 + static_cast<int32_t>(blockIdx.x) * 4;
  const int32_t cnt = min(4, leaf0 + count - first);
  const int32_t lane = static_cast<int32_t>(threadIdx.x);
  const int32_t g = lane / kQLanes, j = lane % kQLanes, base = lane - j;
  const bool live = g < cnt;
  const int32_t leaf = first + (live ? g : cnt - 1);
  double* xw = smem + static_cast<size_t>(g) * wmax;
  const int32_t lo = a.leaf_lo[leaf], h0 = a.halo_ptr[leaf];
  const int32_t R = live ? a.leaf_hi[leaf] - lo : 0, H = live ? a.halo_ptr[leaf + 1] - h0 : 0;
  stage_window<kQLanes, false>(x, a.halo + h0, lo, R, H, j, xw);
  int32_t rmax = R;
  rmax = max(rmax, __shfl_xor(rmax, 16));
  rmax = max(rmax, __shfl_xor(rmax, 32));
  rmax = __builtin_amdgcn_readfirstlane(rmax);
  // per-row metadata, lane j of the group holding row t0 + j of its leaf
  KzMeta cur, next;
  auto load_meta = [&](int32_t t0, KzMeta& m) {
    m = KzMeta{};
    const int32_t t = t0 + j;
    if (t < R) {
      const int32_t i = kBackward ? lo + R - 1 - t : lo + t;
      m.e0 = a.row_ptr[i];
      m.e1 = a.row_ptr[i + 1];
      m.b = bvec[i];
      m.d = a.diag[i];
      m.q = a.nrm[i];
    }
  };
  auto load_row = [&](const KzMeta& m, int32_t src, GsQRow& r) {
    const int32_t e0 = __shfl(m.e0, src), e1 = __shfl(m.e1, src);
    r = GsQRow{};
    if (e0 + j < e1) {
      r.v0 = a.val[e0 + j];
      r.s0 = a.slot[e0 + j];
    }
    if (e0 + kQLanes + j < e1) {
      r.v1 = a.val[e0 + kQLanes + j];
      r.s1 = a.slot[e0 + kQLanes + j];
    }
  };
  load_meta(0, cur);
  load_meta(kQLanes, next);
  GsQRow ring[kQAhead];
#pragma unroll
  for (int p = 0; p < kQAhead; ++p)
    if (p < rmax) load_row(cur, base + p, ring[p]);
  __syncthreads();
  for (int32_t t0 = 0; t0 < rmax; t0 += kQAhead) {
#pragma unroll
    for (int p = 0; p < kQAhead; ++p) {
      const int32_t t = t0 + p;
      if (t < rmax) {
        const int32_t l = t & (kQLanes - 1);
        const int32_t src = base + l;
        const int32_t e0 = __shfl(cur.e0, src), e1 = __shfl(cur.e1, src);
        const double bi = __shfl(cur.b, src), di = __shfl(cur.d, src), qi = __shfl(cur.q, src);
        const GsQRow row = ring[p];
        const int32_t il = kBackward ? R - 1 - t : t;  // the row's slot (t < R)
        const double xd = t < R ? xw[il] : 0.0;
        double s = row.v0 * xw[row.s0] + row.v1 * xw[row.s1] + (j == 0 ? di * xd : 0.0);
        // entries past the first 32 (long rows) are loaded when the row runs
        for (int32_t e = e0 + 2 * kQLanes + j; e < e1; e += kQLanes) s += a.val[e] * xw[a.slot[e]];
        const int32_t tn = t + kQAhead;
        // kQAhead divides 16, so row tn is in the current or the next chunk
        if (tn < rmax) {
          const int32_t ln = tn & (kQLanes - 1);
          load_row(ln >= l ? cur : next, base + ln, ring[p]);
        }
        const double c = omega * (bi - group_sum(s)) * qi;
        if (e0 + j < e1) xw[row.s0] += c * row.v0;
        if (e0 + kQLanes + j < e1) xw[row.s1] += c * row.v1;
        for (int32_t e = e0 + 2 * kQLanes + j; e < e1; e += kQLanes) xw[a.slot[e]] += c * a.val[e];
        if (t < R && j == 0) xw[il] = xd + c * di;
        lds_row_order();
        if (l == kQLanes - 1) {
          cur = next;
          load_meta(t + 1 + kQLanes, next);
        }
      }
    }
  }
  for (int32_t s = j; s < R; s += kQLanes) x[lo + s] = xw[s];
  for (int32_t s = j; s < H; s += kQLanes) x[a.halo[h0 + s]] = xw[R + s];
}

// Waits until every ticket in ticket t's list has published.  A wait that
// runs past kGsWaitTicks sets *status (reported to the host) and *drain to
// the launch's epoch and goes on; every other wait of the same launch then
// stops at once, so the grid drains quickly.
__device__ __forceinline__ void wait_tickets(const GsFlowArgs& f, int32_t t, int32_t lane) {
  const int32_t d0 = gs_uniform(f.dep_ptr, t), d1 = gs_uniform(f.dep_ptr, t + 1);
  for (int32_t i = d0 + lane; i < d1; i += kGsLanes) {
    const uint32_t* flag = f.flags + f.dep_idx[i];
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != f.epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (__hip_atomic_load(f.drain, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == f.epoch) break;
      if (__builtin_amdgcn_s_memrealtime() - t0 > kGsWaitTicks) {
        atomicOr(f.status, 1u);
        __hip_atomic_store(f.drain, f.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
}

// A whole sweep in one launch (dataflow, see GsFlowArgs): workgroup w runs
// tickets w, w + grid, ... in order; before a ticket it waits until every
// ticket in its list has published (bounded, see wait_tickets, so the grid
// always drains), after it every x store has completed before the ticket's
// flag is set.  The launch is cooperative (every workgroup resident), so the
// lowest unfinished ticket always has a running owner whose own earlier
// tickets are done.  (Claiming tickets from one atomic counter instead
// serialises the claims at that address: 3.6 ms per 128^3 sweep against
// 0.61 ms.)
__global__ void __launch_bounds__(kGsLanes) gs_flow_kernel(GsArgs a, GsFlowArgs f, int32_t wmax,
                                                          const double* __restrict__ bvec, double* __restrict__ x) {
  extern __shared__ double smem[];
  const int32_t lane = static_cast<int32_t>(threadIdx.x);
  for (int32_t t = static_cast<int32_t>(blockIdx.x); t < f.n_tickets; t += static_cast<int32_t>(gridDim.x)) {
    wait_tickets(f, t, lane);
    const int32_t item = gs_uniform(f.ticket_item, t);
    const int32_t first = gs_uniform(f.item_leaf0, item), cnt = gs_uniform(f.item_count, item);
    if (gs_uniform(f.ticket_back, t))
      gs_quad_leaves<true, true>(a, first, cnt, wmax, bvec, x, smem);
    else
      gs_quad_leaves<false, true>(a, first, cnt, wmax, bvec, x, smem);
    // every lane's x stores complete before the flag
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __syncthreads();
    if (lane == 0) __hip_atomic_store(f.flags + t, f.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// A whole Kaczmarz sweep in one launch: as gs_flow_kernel, one leaf per
// ticket (GsFlowArgs items of one leaf), its window read and written with
// agent-scope loads and stores.
__global__ void __launch_bounds__(kGsLanes) kacz_flow_kernel(GsArgs a, GsFlowArgs f, double omega,
                                                            const double* __restrict__ bvec, double* __restrict__ x) {
  extern __shared__ double xw[];
  const int32_t lane = static_cast<int32_t>(threadIdx.x);
  for (int32_t t = static_cast<int32_t>(blockIdx.x); t < f.n_tickets; t += static_cast<int32_t>(gridDim.x)) {
    wait_tickets(f, t, lane);
    const int32_t leaf = gs_uniform(f.item_leaf0, gs_uniform(f.ticket_item, t));
    if (gs_uniform(f.ticket_back, t))
      kacz_leaf<true, true>(a, leaf, omega, bvec, x, xw);
    else
      kacz_leaf<false, true>(a, leaf, omega, bvec, x, xw);
    // every lane's x stores complete before the flag
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __syncthreads();
    if (lane == 0) __hip_atomic_store(f.flags + t, f.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace dev

// LDS of a dataflow sweep's workgroup.
static size_t flow_lds(size_t bytes) { return std::max<size_t>(bytes, 1); }

// Workgroups per CU of a dataflow sweep.  The tickets are dealt round robin
// and every workgroup must be running (a ticket whose owner never starts
// stalls its dependents until the bounded waits give up).  On this device
// some launches at the count the occupancy query reports stalled, the cause
// not identified: Gauss-Seidel, N_t 16384 (11,232 B of LDS per workgroup):
// 14 per CU ran, 13 x 12,288 B stalled; Kaczmarz, N_t 8192 (6,656 B): 24 and
// 22 per CU (and 20 x 8,192 B) stalled, 12 and 13 ran, while N_t 4096
// (6,072 B) ran at 24.  The count is therefore capped at 144 KiB of LDS per
// CU, and the Kaczmarz query asks for its LDS rounded up to 2 KiB plus 4 KiB
// (13 per CU at 6,656 B), the settings every measured case ran with.
static hipError_t flow_per_cu(const void* fn, size_t lds, size_t query_lds, int* per_cu) {
  constexpr size_t kCuLdsUsable = 144 * 1024;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, fn, dev::kGsLanes, query_lds);
  if (e != hipSuccess) return e;
  const int cap = static_cast<int>(kCuLdsUsable / lds);
  if (*per_cu > cap) *per_cu = cap;
  return hipSuccess;
}

hipError_t kacz_flow_grid(int32_t wmax, int32_t n_cus, int32_t* grid) {
  const size_t lds = flow_lds(static_cast<size_t>(wmax > 0 ? wmax : 1) * sizeof(double));
  int per_cu = 0;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&dev::kacz_flow_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kGsMaxWindowBytes);
  if (e != hipSuccess) return e;
  e = flow_per_cu(reinterpret_cast<const void*>(&dev::kacz_flow_kernel), lds, (lds + 2047) / 2048 * 2048 + 4096,
                  &per_cu);
  if (e != hipSuccess) return e;
  *grid = per_cu * n_cus;
  return hipSuccess;
}

hipError_t launch_kacz_flow(const GsArgs& a, const GsFlowArgs& f, int32_t wmax, int32_t grid, double omega,
                            const double* b, double* x, hipStream_t st) {
  if (f.n_tickets == 0) return hipSuccess;
  const size_t lds = flow_lds(static_cast<size_t>(wmax > 0 ? wmax : 1) * sizeof(double));
  GsArgs aa = a;
  GsFlowArgs ff = f;
  double om = omega;
  void* args[] = {&aa, &ff, &om, const_cast<double**>(&b), &x};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&dev::kacz_flow_kernel),
                                    dim3(static_cast<uint32_t>(grid)), dim3(dev::kGsLanes), args,
                                    static_cast<unsigned int>(lds), st);
}

hipError_t gs_flow_grid(int32_t wmax, int32_t n_cus, int32_t* grid) {
  const size_t lds = flow_lds(4 * static_cast<size_t>(wmax > 0 ? wmax : 1) * sizeof(double));
  int per_cu = 0;
  hipError_t e = flow_per_cu(reinterpret_cast<const void*>(&dev::gs_flow_kernel), lds, lds, &per_cu);
  if (e != hipSuccess) return e;
  *grid = per_cu * n_cus;
  return hipSuccess;
}

hipError_t launch_gs_flow(const GsArgs& a, const GsFlowArgs& f, int32_t wmax, int32_t grid, const double* b, double* x,
                          hipStream_t st) {
  if (f.n_tickets == 0) return hipSuccess;
  const size_t lds = flow_lds(4 * static_cast<size_t>(wmax > 0 ? wmax : 1) * sizeof(double));
  GsArgs aa = a;
  GsFlowArgs ff = f;
  int32_t ww = wmax > 0 ? wmax : 1;
  void* args[] = {&aa, &ff, &ww, const_cast<double**>(&b), &x};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&dev::gs_flow_kernel), dim3(static_cast<uint32_t>(grid)),
                                    dim3(dev::kGsLanes), args, static_cast<unsigned int>(lds), st);
}

hipError_t launch_kacz_phase(const GsArgs& a, int32_t leaf0, int32_t count, int32_t wmax, bool backward, double omega,
                             int32_t quad_min_leaves, const double* b, double* x, hipStream_t st) {
  if (count == 0) return hipSuccess;
  if (wmax <= kGsQuadMaxWindow && count >= quad_min_leaves) {
    // four leaves per wavefront
    const size_t qlds = 4 * static_cast<size_t>(wmax > 0 ? wmax : 1) * sizeof(double);
    const dim3 grid(static_cast<uint32_t>((count + 3) / 4));
    if (backward)
      hipLaunchKernelGGL(dev::kacz_quad_kernel<true>, grid, dim3(dev::kGsLanes), qlds, st, a, leaf0, count,
                         wmax > 0 ? wmax : 1, omega, b, x);
    else
      hipLaunchKernelGGL(dev::kacz_quad_kernel<false>, grid, dim3(dev::kGsLanes), qlds, st, a, leaf0, count,
                         wmax > 0 ? wmax : 1, omega, b, x);
    return hipGetLastError();
  }
  static bool attr_done[2] = {false, false};
  const void* fn = backward ? reinterpret_cast<const void*>(&dev::kacz_leaf_kernel<true>)
                            : reinterpret_cast<const void*>(&dev::kacz_leaf_kernel<false>);
  if (!attr_done[backward]) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kGsMaxWindowBytes);
    if (e != hipSuccess) return e;
    attr_done[backward] = true;
  }
  const size_t lds = static_cast<size_t>(wmax > 0 ? wmax : 1) * sizeof(double);
  if (backward)
    hipLaunchKernelGGL(dev::kacz_leaf_kernel<true>, dim3(static_cast<uint32_t>(count)), dim3(dev::kGsLanes), lds, st,
                       a, leaf0, omega, b, x);
  else
    hipLaunchKernelGGL(dev::kacz_leaf_kernel<false>, dim3(static_cast<uint32_t>(count)), dim3(dev::kGsLanes), lds, st,
                       a, leaf0, omega, b, x);
  return hipGetLastError();
}

hipError_t launch_gs_phase(const GsArgs& a, int32_t leaf0, int32_t count, int32_t wmax, bool backward,
                           int32_t quad_min_leaves, const double* b, double* x, hipStream_t st) {
  if (count == 0) return hipSuccess;
  static bool attr_done[2] = {false, false};
  const void* fn = backward ? reinterpret_cast<const void*>(&dev::gs_leaf_kernel<true>)
                            : reinterpret_cast<const void*>(&dev::gs_leaf_kernel<false>);
  if (!attr_done[backward]) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kGsMaxWindowBytes);
    if (e != hipSuccess) return e;
    attr_done[backward] = true;
  }
  if (wmax <= kGsQuadMaxWindow && count >= quad_min_leaves) {
    // four leaves per wavefront
    const size_t qlds = 4 * static_cast<size_t>(wmax > 0 ? wmax : 1) * sizeof(double);
    const dim3 grid(static_cast<uint32_t>((count + 3) / 4));
    if (backward)
      hipLaunchKernelGGL(dev::gs_quad_kernel<true>, grid, dim3(dev::kGsLanes), qlds, st, a, leaf0, count,
                         wmax > 0 ? wmax : 1, b, x);
    else
      hipLaunchKernelGGL(dev::gs_quad_kernel<false>, grid, dim3(dev::kGsLanes), qlds, st, a, leaf0, count,
                         wmax > 0 ? wmax : 1, b, x);
    return hipGetLastError();
  }
  const size_t lds = static_cast<size_t>(wmax > 0 ? wmax : 1) * sizeof(double);
  if (backward)
    hipLaunchKernelGGL(dev::gs_leaf_kernel<true>, dim3(static_cast<uint32_t>(count)), dim3(dev::kGsLanes), lds, st, a,
                       leaf0, b, x);
  else
    hipLaunchKernelGGL(dev::gs_leaf_kernel<false>, dim3(static_cast<uint32_t>(count)), dim3(dev::kGsLanes), lds, st,
                       a, leaf0, b, x);
  return hipGetLastError();
}

}  // namespace race
