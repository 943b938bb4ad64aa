// gfx950 kernels: RACE SymmSpMV / SymmSpMM, the full-CRS SpMV and the
// global-atomic SymmSpMV baselines, and the permutation kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.hpp"
#include "unit_device.hpp"

namespace race {
namespace dev {

// Phase-by-phase execution: one launch per phase; one workgroup per leaf
// running the leaf's units in order, or (per_unit, when the units of a leaf
// combine shared indices atomically) one workgroup per unit.
template <typename ValT, int K>
__global__ void __launch_bounds__(1024) race_leaf_kernel(UnitArgs<ValT> a, int32_t base, int32_t per_unit,
                                                         const double* __restrict__ x, double* __restrict__ y,
                                                         int32_t ld, int32_t wmax, uint64_t* trace) {
  extern __shared__ double smem[];
  double* xw = smem;
  double* yw = smem + static_cast<size_t>(wmax) * K;
  uint32_t* gw = reinterpret_cast<uint32_t*>(smem + 2 * static_cast<size_t>(wmax) * K);
  const int32_t item = base + static_cast<int32_t>(blockIdx.x);
  const int32_t u0 = per_unit ? item : a.leaf_units[2 * item];
  const int32_t u1 = per_unit ? item + 1 : a.leaf_units[2 * item + 1];
  const int32_t tid = static_cast<int32_t>(threadIdx.x), nthr = static_cast<int32_t>(blockDim.x);
  for (int32_t u = u0; u < u1; ++u) {
    const uint64_t t0 = trace ? wall_clock() : 0;
    const UnitDesc ud = uniform_load(a.unit_desc, u);
    compute_unit<ValT, K>(a, ud, x, ld, xw, yw, gw, tid, nthr);
    const uint64_t t1 = trace ? wall_clock() : 0;
    flush_unit<K, false>(ud, y, ld, yw, gw, tid, nthr);
    __syncthreads();
    if (trace && tid == 0) {
      const uint64_t t2 = wall_clock();
      trace[4 * static_cast<size_t>(u) + 0] = t0;
      trace[4 * static_cast<size_t>(u) + 1] = t1;
      trace[4 * static_cast<size_t>(u) + 2] = t1;
      trace[4 * static_cast<size_t>(u) + 3] = t2;
    }
  }
}

// Dataflow execution in one persistent launch.  Tickets are the clearing
// tasks, then the units in ticket order (by default the execution order:
// phase, then heaviest leaf first, a leaf's units in row order; or any other
// topological order of the conflict edges).  Workgroup b starts on static ticket b,
// later tickets come from a counter once every static ticket is claimed.  A
// unit computes right away and, before its flush, waits until every earlier
// unit whose touch set meets its own has published completion (the conflict
// edges of the tree's coloring).  Only y crosses units, and it does so
// through coherent (agent-scope atomic) accesses whose completion each
// thread awaits before the publishing barrier; x and the matrix are
// read-only.
//
// Progress needs no co-residency: waits point only to smaller tickets; a
// counter ticket is handed out only after every static ticket has a running
// owner, and a static ticket whose own workgroup is not running is claimed
// by a running workgroup that waits for it (which sets its computed unit
// aside, runs that ticket and computes its unit again) or by a free one.
// So the lowest unfinished ticket is always owned by a running workgroup or
// claimable by one.  Every wait is bounded and reports through `status` if
// it gives up, so the grid always drains.
template <typename ValT, int K>
__global__ void __launch_bounds__(1024) race_flow_kernel(UnitArgs<ValT> a, FlowArgs f, const double* __restrict__ x,
                                                         double* __restrict__ y, int32_t ld, int32_t wmax,
                                                         uint32_t epoch, uint64_t ticket_base) {
  extern __shared__ double smem[];
  double* xw = smem;
  double* yw = smem + static_cast<size_t>(wmax) * K;
  uint32_t* gw = reinterpret_cast<uint32_t*>(smem + 2 * static_cast<size_t>(wmax) * K);
  __shared__ int32_t s_red[2];
  __shared__ int32_t s_aside[kSetAside];
  const int32_t tid = static_cast<int32_t>(threadIdx.x), nthr = static_cast<int32_t>(blockDim.x);
  const int32_t bid = static_cast<int32_t>(blockIdx.x);
  // wave 0 as a scalar condition: the lane-0 work below sits in small
  // diamonds inside a wave-uniform branch, and barriers close them on both
  // sides, so no lane can run ahead into the next unit's barriers
  const bool wave0 = __builtin_amdgcn_readfirstlane(tid) < kSlice;
  const bool late = f.late_stride > 0 && bid % f.late_stride == f.late_stride - 1;
  if (late) {
    // tests only: join about 0.2 ms late without claiming the own ticket
    for (int i = 0; i < 64; ++i) __builtin_amdgcn_s_sleep(127);
  }
  if (wave0) {
    if (tid == 0) {
      s_red[0] = INT32_MAX;
      s_red[1] = (!late && bid < f.n_static && claim_ticket(f.claim, bid, epoch)) ? bid : -1;
    }
  }
  __syncthreads();
  // tickets and counts live in scalar registers, so the loop's exits and
  // the barriers inside stay in uniform control flow
  int32_t t = __builtin_amdgcn_readfirstlane(s_red[1]);
  int32_t aside = 0;
  bool all_claimed = false;
  for (;;) {
    if (t < 0) {
      if (aside > 0) {
        --aside;
        t = __builtin_amdgcn_readfirstlane(s_aside[aside]);
      } else {
        t = next_ticket(f, epoch, ticket_base, all_claimed, s_red, bid, tid, nthr, wave0);
        if (t < 0) break;
      }
    }
    if (t < f.n_zero_tasks) {
      const int64_t i0 = static_cast<int64_t>(t) * f.zero_chunk;
      clear_task<K>(f.zero_idx, i0, i0 + f.zero_chunk < f.n_zero ? i0 + f.zero_chunk : f.n_zero, y, ld,
                    f.done + f.n_units + t, epoch, tid, nthr, wave0);
      t = -1;
      continue;
    }
    const int32_t u = uniform_load(f.ticket_unit, t - f.n_zero_tasks);
    const uint64_t t0 = f.trace ? wall_clock() : 0;
    // the unit's arithmetic needs nothing from other units; only its flush
    // must follow the earlier units it conflicts with
    const UnitDesc ud = uniform_load(a.unit_desc, u);
    compute_unit<ValT, K>(a, ud, x, ld, xw, yw, gw, tid, nthr);
    const uint64_t t1 = f.trace ? wall_clock() : 0;
    const int32_t r = wait_edges(f, ud.d0, ud.d1, epoch, aside < kSetAside, s_red, tid, nthr, wave0);
    if (r >= 0) {
      // run the ownerless ticket first; this unit is computed again later
      if (wave0) {
        if (tid == 0) {
          s_aside[aside] = t;
          atomicAdd(f.takeovers, 1u);
        }
      }
      ++aside;
      t = r;
      continue;
    }
    const uint64_t t2 = f.trace ? wall_clock() : 0;
    flush_unit<K, true>(ud, y, ld, yw, gw, tid, nthr);
    // every thread's coherent y stores complete before the barrier, so the
    // completion flag written after it is only seen once they are visible
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __syncthreads();
    if (wave0) {
      if (tid == 0) {
        if (f.trace) {
          const uint64_t t3 = wall_clock();
          f.trace[4 * static_cast<size_t>(u) + 0] = t0;
          f.trace[4 * static_cast<size_t>(u) + 1] = t1;
          f.trace[4 * static_cast<size_t>(u) + 2] = t2;
          f.trace[4 * static_cast<size_t>(u) + 3] = t3;
        }
        __hip_atomic_store(f.done + u, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    t = -1;
  }
}

// Clears a batch's dataflow state (done flags, status, ticket counter) with
// plain stores, so a captured graph can replay the run.
__global__ void __launch_bounds__(256) batch_reset_kernel(uint32_t* state, int64_t words) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < words; i += stride) state[i] = 0u;
}

__global__ void __launch_bounds__(256) zero_entries_kernel(double* __restrict__ y, int32_t ld, int32_t k,
                                                           const int32_t* __restrict__ idx, int64_t count) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count * k; i += stride)
    y[static_cast<size_t>(idx[i / k]) * ld + i % k] = 0.0;
}

// Many matrices in one persistent launch: tickets are (matrix, unit) pairs
// merged in phase order with every matrix's own order kept, so the same
// argument as in race_flow_kernel makes it deadlock-free.
template <typename ValT, int K>
__global__ void __launch_bounds__(1024) race_batch_kernel(const BatchMat<ValT>* __restrict__ mats, BatchArgs b,
                                                          int32_t wmax) {
  extern __shared__ double smem[];
  double* xw = smem;
  double* yw = smem + static_cast<size_t>(wmax) * K;
  uint32_t* gw = reinterpret_cast<uint32_t*>(smem + 2 * static_cast<size_t>(wmax) * K);
  __shared__ int32_t s_ticket[1];
  const int32_t tid = static_cast<int32_t>(threadIdx.x), nthr = static_cast<int32_t>(blockDim.x);
  const bool wave0 = __builtin_amdgcn_readfirstlane(tid) < kSlice;
  uint64_t* counter = reinterpret_cast<uint64_t*>(b.state + b.state_words - 2);
  uint32_t* status = b.state + b.state_words - 4;
  for (;;) {
    __syncthreads();
    if (wave0) {
      if (tid == 0) {
        const uint64_t t = atomicAdd(reinterpret_cast<unsigned long long*>(counter), 1ull);
        s_ticket[0] = t < static_cast<uint64_t>(b.n_tickets) ? static_cast<int32_t>(t) : -1;
      }
    }
    __syncthreads();
    const int32_t t = __builtin_amdgcn_readfirstlane(s_ticket[0]);
    if (t < 0) break;
    const int32_t m = uniform_load(b.ticket_mat, t);
    const int32_t lt = uniform_load(b.ticket_unit, t);
    const BatchMat<ValT> mm = mats[m];
    if (lt < mm.n_zero_tasks) {
      const int64_t i0 = static_cast<int64_t>(lt) * mm.zero_chunk;
      double* yp = b.tiled ? mm.yt + static_cast<size_t>(mm.n) * b.col0 : mm.y + b.col0;
      clear_task<K>(mm.zero_idx, i0, i0 + mm.zero_chunk < mm.n_zero ? i0 + mm.zero_chunk : mm.n_zero, yp, b.ld,
                    mm.done + mm.n_units + lt, 1u, tid, nthr, wave0);
      continue;
    }
    const double* xp = b.tiled ? mm.xt + static_cast<size_t>(mm.n) * b.col0 : mm.x + b.col0;
    double* yp = b.tiled ? mm.yt + static_cast<size_t>(mm.n) * b.col0 : mm.y + b.col0;
    flow_unit<ValT, K>(mm.a, lt - mm.n_zero_tasks, mm.dep_idx, mm.done, status, nullptr, 1u, xp, yp, b.ld,
                       xw, yw, gw, tid, nthr, wave0);
  }
}

// Full-matrix CRS SpMV (Algorithm "SpMV"), LPR lanes per row; values
// float64 or float32 (promoted, float64 arithmetic).
template <int LPR, typename ValT>
__global__ void __launch_bounds__(256) csr_spmv_kernel(int32_t n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col, const ValT* __restrict__ val,
                                                       const double* __restrict__ x, double* __restrict__ y) {
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t row = gid / LPR;
  const int32_t l = static_cast<int32_t>(gid % LPR);
  if (row >= n) return;  // whole lane groups leave together
  double s = 0.0;
  const int32_t e = rp[row + 1];
  // plain loads: a lane group takes a row's entries a part of a cache line
  // at a time, so a line that is not kept would be fetched again
  for (int32_t i = rp[row] + l; i < e; i += LPR) s += static_cast<double>(val[i]) * x[col[i]];
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) s += __shfl_down(s, o, LPR);
  if (l == 0) y[row] = s;
}

// Full-matrix CRS SpMV over row blocks (Algorithm "SpMV" with the entries
// of consecutive rows streamed together).  Block b covers rows
// [blk[b], blk[b+1]); their entries, at most 256 * PER, are consecutive in
// the CRS arrays, so thread t loads entries t, t + 256, ... with unit
// stride across the workgroup (every load instruction takes whole cache
// lines, read non-temporally), multiplies each by its x entry and keeps the
// product in LDS; after a barrier one thread per row adds its row's
// products in entry order.  A block of a single row longer than 256 * PER
// strides over the row and reduces across the workgroup instead.  Loads of
// the lanes past the block's last entry repeat that entry (no per-lane
// branch around the loads) and their products are dropped.  Workgroups are
// dealt to the 8 XCDs in turn, so workgroup g runs block (g % 8) * G8 + g / 8
// (G8 = grid / 8, the grid padded to a multiple of 8): each XCD streams a
// contiguous eighth of the rows, and the x entries its rows gather stay in
// its own L2 instead of being fetched by all eight.
// One row block (rows r0..r1 of one matrix) of the row-block product, run
// by a 256-thread workgroup with `prod` its LDS array of 256 * PER doubles.
template <typename ValT, int PER>
__device__ __forceinline__ void csr_block_rows(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                               const ValT* __restrict__ val, const double* __restrict__ x,
                                               double* __restrict__ y, int32_t r0, int32_t r1, double* prod) {
  constexpr int32_t kCap = 256 * PER;
  const int32_t t = static_cast<int32_t>(threadIdx.x);
  const int32_t e0 = uniform_load(rp, r0);
  const int32_t ne = uniform_load(rp, r1) - e0;
  if (ne > kCap) {
    // one long row (the partition gives such a row a block of its own)
    double s = 0.0;
    for (int32_t i = e0 + t; i < e0 + ne; i += 256) s += static_cast<double>(val[i]) * x[col[i]];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((t & 63) == 0) prod[t >> 6] = s;
    __syncthreads();
    if (t == 0) y[r0] = (prod[0] + prod[1]) + (prod[2] + prod[3]);
    return;
  }
  if (ne > 0) {
    int32_t c[PER];
    ValT v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int32_t i = e0 + min(t + k * 256, ne - 1);
      c[k] = stream_load(col + i);
      v[k] = stream_load(val + i);
    }
    double xv[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) xv[k] = x[c[k]];
#pragma unroll
    for (int k = 0; k < PER; ++k)
      if (t + k * 256 < ne) prod[t + k * 256] = static_cast<double>(v[k]) * xv[k];
  }
  __syncthreads();
  for (int32_t r = r0 + t; r < r1; r += 256) {
    const int32_t a = rp[r] - e0, b = rp[r + 1] - e0;
    double s = 0.0;
    for (int32_t j = a; j < b; ++j) s += prod[j];
    y[r] = s;
  }
}

// Workgroup g of a grid padded to a multiple of 8 runs block
// (g % 8) * (grid / 8) + g / 8 (see above).
__device__ __forceinline__ int32_t xcd_block() {
  const uint32_t g8 = gridDim.x / 8u;
  return static_cast<int32_t>((blockIdx.x % 8u) * g8 + blockIdx.x / 8u);
}

template <typename ValT, int PER>
__global__ void __launch_bounds__(256) csr_block_kernel(const int32_t* __restrict__ blk,
                                                        const int32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ col,
                                                        const ValT* __restrict__ val,
                                                        const double* __restrict__ x, double* __restrict__ y,
                                                        int32_t n_blocks) {
  __shared__ double prod[256 * PER];
  const int32_t b = xcd_block();
  if (b >= n_blocks) return;  // padding of the grid (uniform per workgroup)
  csr_block_rows<ValT, PER>(rp, col, val, x, y, uniform_load(blk, b), uniform_load(blk, b + 1), prod);
}

// The row-block product of several matrices in one launch (the members of a
// batch that run it): global block g belongs to matrix blk_mat[g] and is
// block g - base of that matrix.
template <typename ValT, int PER>
__global__ void __launch_bounds__(256) csr_block_batch_kernel(const BlockMat<ValT>* __restrict__ mats,
                                                              const int32_t* __restrict__ blk_mat,
                                                              int32_t n_blocks) {
  __shared__ double prod[256 * PER];
  const int32_t g = xcd_block();
  if (g >= n_blocks) return;
  const BlockMat<ValT> m = mats[uniform_load(blk_mat, g)];
  const int32_t b = g - m.base;
  csr_block_rows<ValT, PER>(m.rp, m.col, m.val, m.x, m.y, uniform_load(m.blk, b), uniform_load(m.blk, b + 1), prod);
}

// Full-matrix CRS SpMM over row blocks for k = 2..KB columns (KB = 2 or 4;
// X, Y row-major n x k): blocks of at most 512 entries (two per thread),
// each entry's k products kept in LDS (entry-major, KB per entry), then one
// thread per (row, column) adds its row's products in entry order.  Column
// indices past k are computed on column k - 1 and never stored.  A block
// of one row longer than 512 entries strides over it and reduces across
// the workgroup per column.  Blocks go to the XCDs in contiguous eighths.
template <typename ValT, int KB>
__global__ void __launch_bounds__(256) csr_block_spmm_kernel(const int32_t* __restrict__ blk,
                                                             const int32_t* __restrict__ rp,
                                                             const int32_t* __restrict__ col,
                                                             const ValT* __restrict__ val,
                                                             const double* __restrict__ X, double* __restrict__ Y,
                                                             int32_t k, int32_t n_blocks) {
  constexpr int32_t kPer = 2, kCap = 256 * kPer;
  __shared__ double prod[kCap * KB];
  const int32_t t = static_cast<int32_t>(threadIdx.x);
  const int32_t b = xcd_block();
  if (b >= n_blocks) return;  // padding of the grid (uniform per workgroup)
  const int32_t r0 = uniform_load(blk, b), r1 = uniform_load(blk, b + 1);
  const int32_t e0 = uniform_load(rp, r0);
  const int32_t ne = uniform_load(rp, r1) - e0;
  if (ne > kCap) {
    double s[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) s[j] = 0.0;
    for (int32_t i = e0 + t; i < e0 + ne; i += 256) {
      const double a = static_cast<double>(val[i]);
      const int64_t c = static_cast<int64_t>(col[i]) * k;
#pragma unroll
      for (int j = 0; j < KB; ++j) s[j] += a * X[c + (j < k ? j : k - 1)];
    }
#pragma unroll
    for (int j = 0; j < KB; ++j)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s[j] += __shfl_xor(s[j], o, 64);
    if ((t & 63) == 0)
#pragma unroll
      for (int j = 0; j < KB; ++j) prod[(t >> 6) * KB + j] = s[j];
    __syncthreads();
    if (t < k) Y[static_cast<int64_t>(r0) * k + t] = (prod[t] + prod[KB + t]) + (prod[2 * KB + t] + prod[3 * KB + t]);
    return;
  }
  if (ne > 0) {
    int32_t c[kPer];
    ValT v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int32_t i = e0 + min(t + u * 256, ne - 1);
      c[u] = stream_load(col + i);
      v[u] = stream_load(val + i);
    }
    double xv[kPer][KB];
#pragma unroll
    for (int u = 0; u < kPer; ++u)
#pragma unroll
      for (int j = 0; j < KB; ++j) xv[u][j] = X[static_cast<int64_t>(c[u]) * k + (j < k ? j : k - 1)];
#pragma unroll
    for (int u = 0; u < kPer; ++u)
      if (t + u * 256 < ne)
#pragma unroll
        for (int j = 0; j < KB; ++j) prod[(t + u * 256) * KB + j] = static_cast<double>(v[u]) * xv[u][j];
  }
  __syncthreads();
  const int32_t pairs = (r1 - r0) * KB;
  for (int32_t p = t; p < pairs; p += 256) {
    const int32_t r = r0 + p / KB, j = p % KB;
    if (j >= k) continue;
    const int32_t a = rp[r] - e0, e = rp[r + 1] - e0;
    double s = 0.0;
    for (int32_t q = a; q < e; ++q) s += prod[q * KB + j];
    Y[static_cast<int64_t>(r) * k + j] = s;
  }
}

// Full-matrix CRS SpMM Y = A X (Algorithm "SpMV" for k columns; X, Y
// row-major n x k, 2 <= k <= KC): a group of KC lanes per row, lane j owns
// column j.  The group steps through its row four entries at a time; every
// lane loads the same value and column (one address per group) and its own
// X entry, so the k entries of an X row arrive as one contiguous segment.
// Lanes j >= k compute on column k - 1 and store nothing.
template <typename ValT, int KC>
__global__ void __launch_bounds__(256) csr_spmm_kernel(int32_t n, int32_t k, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col,
                                                       const ValT* __restrict__ val,
                                                       const double* __restrict__ X, double* __restrict__ Y) {
  constexpr int kU = 4;
  const int64_t gid = static_cast<int64_t>(xcd_block()) * blockDim.x + threadIdx.x;
  const int64_t row = gid / KC;
  const int32_t j = static_cast<int32_t>(gid % KC);
  if (row >= n) return;  // whole lane groups leave together
  const int32_t jj = j < k ? j : k - 1;
  const int32_t b = rp[row], e = rp[row + 1];
  double s = 0.0;
  for (int32_t i = b; i < e; i += kU) {
    int32_t c[kU];
    ValT v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int32_t ii = i + u < e ? i + u : e - 1;
      c[u] = col[ii];
      v[u] = val[ii];
    }
    double xv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) xv[u] = X[static_cast<int64_t>(c[u]) * k + jj];
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (i + u < e) s += static_cast<double>(v[u]) * xv[u];
  }
  if (j < k) Y[row * k + j] = s;
}

// SymmSpMV with device-wide float64 atomics for every update of y.
template <int LPR>
__global__ void __launch_bounds__(256) atomic_symm_kernel(int32_t n, const int32_t* __restrict__ rp,
                                                          const int32_t* __restrict__ col,
                                                          const double* __restrict__ val,
                                                          const double* __restrict__ x, double* y) {
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t row = gid / LPR;
  const int32_t l = static_cast<int32_t>(gid % LPR);
  if (row >= n) return;
  const double xr = x[row];
  double s = 0.0;
  const int32_t e = rp[row + 1];
  for (int32_t i = rp[row] + l; i < e; i += LPR) {
    const int32_t c = col[i];
    const double v = val[i];
    s += v * x[c];
    if (c != row) unsafeAtomicAdd(&y[c], v * xr);
  }
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) s += __shfl_down(s, o, LPR);
  if (l == 0) unsafeAtomicAdd(&y[row], s);
}

__global__ void __launch_bounds__(256) fill_zero_kernel(double* __restrict__ y, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = 0.0;
}

// Row-major n x k <-> column tiles: tile t holds columns [t kt, t kt + kc)
// as a contiguous row-major n x kc block at offset n kt t (kc = kt but for
// a narrower last tile).  to_tiles: tiles[...] = full[...]; else back.
__global__ void __launch_bounds__(256) tile_kernel(int32_t n, int32_t k, int32_t kt, double* __restrict__ full,
                                                   double* __restrict__ tiles, int32_t to_tiles) {
  const int64_t total = static_cast<int64_t>(n) * k;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e / k;
    const int32_t c = static_cast<int32_t>(e % k);
    const int32_t t = c / kt, c0 = t * kt;
    const int32_t kc = k - c0 < kt ? k - c0 : kt;
    const int64_t at = static_cast<int64_t>(n) * kt * t + i * kc + (c - c0);
    if (to_tiles) tiles[at] = full[e];
    else full[e] = tiles[at];
  }
}

// tile_kernel for every matrix of a batch: blockIdx.y selects the matrix.
template <typename ValT>
__global__ void __launch_bounds__(256) batch_tile_kernel(const BatchMat<ValT>* __restrict__ mats, int32_t k, int32_t kt,
                                                         int32_t to_tiles) {
  const BatchMat<ValT>& mm = mats[blockIdx.y];
  const int64_t total = static_cast<int64_t>(mm.n) * k;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e / k;
    const int32_t c = static_cast<int32_t>(e % k);
    const int32_t t = c / kt, c0 = t * kt;
    const int32_t kc = k - c0 < kt ? k - c0 : kt;
    const int64_t at = static_cast<int64_t>(mm.n) * kt * t + i * kc + (c - c0);
    if (to_tiles) mm.xt[at] = mm.x[e];
    else mm.y[e] = mm.yt[at];
  }
}

__global__ void __launch_bounds__(256) permute_kernel(int32_t n, int32_t k, const int32_t* __restrict__ new2old,
                                                      const double* __restrict__ in, double* __restrict__ out,
                                                      int32_t to_permuted) {
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= static_cast<int64_t>(n) * k) return;
  const int64_t i = gid / k;
  const int32_t j = static_cast<int32_t>(gid % k);
  const int64_t o = new2old[i];
  if (to_permuted) out[i * k + j] = in[o * k + j];
  else out[o * k + j] = in[i * k + j];
}

}  // namespace dev

// ---------------------------------------------------------------------------
// launchers

template <typename ValT, int K>
static hipError_t set_lds_attr(const void* fn) {
  static bool done = false;
  if (done) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 159 * 1024);
  if (e == hipSuccess) done = true;
  return e;
}

template <typename ValT, int K>
static hipError_t launch_leaf(const UnitArgs<ValT>& a, int32_t base, int32_t count, int32_t per_unit, const double* x,
                              double* y, int32_t ld, int32_t wmax, int32_t threads, uint64_t* trace, hipStream_t st) {
  const size_t lds = window_lds_bytes(wmax, K);
  hipError_t e = set_lds_attr<ValT, K>(reinterpret_cast<const void*>(&dev::race_leaf_kernel<ValT, K>));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((dev::race_leaf_kernel<ValT, K>), dim3(count), dim3(threads), lds, st, a, base, per_unit, x, y,
                     ld, wmax, trace);
  return hipGetLastError();
}

// Grid of a grid-stride fill over `items` elements: enough workgroups to
// cover them once, at most 4096.
static dim3 fill_grid(int64_t items) {
  return dim3(static_cast<uint32_t>(std::max<int64_t>(1, std::min<int64_t>(4096, (items + 255) / 256))));
}

hipError_t launch_zero_entries(double* y, int32_t ld, int32_t k, const int32_t* idx, int64_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::zero_entries_kernel, fill_grid(count * k), dim3(256), 0, st, y, ld, k, idx, count);
  return hipGetLastError();
}

template <typename ValT, int K>
struct FlowTag {};

template <typename ValT, int K>
static hipError_t launch_flow(const UnitArgs<ValT>& a, const FlowArgs& f, const double* x, double* y, int32_t ld,
                              int32_t wmax, int32_t threads, int32_t grid, uint32_t epoch, uint64_t ticket_base,
                              hipStream_t st) {
  const size_t lds = window_lds_bytes(wmax, K);
  hipError_t e = set_lds_attr<FlowTag<ValT, K>, K>(reinterpret_cast<const void*>(&dev::race_flow_kernel<ValT, K>));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((dev::race_flow_kernel<ValT, K>), dim3(grid), dim3(threads), lds, st, a, f, x, y, ld, wmax,
                     epoch, ticket_base);
  return hipGetLastError();
}

// Workgroups of the dataflow kernel one CU holds at once, from the kernel's
// registers and static LDS, the dynamic windows, 160 KB of LDS and 32
// wavefronts per CU (512 VGPRs per SIMD lane, allocated in blocks of 8).
// Only the launch size depends on it: the dataflow scheme itself needs no
// co-residency.
template <typename ValT, int K>
static hipError_t flow_occupancy(int32_t threads, int32_t wmax, int32_t* blocks_per_cu) {
  const size_t lds = window_lds_bytes(wmax, K);
  hipFuncAttributes attr{};
  hipError_t e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(&dev::race_flow_kernel<ValT, K>));
  int32_t regs = 128, static_lds = 64;
  if (e == hipSuccess) {
    regs = std::max(attr.numRegs, 1);
    static_lds = static_cast<int32_t>(attr.sharedSizeBytes);
  } else {
    (void)hipGetLastError();
  }
  const int32_t waves_per_block = std::max(1, threads / 64);
  const int32_t regs_rounded = (regs + 7) / 8 * 8;
  const int32_t waves_per_simd = std::max(1, std::min(8, 512 / regs_rounded));
  const int32_t by_waves = (4 * waves_per_simd) / waves_per_block;
  const int32_t by_lds = static_cast<int32_t>((160 * 1024) / (lds + static_cast<size_t>(static_lds) + 1));
  *blocks_per_cu = std::max(0, std::min(by_waves, by_lds));
  return hipSuccess;
}

#define RACE_K_SWITCH(CALL)                                                                              \
  switch (k) {                                                                                           \
    case 1: return CALL(1);   case 2: return CALL(2);   case 3: return CALL(3);   case 4: return CALL(4); \
    case 5: return CALL(5);   case 6: return CALL(6);   case 7: return CALL(7);   case 8: return CALL(8); \
    case 9: return CALL(9);   case 10: return CALL(10); case 11: return CALL(11); case 12: return CALL(12); \
    case 13: return CALL(13); case 14: return CALL(14); case 15: return CALL(15); case 16: return CALL(16); \
    default: return hipErrorInvalidValue;                                                                \
  }

template <typename ValT>
hipError_t launch_race_phase(const UnitArgs<ValT>& a, int32_t base, int32_t count, int32_t per_unit, int32_t k,
                             const double* x, double* y, int32_t ld, int32_t wmax, int32_t threads, uint64_t* trace,
                             hipStream_t st) {
#define CALL(KK) launch_leaf<ValT, KK>(a, base, count, per_unit, x, y, ld, wmax, threads, trace, st)
  RACE_K_SWITCH(CALL)
#undef CALL
}

template <typename ValT>
hipError_t launch_race_flow(const UnitArgs<ValT>& a, const FlowArgs& f, int32_t k, const double* x, double* y,
                            int32_t ld, int32_t wmax, int32_t threads, int32_t grid, uint32_t epoch,
                            uint64_t ticket_base, hipStream_t st) {
#define CALL(KK) launch_flow<ValT, KK>(a, f, x, y, ld, wmax, threads, grid, epoch, ticket_base, st)
  RACE_K_SWITCH(CALL)
#undef CALL
}

template <typename ValT>
hipError_t race_flow_occupancy(int32_t k, int32_t threads, int32_t wmax, int32_t* blocks_per_cu) {
#define CALL(KK) flow_occupancy<ValT, KK>(threads, wmax, blocks_per_cu)
  RACE_K_SWITCH(CALL)
#undef CALL
}

template hipError_t launch_race_phase<double>(const UnitArgs<double>&, int32_t, int32_t, int32_t, int32_t,
                                              const double*, double*, int32_t, int32_t, int32_t, uint64_t*,
                                              hipStream_t);
template hipError_t launch_race_phase<float>(const UnitArgs<float>&, int32_t, int32_t, int32_t, int32_t, const double*,
                                             double*, int32_t, int32_t, int32_t, uint64_t*, hipStream_t);
template hipError_t launch_race_flow<double>(const UnitArgs<double>&, const FlowArgs&, int32_t, const double*, double*,
                                             int32_t, int32_t, int32_t, int32_t, uint32_t, uint64_t, hipStream_t);
template hipError_t launch_race_flow<float>(const UnitArgs<float>&, const FlowArgs&, int32_t, const double*, double*,
                                            int32_t, int32_t, int32_t, int32_t, uint32_t, uint64_t, hipStream_t);
template hipError_t race_flow_occupancy<double>(int32_t, int32_t, int32_t, int32_t*);
template hipError_t race_flow_occupancy<float>(int32_t, int32_t, int32_t, int32_t*);

// Complex values: one instantiation, the two columns being the real and
// imaginary part of x and y.
template <>
hipError_t launch_race_flow<Cplx<false>>(const UnitArgs<Cplx<false>>& a, const FlowArgs& f, int32_t k,
                                         const double* x, double* y, int32_t ld, int32_t wmax, int32_t threads,
                                         int32_t grid, uint32_t epoch, uint64_t ticket_base, hipStream_t st) {
  if (k != 2) return hipErrorInvalidValue;
  return launch_flow<Cplx<false>, 2>(a, f, x, y, ld, wmax, threads, grid, epoch, ticket_base, st);
}
template <>
hipError_t launch_race_flow<Cplx<true>>(const UnitArgs<Cplx<true>>& a, const FlowArgs& f, int32_t k,
                                        const double* x, double* y, int32_t ld, int32_t wmax, int32_t threads,
                                        int32_t grid, uint32_t epoch, uint64_t ticket_base, hipStream_t st) {
  if (k != 2) return hipErrorInvalidValue;
  return launch_flow<Cplx<true>, 2>(a, f, x, y, ld, wmax, threads, grid, epoch, ticket_base, st);
}
template <>
hipError_t race_flow_occupancy<Cplx<false>>(int32_t k, int32_t threads, int32_t wmax, int32_t* blocks_per_cu) {
  if (k != 2) return hipErrorInvalidValue;
  return flow_occupancy<Cplx<false>, 2>(threads, wmax, blocks_per_cu);
}
template <>
hipError_t race_flow_occupancy<Cplx<true>>(int32_t k, int32_t threads, int32_t wmax, int32_t* blocks_per_cu) {
  if (k != 2) return hipErrorInvalidValue;
  return flow_occupancy<Cplx<true>, 2>(threads, wmax, blocks_per_cu);
}

template <typename ValT, int K>
struct BatchTag {};

template <typename ValT, int K>
static hipError_t launch_batch_k(const BatchMat<ValT>* mats, const BatchArgs& b, int32_t wmax, int32_t threads,
                                 int32_t grid, hipStream_t st) {
  const size_t lds = window_lds_bytes(wmax, K);
  hipError_t e = set_lds_attr<BatchTag<ValT, K>, K>(reinterpret_cast<const void*>(&dev::race_batch_kernel<ValT, K>));
  if (e != hipSuccess) return e;
  const int64_t words = b.state_words;
  hipLaunchKernelGGL(dev::batch_reset_kernel, fill_grid(words), dim3(256), 0, st, b.state, words);
  hipLaunchKernelGGL((dev::race_batch_kernel<ValT, K>), dim3(grid), dim3(threads), lds, st, mats, b, wmax);
  return hipGetLastError();
}

template <typename ValT>
hipError_t launch_race_batch(const BatchMat<ValT>* mats, const BatchArgs& b, int32_t k, int32_t wmax, int32_t threads,
                             int32_t grid, hipStream_t st) {
#define CALL(KK) launch_batch_k<ValT, KK>(mats, b, wmax, threads, grid, st)
  RACE_K_SWITCH(CALL)
#undef CALL
}

template <typename ValT>
hipError_t prepare_race_batch(int32_t k) {
#define CALL(KK) set_lds_attr<BatchTag<ValT, KK>, KK>(reinterpret_cast<const void*>(&dev::race_batch_kernel<ValT, KK>))
  RACE_K_SWITCH(CALL)
#undef CALL
}

template <typename ValT>
hipError_t launch_batch_tile(const BatchMat<ValT>* mats, int32_t count, int32_t k, int32_t kt, int32_t to_tiles,
                             hipStream_t st) {
  hipLaunchKernelGGL(dev::batch_tile_kernel<ValT>, dim3(256, static_cast<uint32_t>(count)), dim3(256), 0, st, mats, k,
                     kt, to_tiles);
  return hipGetLastError();
}

template hipError_t launch_batch_tile<double>(const BatchMat<double>*, int32_t, int32_t, int32_t, int32_t,
                                              hipStream_t);
template hipError_t launch_batch_tile<float>(const BatchMat<float>*, int32_t, int32_t, int32_t, int32_t, hipStream_t);
template hipError_t prepare_race_batch<double>(int32_t);
template hipError_t prepare_race_batch<float>(int32_t);
template hipError_t launch_race_batch<double>(const BatchMat<double>*, const BatchArgs&, int32_t, int32_t, int32_t,
                                              int32_t, hipStream_t);
template hipError_t launch_race_batch<float>(const BatchMat<float>*, const BatchArgs&, int32_t, int32_t, int32_t,
                                             int32_t, hipStream_t);

hipError_t launch_clear_words(uint32_t* p, int64_t words, hipStream_t st) {
  if (words == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::batch_reset_kernel, fill_grid(words), dim3(256), 0, st, p, words);
  return hipGetLastError();
}

template <typename ValT>
hipError_t launch_csr_spmv(int32_t n, const int32_t* rp, const int32_t* col, const ValT* val, const double* x,
                           double* y, int32_t lpr, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t threads = static_cast<int64_t>(n) * lpr;
  const dim3 grid(static_cast<uint32_t>((threads + 255) / 256));
  switch (lpr) {
#define CSR_L(L)                                                                                         \
  case L:                                                                                                \
    hipLaunchKernelGGL((dev::csr_spmv_kernel<L, ValT>), grid, dim3(256), 0, st, n, rp, col, val, x, y); \
    break;
    CSR_L(1) CSR_L(2) CSR_L(4) CSR_L(8) CSR_L(16) CSR_L(32) CSR_L(64)
#undef CSR_L
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_csr_spmv<double>(int32_t, const int32_t*, const int32_t*, const double*, const double*,
                                            double*, int32_t, hipStream_t);
template hipError_t launch_csr_spmv<float>(int32_t, const int32_t*, const int32_t*, const float*, const double*,
                                           double*, int32_t, hipStream_t);

template <typename ValT>
hipError_t launch_csr_block(int32_t n_blocks, const int32_t* blk, const int32_t* rp, const int32_t* col,
                            const ValT* val, const double* x, double* y, int32_t per, hipStream_t st) {
  if (n_blocks == 0) return hipSuccess;
  const dim3 grid(static_cast<uint32_t>((static_cast<int64_t>(n_blocks) + 7) / 8 * 8));
  switch (per) {
#define CSR_B(P)                                                                                         \
  case P:                                                                                                \
    hipLaunchKernelGGL((dev::csr_block_kernel<ValT, P>), grid, dim3(256), 0, st, blk, rp, col, val, x, y, n_blocks); \
    break;
    CSR_B(4) CSR_B(8) CSR_B(16)
#undef CSR_B
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_csr_block<double>(int32_t, const int32_t*, const int32_t*, const int32_t*, const double*,
                                             const double*, double*, int32_t, hipStream_t);
template hipError_t launch_csr_block<float>(int32_t, const int32_t*, const int32_t*, const int32_t*, const float*,
                                            const double*, double*, int32_t, hipStream_t);

template <typename ValT>
hipError_t launch_csr_block_batch(const BlockMat<ValT>* mats, const int32_t* blk_mat, int32_t n_blocks,
                                  hipStream_t st) {
  if (n_blocks == 0) return hipSuccess;
  const dim3 grid(static_cast<uint32_t>((static_cast<int64_t>(n_blocks) + 7) / 8 * 8));
  hipLaunchKernelGGL((dev::csr_block_batch_kernel<ValT, kExpandedPerThread>), grid, dim3(256), 0, st, mats, blk_mat,
                     n_blocks);
  return hipGetLastError();
}

template hipError_t launch_csr_block_batch<double>(const BlockMat<double>*, const int32_t*, int32_t, hipStream_t);
template hipError_t launch_csr_block_batch<float>(const BlockMat<float>*, const int32_t*, int32_t, hipStream_t);

template <typename ValT>
hipError_t launch_csr_spmm(int32_t n, int32_t k, const int32_t* rp, const int32_t* col, const ValT* val,
                           const double* X, double* Y, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (k < 2 || k > 16) return hipErrorInvalidValue;
  const int32_t kc = k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : 16;
  const int64_t blocks = (static_cast<int64_t>(n) * kc + 255) / 256;
  const dim3 grid(static_cast<uint32_t>((blocks + 7) / 8 * 8));
  switch (kc) {
#define CSR_M(C)                                                                                           \
  case C:                                                                                                  \
    hipLaunchKernelGGL((dev::csr_spmm_kernel<ValT, C>), grid, dim3(256), 0, st, n, k, rp, col, val, X, Y); \
    break;
    CSR_M(2) CSR_M(4) CSR_M(8) CSR_M(16)
#undef CSR_M
  }
  return hipGetLastError();
}

template hipError_t launch_csr_spmm<double>(int32_t, int32_t, const int32_t*, const int32_t*, const double*,
                                            const double*, double*, hipStream_t);
template hipError_t launch_csr_spmm<float>(int32_t, int32_t, const int32_t*, const int32_t*, const float*,
                                           const double*, double*, hipStream_t);

template <typename ValT>
hipError_t launch_csr_block_spmm(int32_t n_blocks, const int32_t* blk, const int32_t* rp, const int32_t* col,
                                 const ValT* val, const double* X, double* Y, int32_t k, hipStream_t st) {
  if (n_blocks == 0) return hipSuccess;
  if (k < 2 || k > 4) return hipErrorInvalidValue;
  const dim3 grid(static_cast<uint32_t>((static_cast<int64_t>(n_blocks) + 7) / 8 * 8));
  if (k == 2)
    hipLaunchKernelGGL((dev::csr_block_spmm_kernel<ValT, 2>), grid, dim3(256), 0, st, blk, rp, col, val, X, Y, k,
                       n_blocks);
  else
    hipLaunchKernelGGL((dev::csr_block_spmm_kernel<ValT, 4>), grid, dim3(256), 0, st, blk, rp, col, val, X, Y, k,
                       n_blocks);
  return hipGetLastError();
}

template hipError_t launch_csr_block_spmm<double>(int32_t, const int32_t*, const int32_t*, const int32_t*,
                                                  const double*, const double*, double*, int32_t, hipStream_t);
template hipError_t launch_csr_block_spmm<float>(int32_t, const int32_t*, const int32_t*, const int32_t*,
                                                 const float*, const double*, double*, int32_t, hipStream_t);

void csr_row_blocks(int32_t n, const int32_t* rp, int32_t per, std::vector<int32_t>& blk) {
  const int64_t cap = 256 * static_cast<int64_t>(per);
  blk.clear();
  blk.push_back(0);
  int32_t r = 0;
  while (r < n) {
    int32_t e = r + 1;  // a row longer than cap still gets a block of its own
    while (e < n && e - r < kCsrBlockRows && rp[e + 1] - rp[r] <= cap) ++e;
    blk.push_back(e);
    r = e;
  }
}

hipError_t launch_atomic_symm(int32_t n, const int32_t* rp, const int32_t* col, const double* val, const double* x,
                              double* y, int32_t lpr, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::fill_zero_kernel, dim3(static_cast<uint32_t>((n + 255) / 256)), dim3(256), 0, st, y,
                     static_cast<int64_t>(n));
  const int64_t threads = static_cast<int64_t>(n) * lpr;
  const dim3 grid(static_cast<uint32_t>((threads + 255) / 256));
  switch (lpr) {
#define ATO_L(L)                                                                                      \
  case L:                                                                                             \
    hipLaunchKernelGGL(dev::atomic_symm_kernel<L>, grid, dim3(256), 0, st, n, rp, col, val, x, y); \
    break;
    ATO_L(1) ATO_L(2) ATO_L(4) ATO_L(8) ATO_L(16) ATO_L(32) ATO_L(64)
#undef ATO_L
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_tile(int32_t n, int32_t k, int32_t kt, double* full, double* tiles, int32_t to_tiles,
                       hipStream_t st) {
  const int64_t total = static_cast<int64_t>(n) * k;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::tile_kernel, fill_grid(total), dim3(256), 0, st, n, k, kt, full, tiles, to_tiles);
  return hipGetLastError();
}

hipError_t launch_permute(int32_t n, int32_t k, const int32_t* new2old, const double* in, double* out,
                          int32_t to_permuted, hipStream_t st) {
  const int64_t total = static_cast<int64_t>(n) * k;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::permute_kernel, dim3(static_cast<uint32_t>((total + 255) / 256)), dim3(256), 0, st, n, k,
                     new2old, in, out, to_permuted);
  return hipGetLastError();
}

}  // namespace race
