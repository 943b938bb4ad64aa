// gfx950 kernels: RACE SymmSpMV / SymmSpMM (phases, dataflow, batch), the
// tile and permutation kernels.  The CRS kernels are in csr_kernels.hip.
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
