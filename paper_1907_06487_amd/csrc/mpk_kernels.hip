// gfx950 matrix-power kernel: the products y_p = A y_(p-1) of several
// powers in one persistent dataflow launch (Section 7 names in-place matrix
// powers and polynomials as the next users of RACE schedules), and the
// combination of the powers into a polynomial.
//
// Tickets are (power, unit) pairs: power-major by default (inside a power
// the schedule's own ticket order with its clearing tasks first), or any
// order from a table that keeps the static tickets and every wait pointing
// to a smaller ticket (a diagonal order lets a unit's next power follow it
// while its part of the matrix may still be cached).  A unit of
// power p first waits until every unit whose touch set meets its window has
// flushed power p - 1 (its x is then final), computes, waits for the
// conflict edges of power p like a single product, flushes into y_p and
// publishes.  Every wait points to a smaller ticket, so the argument of the
// single-product launch carries over; static tickets are all of power 0.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.hpp"
#include "unit_device.hpp"

namespace race {
namespace dev {

// Waits until every unit in the read-dependency list of unit u has
// published power p - 1 (flags done_prev); bounded, reported through status.
__device__ __forceinline__ void wait_reads(const MpkArgs& m, int32_t u, const uint32_t* done_prev, uint32_t* status,
                                           uint32_t epoch, int32_t tid, int32_t nthr) {
  const int32_t r0 = uniform_load(m.rdep_ptr, u), r1 = uniform_load(m.rdep_ptr, u + 1);
  for (int32_t i = r0 + tid; i < r1; i += nthr) {
    const int32_t v = m.rdep_idx[i];
    uint32_t spins = 0;
    while (coherent_load(done_prev + v) != epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        atomicOr(status, 1u);
        break;
      }
    }
  }
  __syncthreads();
}

template <typename ValT, bool kNT>
__global__ void __launch_bounds__(1024) race_mpk_kernel(UnitArgs<ValT> a, FlowArgs f, MpkArgs m,
                                                        const double* __restrict__ x, double* __restrict__ Y,
                                                        int32_t wmax, uint32_t epoch, uint64_t ticket_base) {
  extern __shared__ double smem[];
  double* xw = smem;
  double* yw = smem + static_cast<size_t>(wmax);
  uint32_t* gw = reinterpret_cast<uint32_t*>(smem + 2 * static_cast<size_t>(wmax));
  __shared__ int32_t s_red[2];
  __shared__ int32_t s_aside[kSetAside];
  const int32_t tid = static_cast<int32_t>(threadIdx.x), nthr = static_cast<int32_t>(blockDim.x);
  const int32_t bid = static_cast<int32_t>(blockIdx.x);
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
  const int32_t n_flags = f.n_units + f.n_zero_tasks;
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
    const int32_t pm = m.order ? uniform_load(m.order, t) : t;
    const int32_t p = pm / m.per_power;
    const int32_t r = pm - p * m.per_power;
    FlowArgs fp = f;
    fp.done = f.done + static_cast<size_t>(p) * n_flags;
    double* yp = Y + static_cast<size_t>(p) * m.n;
    if (r < f.n_zero_tasks) {
      const int64_t i0 = static_cast<int64_t>(r) * f.zero_chunk;
      clear_task<1>(f.zero_idx, i0, i0 + f.zero_chunk < f.n_zero ? i0 + f.zero_chunk : f.n_zero, yp, 1,
                    fp.done + f.n_units + r, epoch, tid, nthr, wave0);
      t = -1;
      continue;
    }
    const int32_t u = uniform_load(f.ticket_unit, r - f.n_zero_tasks);
    const UnitDesc ud = uniform_load(a.unit_desc, u);
    if (p == 0) {
      compute_unit<ValT, 1, false, kNT>(a, ud, x, 1, xw, yw, gw, tid, nthr);
    } else {
      // x of this power is the previous power's y: final once every unit
      // touching the window has flushed it
      wait_reads(m, u, f.done + static_cast<size_t>(p - 1) * n_flags, f.status, epoch, tid, nthr);
      compute_unit<ValT, 1, true, kNT>(a, ud, Y + static_cast<size_t>(p - 1) * m.n, 1, xw, yw, gw, tid, nthr);
    }
    // static tickets are all of power 0: only there can a waited-for
    // ticket lack a running owner
    const int32_t rr = wait_edges(fp, ud.d0, ud.d1, epoch, p == 0 && aside < kSetAside, s_red, tid, nthr, wave0);
    if (rr >= 0) {
      if (wave0) {
        if (tid == 0) {
          s_aside[aside] = t;
          atomicAdd(f.takeovers, 1u);
        }
      }
      ++aside;
      t = rr;
      continue;
    }
    flush_unit<1, true>(ud, yp, 1, yw, gw, tid, nthr);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __syncthreads();
    if (wave0) {
      if (tid == 0) __hip_atomic_store(fp.done + u, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    t = -1;
  }
}

// z = c[0] x + sum_{p=1..P} c[p] Y[p - 1], elementwise (coefficients as
// kernel arguments).
__global__ void __launch_bounds__(256) poly_combine_kernel(int64_t n, int32_t P, PolyCoeffs c,
                                                           const double* __restrict__ x, const double* __restrict__ Y,
                                                           double* __restrict__ z) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    double acc = c.c[0] * x[i];
    for (int32_t p = 1; p <= P; ++p) acc += c.c[p] * Y[static_cast<size_t>(p - 1) * n + i];
    z[i] = acc;
  }
}

}  // namespace dev

template <typename ValT>
struct MpkTag {};

template <typename ValT>
hipError_t launch_race_mpk(const UnitArgs<ValT>& a, const FlowArgs& f, const MpkArgs& m, const double* x, double* Y,
                           int32_t wmax, int32_t threads, int32_t grid, uint32_t epoch, uint64_t ticket_base,
                           hipStream_t st) {
  static bool attr_done = false;
  const void* fns[2] = {reinterpret_cast<const void*>(&dev::race_mpk_kernel<ValT, true>),
                        reinterpret_cast<const void*>(&dev::race_mpk_kernel<ValT, false>)};
  if (!attr_done) {
    for (const void* fn : fns) {
      hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 159 * 1024);
      if (e != hipSuccess) return e;
    }
    attr_done = true;
  }
  if (m.cache_matrix)
    hipLaunchKernelGGL((dev::race_mpk_kernel<ValT, false>), dim3(static_cast<uint32_t>(grid)),
                       dim3(static_cast<uint32_t>(threads)), window_lds_bytes(wmax, 1), st, a, f, m, x, Y, wmax, epoch,
                       ticket_base);
  else
    hipLaunchKernelGGL((dev::race_mpk_kernel<ValT, true>), dim3(static_cast<uint32_t>(grid)),
                       dim3(static_cast<uint32_t>(threads)), window_lds_bytes(wmax, 1), st, a, f, m, x, Y, wmax, epoch,
                       ticket_base);
  return hipGetLastError();
}

template <typename ValT>
hipError_t race_mpk_occupancy(int32_t threads, int32_t wmax, int32_t* blocks_per_cu) {
  // both forms (non-temporal or cacheable matrix loads): the larger need
  hipFuncAttributes attr{}, attr2{};
  hipError_t e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(&dev::race_mpk_kernel<ValT, true>));
  if (e == hipSuccess) e = hipFuncGetAttributes(&attr2, reinterpret_cast<const void*>(&dev::race_mpk_kernel<ValT, false>));
  if (e != hipSuccess) return e;
  attr.sharedSizeBytes = std::max(attr.sharedSizeBytes, attr2.sharedSizeBytes);
  const int32_t regs = std::max({attr.numRegs, attr2.numRegs, 1});
  const int32_t waves_per_block = std::max(1, threads / 64);
  const int32_t waves_per_simd = std::max(1, std::min(8, 512 / ((regs + 7) / 8 * 8)));
  const int32_t by_waves = (4 * waves_per_simd) / waves_per_block;
  const size_t lds = window_lds_bytes(wmax, 1) + static_cast<size_t>(attr.sharedSizeBytes);
  const int32_t by_lds = static_cast<int32_t>((160 * 1024) / (lds + 1));
  *blocks_per_cu = std::max(0, std::min(by_waves, by_lds));
  return hipSuccess;
}

hipError_t launch_poly_combine(int64_t n, int32_t P, const PolyCoeffs& c, const double* x, const double* Y, double* z,
                               hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint32_t grid = static_cast<uint32_t>(std::max<int64_t>(1, std::min<int64_t>(8192, (n + 255) / 256)));
  hipLaunchKernelGGL(dev::poly_combine_kernel, dim3(grid), dim3(256), 0, st, n, P, c, x, Y, z);
  return hipGetLastError();
}

template hipError_t launch_race_mpk<double>(const UnitArgs<double>&, const FlowArgs&, const MpkArgs&, const double*,
                                            double*, int32_t, int32_t, int32_t, uint32_t, uint64_t, hipStream_t);
template hipError_t launch_race_mpk<float>(const UnitArgs<float>&, const FlowArgs&, const MpkArgs&, const double*,
                                           double*, int32_t, int32_t, int32_t, uint32_t, uint64_t, hipStream_t);
template hipError_t race_mpk_occupancy<double>(int32_t, int32_t, int32_t*);
template hipError_t race_mpk_occupancy<float>(int32_t, int32_t, int32_t*);

}  // namespace race
