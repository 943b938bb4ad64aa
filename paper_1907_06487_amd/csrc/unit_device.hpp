// Device building blocks shared by the gfx950 kernels that run RACE units:
// the unit computation (window staging, slices, flush), clearing tasks and
// the dataflow ticket machinery.  Included by race_kernels.hip and
// mpk_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace race {
namespace dev {

constexpr int kSlice = 64;
constexpr uint16_t kNoRow = 0xFFFF;
// slots per lane loaded before any arithmetic: FP32 values take one register
// each, so a batch of 24 costs what 16 FP64 values do
template <typename ValT>
struct BatchSize {
  static constexpr int value = sizeof(ValT) == 4 ? 24 : (sizeof(ValT) == 8 ? 16 : 8);
};

// A value as a lane holds it in registers: real values in double, complex
// ones as they are; zero test and the zero of each type.
template <typename ValT>
struct RegOf {
  using type = double;
};
template <bool H>
struct RegOf<Cplx<H>> {
  using type = Cplx<H>;
};
__device__ __forceinline__ double to_reg(double v) { return v; }
__device__ __forceinline__ double to_reg(float v) { return static_cast<double>(v); }
template <bool H>
__device__ __forceinline__ Cplx<H> to_reg(Cplx<H> v) { return v; }
template <typename ValT>
__device__ __forceinline__ ValT zero_value() { return ValT(0); }
template <>
__device__ __forceinline__ Cplx<false> zero_value<Cplx<false>>() { return Cplx<false>{0.0, 0.0}; }
template <>
__device__ __forceinline__ Cplx<true> zero_value<Cplx<true>>() { return Cplx<true>{0.0, 0.0}; }
__device__ __forceinline__ bool nonzero(double v) { return v != 0.0; }
__device__ __forceinline__ bool nonzero(float v) { return v != 0.0f; }
template <bool H>
__device__ __forceinline__ bool nonzero(Cplx<H> v) { return v.re != 0.0 || v.im != 0.0; }

// acc = diag * x_r: per column for real values; one complex product (the
// two columns are the real and imaginary part) for complex ones
template <int K>
__device__ __forceinline__ void init_acc(double d, const double (&xr)[K], double (&acc)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = d * xr[k];
}
template <int K, bool H>
__device__ __forceinline__ void init_acc(Cplx<H> d, const double (&xr)[K], double (&acc)[K]) {
  static_assert(K == 2, "complex values take two columns");
  acc[0] = d.re * xr[0] - d.im * xr[1];
  acc[1] = d.re * xr[1] + d.im * xr[0];
}
constexpr uint32_t kSpinLimit = 1u << 16;  // bounded wait (milliseconds), then report and go on

// Load of a layout word that no kernel writes, at an index that is the same
// in every lane: through the constant address space the compiler issues a
// scalar load, which needs no vector-memory wait and no readfirstlane.
template <typename T>
__device__ __forceinline__ T uniform_load(const T* p, int64_t i) {
  using ConstT = const __attribute__((address_space(4))) T;
  return ((ConstT*)p)[i];
}

__device__ __forceinline__ UnitDesc uniform_load(const UnitDesc* p, int64_t i) {
  using I8 = int32_t __attribute__((ext_vector_type(8)));
  using ConstI8 = const __attribute__((address_space(4))) I8;
  const I8 w = ((ConstI8*)p)[i];
  return UnitDesc{w[0], w[1], w[2], w[3], w[4], w[5], w[6], w[7]};
}

// The matrix stream (slice values and slots) is read once per product:
// non-temporal loads, which do not keep the lines in the caches (measured
// 1-2% faster than plain loads on the 128^3 stencil; plain loads stay for
// x, which halos re-read, and for the small per-lane and halo arrays, where
// non-temporal loads were slower).
template <typename T>
__device__ __forceinline__ T stream_load(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <bool H>
__device__ __forceinline__ Cplx<H> stream_load(const Cplx<H>* p) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const d2 t = __builtin_nontemporal_load(reinterpret_cast<const d2*>(p));
  return Cplx<H>{t.x, t.y};
}

// One slice descriptor as held in registers by a wavefront.
template <typename ValT>
struct SliceRegs {
  static constexpr int kBatch = BatchSize<ValT>::value;
  int32_t len = 0, width = 0;
  uint32_t off = 0;
  uint16_t rs = kNoRow;
  typename RegOf<ValT>::type d{};
  ValT v[kBatch];
  int32_t sl[kBatch];
};

template <typename ValT>
__device__ __forceinline__ void load_slice_head(const UnitArgs<ValT>& a, int32_t c, int32_t lane, SliceRegs<ValT>& r) {
  // c is the same in every lane: the descriptor lives in scalar registers
  const int32_t meta = uniform_load(a.chunk_len, c);
  r.len = meta & 0xFFFF;
  r.width = meta >> 16;
  r.off = uniform_load(a.chunk_off, c);
  r.rs = a.lane_slot[static_cast<size_t>(c) * kSlice + lane];
  r.d = to_reg(a.lane_diag[static_cast<size_t>(c) * kSlice + lane]);
}

// Loads entries j0 .. j0 + kBatch - 1 of every lane's row.  The bound on j
// is the same for the whole wavefront, and lanes past the slice's rows read
// the last row's entries (in bounds, never applied), so the loads of a batch
// are issued back to back with no per-lane branches between them.
// kNT: non-temporal loads (the matrix streams once per product); false
// keeps its lines cacheable (matrix powers that come back to a unit soon).
template <bool kNT, typename T>
__device__ __forceinline__ T matrix_load(const T* p) {
  if constexpr (kNT) return stream_load(p);
  else return *p;
}

template <typename ValT, bool kNT = true>
__device__ __forceinline__ void load_batch(const UnitArgs<ValT>& a, int32_t lane, int32_t j0, SliceRegs<ValT>& r) {
  const int32_t l = lane < r.width ? lane : r.width - 1;
  // a wave-uniform base and a 32-bit per-lane byte offset (a slice spans
  // at most 2^22 entries): one offset register per load
  const char* vp = reinterpret_cast<const char*>(a.sell_val + r.off);
  const char* sp = reinterpret_cast<const char*>(a.sell_slot + r.off);
#pragma unroll
  for (int b = 0; b < SliceRegs<ValT>::kBatch; ++b) {
    const int32_t j = j0 + b;
    if (j < r.len) {
      const uint32_t e = static_cast<uint32_t>(l + j * r.width);
      r.v[b] = matrix_load<kNT>(reinterpret_cast<const ValT*>(vp + e * static_cast<uint32_t>(sizeof(ValT))));
      r.sl[b] = matrix_load<kNT>(reinterpret_cast<const uint16_t*>(sp + e * 2u));
    } else {
      r.v[b] = zero_value<ValT>();
      r.sl[b] = r.rs;
    }
  }
}

// Applies a loaded batch.  With one right-hand side the gathers of a group
// of kGather entries are all issued before the first is used; with more,
// each entry's K gathers already overlap and entries go one at a time
// (measured faster from K = 2 on).  A zero value (row padding) adds +0 to
// its own row's slot and nothing to acc.
template <int K, int B, typename ValT>
__device__ __forceinline__ void apply_batch(const ValT* v, const int32_t* sl, const double* xw, double* yw,
                                            const double (&xr)[K], double (&acc)[K]) {
  if constexpr (K > 1) {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (v[b] != ValT(0)) {
        const double vb = static_cast<double>(v[b]);
#pragma unroll
        for (int k = 0; k < K; ++k) {
          acc[k] += vb * xw[sl[b] * K + k];
          atomicAdd(&yw[sl[b] * K + k], vb * xr[k]);
        }
      }
    }
    return;
  }
  constexpr int kGather = 8;
#pragma unroll
  for (int g = 0; g < B; g += kGather) {
    double xg[kGather][K];
#pragma unroll
    for (int b = 0; b < kGather; ++b)
#pragma unroll
      for (int k = 0; k < K; ++k) xg[b][k] = g + b < B ? xw[sl[g + b] * K + k] : 0.0;
#pragma unroll
    for (int b = 0; b < kGather && g + b < B; ++b) {
      const bool nz = v[g + b] != ValT(0);
      const double vb = static_cast<double>(v[g + b]);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        acc[k] += vb * (nz ? xg[b][k] : 0.0);
        atomicAdd(&yw[sl[g + b] * K + k], nz ? vb * xr[k] : 0.0);
      }
    }
  }
}

// Complex values: the columns are the real and imaginary part of x and y.
// The gather takes a_rj x_j, the scatter a_jr x_r with a_jr = a_rj
// (complex symmetric) or conj(a_rj) (Hermitian).
template <int K, int B, bool H>
__device__ __forceinline__ void apply_batch(const Cplx<H>* v, const int32_t* sl, const double* xw, double* yw,
                                            const double (&xr)[K], double (&acc)[K]) {
  static_assert(K == 2, "complex values take two columns");
#pragma unroll
  for (int b = 0; b < B; ++b) {
    if (nonzero(v[b])) {
      const double re = v[b].re, im = v[b].im;
      const double xj_re = xw[sl[b] * 2], xj_im = xw[sl[b] * 2 + 1];
      acc[0] += re * xj_re - im * xj_im;
      acc[1] += re * xj_im + im * xj_re;
      const double sim = H ? -im : im;
      atomicAdd(&yw[sl[b] * 2], re * xr[0] - sim * xr[1]);
      atomicAdd(&yw[sl[b] * 2 + 1], re * xr[1] + sim * xr[0]);
    }
  }
}

// One unit with own rows [lo, lo + R) and halo list h[0..H), on one
// workgroup:
//   1. x window  xw[s] = x[row of slot s], y window yw[s] = 0   (LDS);
//      each wavefront's first slice is already being fetched meanwhile
//   2. every slice (up to 64 rows) is taken by one wavefront, one row per
//      lane:
//        acc  = diag * x[r] + sum_j v_j * xw[slot_j]      (the gather)
//        yw[slot_j] += v_j * x[r]  for every j           (the scatter, LDS atomics)
//        yw[slot_r] += acc
//   3. flush the window: y[g] = yw[s] when this unit is the first writer of
//      y[g], else y[g] += yw[s].  Units of different leaves that may run at
//      the same time never share an index (distance-2 coloring), so this
//      needs no global atomics; only indices shared with other units of the
//      unit's own leaf (when the layout marks them) take a global atomic add.
// x as a unit stages it: plain loads, or (kCoherent) agent-scope relaxed
// atomic loads for an x that other workgroups of the same launch wrote (the
// powers of a matrix-power launch), which read around the per-XCD caches
// where a line fetched early could hold entries not yet final.
template <bool kCoherent>
__device__ __forceinline__ double x_load(const double* p) {
  if constexpr (kCoherent) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return *p;
}

template <typename ValT, int K, bool kCohX = false, bool kNT = true>
__device__ __forceinline__ void compute_unit(const UnitArgs<ValT>& a, const UnitDesc& ud,
                                             const double* __restrict__ x, int32_t ld, double* xw, double* yw,
                                             uint32_t* gw, int32_t tid, int32_t nthr) {
  // window entries per thread per staging round, own rows and halo each
  constexpr int kStage = K == 1 ? 4 : (K <= 3 ? 2 : 1);
  const int32_t lane = tid & (kSlice - 1), nwaves = nthr / kSlice;
  const int32_t wave = __builtin_amdgcn_readfirstlane(tid / kSlice);
  const int32_t lo = ud.lo;
  const int32_t R = ud.hi - lo;
  const int32_t h0 = ud.h0;
  const int32_t H = ud.h1 - h0;
  const int32_t c1 = ud.c1;
  int32_t c = ud.c0 + wave;
  SliceRegs<ValT> cur;
  // 1. stage the windows.  Own rows [0, R) need no index (x is contiguous
  // there); halo slots R + [0, H) gather x through the halo list.  All loads
  // of a round are issued before the first wait, the wavefront's first slice
  // descriptor rides along with the first round and its first batch is
  // requested before the barrier; lanes past an end read a clamped, valid
  // address and drop the value.  A unit has at least one own row.
  const uint32_t* hal = a.halo + h0;
  const int32_t rounds_end = R > H ? R : H;
  for (int32_t base = 0; base < rounds_end; base += kStage * nthr) {
    uint32_t hw[kStage], fw[kStage];
    double xo[kStage][K], xh[kStage][K];
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
      const int32_t s = base + q * nthr + tid;
      hw[q] = H > 0 ? hal[s < H ? s : H - 1] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
      const int32_t s = base + q * nthr + tid;
      const uint32_t r = static_cast<uint32_t>(lo + (s < R ? s : R - 1));
      fw[q] = a.row_flags[r >> 4];
#pragma unroll
      for (int k = 0; k < K; ++k) xo[q][k] = x_load<kCohX>(x + static_cast<size_t>(r) * ld + k);
    }
    if (base == 0 && c < c1) load_slice_head(a, c, lane, cur);
    // window index with the first-writer flag in bit 31 and the shared flag
    // in bit 30, kept in LDS for the flush
    auto put_own = [&]() {
#pragma unroll
      for (int q = 0; q < kStage; ++q) {
        const int32_t s = base + q * nthr + tid;
        if (s < R) {
          const uint32_t r = static_cast<uint32_t>(lo + s);
          const uint32_t f = (fw[q] >> (2 * (r & 15))) & 3u;
          gw[s] = r | ((f & 1u) << 31) | ((f & 2u) << 29);
#pragma unroll
          for (int k = 0; k < K; ++k) {
            xw[s * K + k] = xo[q][k];
            yw[s * K + k] = 0.0;
          }
        }
      }
    };
    // with several right-hand sides the own rows go to LDS before the halo
    // values are requested, so both never occupy registers at once
    if constexpr (K > 2) put_own();
#pragma unroll
    for (int q = 0; q < kStage; ++q)
#pragma unroll
      for (int k = 0; k < K; ++k)
        xh[q][k] = H > 0 ? x_load<kCohX>(x + static_cast<size_t>(hw[q] & 0x3fffffffu) * ld + k) : 0.0;
    if constexpr (K <= 2) put_own();
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
      const int32_t s = base + q * nthr + tid;
      if (s < H) {
        gw[R + s] = hw[q];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          xw[(R + s) * K + k] = xh[q][k];
          yw[(R + s) * K + k] = 0.0;
        }
      }
    }
  }
  if (c < c1) load_batch<ValT, kNT>(a, lane, 0, cur);
  __syncthreads();
  // 2. slices: the next slice's descriptor is in flight during this slice's
  // arithmetic, its elements are requested right after
  while (c < c1) {
    const int32_t cn = c + nwaves;
    // the last wavefront's slice re-reads its own descriptor instead of
    // branching around the loads
    const int32_t cq = cn < c1 ? cn : c;
    const int32_t meta_n = uniform_load(a.chunk_len, cq);
    const uint32_t off_n = uniform_load(a.chunk_off, cq);
    const uint16_t rs_n = a.lane_slot[static_cast<size_t>(cq) * kSlice + lane];
    const ValT d_n = a.lane_diag[static_cast<size_t>(cq) * kSlice + lane];
    if (cur.rs != kNoRow) {
      double xr[K], acc[K];
#pragma unroll
      for (int k = 0; k < K; ++k) xr[k] = xw[cur.rs * K + k];
      init_acc<K>(cur.d, xr, acc);
      constexpr int B = SliceRegs<ValT>::kBatch;
      apply_batch<K, B>(cur.v, cur.sl, xw, yw, xr, acc);
      for (int32_t j0 = B; j0 < cur.len; j0 += B) {
        load_batch<ValT, kNT>(a, lane, j0, cur);
        apply_batch<K, B>(cur.v, cur.sl, xw, yw, xr, acc);
      }
#pragma unroll
      for (int k = 0; k < K; ++k) atomicAdd(&yw[cur.rs * K + k], acc[k]);
    }
    if (cn < c1) {
      cur.len = meta_n & 0xFFFF;
      cur.width = meta_n >> 16;
      cur.off = off_n;
      cur.rs = rs_n;
      cur.d = to_reg(d_n);
      load_batch<ValT, kNT>(a, lane, 0, cur);
    }
    c = cn;
  }
  __syncthreads();
}

// y entries that another workgroup may later read back go through
// agent-scope relaxed atomic loads and stores when kCoherent: on this
// architecture those bypass the non-coherent per-XCD caches, so a unit that
// waited for a predecessor's completion flag reads the predecessor's y
// without any cache-wide writeback or invalidation.
template <bool kCoherent>
__device__ __forceinline__ double y_load(const double* p) {
  if constexpr (kCoherent) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return *p;
}

template <bool kCoherent>
__device__ __forceinline__ void y_store(double* p, double v) {
  if constexpr (kCoherent) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else *p = v;
}

// Step 3 of a unit: flush the y window.  y[g] = yw[s] when this unit is the
// first writer of y[g], else y[g] += yw[s]; units of different leaves that
// may run at the same time never share an index (distance-2 coloring), so
// these need no global atomics.  Indices flagged shared (touched by several
// units of this unit's own leaf, which run concurrently) are combined with
// a global atomic add instead; they were cleared before the product when no
// earlier unit wrote them.
template <int K, bool kCoherent>
__device__ __forceinline__ void flush_unit(const UnitDesc& ud, double* __restrict__ y, int32_t ld, const double* yw,
                                           const uint32_t* gw, int32_t tid, int32_t nthr) {
  constexpr int kStage = K >= 8 ? 1 : (K >= 4 ? 2 : 8);
  const int32_t W = (ud.hi - ud.lo) + (ud.h1 - ud.h0);
  for (int32_t base = 0; base < W; base += kStage * nthr) {
    // the window's indices and values come out of LDS before the first y
    // load is issued
    uint32_t h[kStage];
    double w[kStage][K];
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
      const int32_t s = base + q * nthr + tid;
      h[q] = s < W ? gw[s] : 0x80000000u;
#pragma unroll
      for (int k = 0; k < K; ++k) w[q][k] = s < W ? yw[s * K + k] : 0.0;
    }
    double old[kStage][K];
#pragma unroll
    for (int q = 0; q < kStage; ++q)
#pragma unroll
      for (int k = 0; k < K; ++k)
        old[q][k] = (h[q] >> 30) ? 0.0 : y_load<kCoherent>(y + static_cast<size_t>(h[q] & 0x3fffffffu) * ld + k);
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
      const int32_t s = base + q * nthr + tid;
      if (s < W) {
        double* p = y + static_cast<size_t>(h[q] & 0x3fffffffu) * ld;
        if (h[q] & 0x40000000u) {
#pragma unroll
          for (int k = 0; k < K; ++k) unsafeAtomicAdd(p + k, w[q][k]);
        } else {
#pragma unroll
          for (int k = 0; k < K; ++k) y_store<kCoherent>(p + k, old[q][k] + w[q][k]);
        }
      }
    }
  }
}

// Device wall clock (constant rate, common to all CUs) for unit traces.
__device__ __forceinline__ uint64_t wall_clock() { return __builtin_amdgcn_s_memrealtime(); }

// One unit in dataflow order: compute, wait for the earlier units its touch
// set meets, flush with coherent y accesses, publish completion.
template <typename ValT, int K>
__device__ __forceinline__ void flow_unit(const UnitArgs<ValT>& a, int32_t u,
                                          const int32_t* dep_idx, uint32_t* done, uint32_t* status, uint64_t* trace,
                                          uint32_t epoch, const double* __restrict__ x, double* __restrict__ y,
                                          int32_t ld, double* xw, double* yw, uint32_t* gw, int32_t tid,
                                          int32_t nthr, bool wave0) {
  const uint64_t t0 = trace ? wall_clock() : 0;
  // the unit's arithmetic needs nothing from other units; only its flush
  // must follow the earlier units it conflicts with
  const UnitDesc ud = uniform_load(a.unit_desc, u);
  compute_unit<ValT, K>(a, ud, x, ld, xw, yw, gw, tid, nthr);
  const uint64_t t1 = trace ? wall_clock() : 0;
  const int32_t d0 = ud.d0, d1 = ud.d1;
  for (int32_t i = d0 + tid; i < d1; i += nthr) {
    const int32_t v = dep_idx[i];
    uint32_t spins = 0;
    while (__hip_atomic_load(done + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        atomicOr(status, 1u);
        break;
      }
    }
  }
  __syncthreads();
  const uint64_t t2 = trace ? wall_clock() : 0;
  flush_unit<K, true>(ud, y, ld, yw, gw, tid, nthr);
  // every thread's coherent y stores complete before the barrier, so the
  // completion flag written after it is only seen once they are visible
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (wave0) {
    if (tid == 0) {
      if (trace) {
        const uint64_t t3 = wall_clock();
        trace[4 * static_cast<size_t>(u) + 0] = t0;
        trace[4 * static_cast<size_t>(u) + 1] = t1;
        trace[4 * static_cast<size_t>(u) + 2] = t2;
        trace[4 * static_cast<size_t>(u) + 3] = t3;
      }
      __hip_atomic_store(done + u, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// A clearing task: y entries zero_idx[i0 .. i1) set to zero with coherent
// stores (later shared units add to them atomically), then published like a
// unit.
template <int K>
__device__ __forceinline__ void clear_task(const int32_t* __restrict__ zero_idx, int64_t i0, int64_t i1,
                                           double* __restrict__ y, int32_t ld, uint32_t* done_slot, uint32_t epoch,
                                           int32_t tid, int32_t nthr, bool wave0) {
  for (int64_t i = i0 + tid; i < i1; i += nthr) {
    double* p = y + static_cast<size_t>(zero_idx[i]) * ld;
#pragma unroll
    for (int k = 0; k < K; ++k) y_store<true>(p + k, 0.0);
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (wave0) {
    if (tid == 0) __hip_atomic_store(done_slot, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

constexpr int kSetAside = 8;          // tickets a workgroup can set aside to run an ownerless one first
constexpr uint32_t kOwnerCheck = 64;  // polls of a flag between checks that its ticket has an owner

// Ticket of completion flag v (units follow the clearing tasks).
__device__ __forceinline__ int32_t ticket_of_flag(const FlowArgs& f, int32_t v) {
  return v < f.n_units ? f.unit_ticket[v] + f.n_zero_tasks : v - f.n_units;
}

// Claims static ticket t for this launch: true when no workgroup had it yet.
__device__ __forceinline__ bool claim_ticket(uint32_t* claim, int32_t t, uint32_t epoch) {
  return atomicMax(claim + t, epoch) != epoch;
}

__device__ __forceinline__ uint32_t coherent_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until the conflict edges [d0, d1) have published.  A flag still
// unset whose ticket is static and unclaimed belongs to a workgroup that is
// not running: when `may_take`, the workgroup claims the lowest such ticket
// it met and returns it (the caller runs that ticket first), else it keeps
// waiting.  Returns -1 once every edge has published or a bounded wait gave
// up (status bit 0).  s_red[0] is INT32_MAX on entry and on return.
__device__ __forceinline__ int32_t wait_edges(const FlowArgs& f, int32_t d0, int32_t d1, uint32_t epoch,
                                              bool may_take, int32_t* s_red, int32_t tid, int32_t nthr,
                                              bool wave0) {
  for (;;) {
    for (int32_t i = d0 + tid; i < d1; i += nthr) {
      const int32_t v = f.dep_idx[i];
      uint32_t spins = 0;
      while (coherent_load(f.done + v) != epoch) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          atomicOr(f.status, 1u);
          break;
        }
        if (may_take && spins % kOwnerCheck == 0) {
          const int32_t tv = ticket_of_flag(f, v);
          if (tv < f.n_static && coherent_load(f.claim + tv) != epoch) {
            atomicMin(s_red, tv);
            break;
          }
        }
      }
    }
    __syncthreads();
    const int32_t c = __builtin_amdgcn_readfirstlane(s_red[0]);
    if (c == INT32_MAX) return -1;
    __syncthreads();
    if (wave0) {
      if (tid == 0) {
        s_red[0] = INT32_MAX;
        s_red[1] = claim_ticket(f.claim, c, epoch) ? c : -1;
      }
    }
    __syncthreads();
    const int32_t got = __builtin_amdgcn_readfirstlane(s_red[1]);
    if (got >= 0) return got;
    // another running workgroup claimed it meanwhile: wait again
  }
}

// Next ticket of a free workgroup: while static tickets may be unclaimed,
// the lowest unclaimed one; once all are claimed, the counter's next ticket
// (-1 when none is left).  Claims never revert within a launch, so a
// workgroup that saw them all claimed goes straight to the counter.
__device__ __forceinline__ int32_t next_ticket(const FlowArgs& f, uint32_t epoch, uint64_t ticket_base,
                                               bool& all_claimed, int32_t* s_red, int32_t bid, int32_t tid,
                                               int32_t nthr, bool wave0) {
  while (!all_claimed) {
    for (int32_t i = tid; i < f.n_static; i += nthr)
      if (coherent_load(f.claim + i) != epoch) {
        atomicMin(s_red, i);
        break;
      }
    __syncthreads();
    const int32_t c = __builtin_amdgcn_readfirstlane(s_red[0]);
    __syncthreads();
    if (c == INT32_MAX) {
      all_claimed = true;
      break;
    }
    if (wave0) {
      if (tid == 0) {
        s_red[0] = INT32_MAX;
        const bool mine = claim_ticket(f.claim, c, epoch);
        s_red[1] = mine ? c : -1;
        if (mine && c != bid) atomicAdd(f.takeovers, 1u);
      }
    }
    __syncthreads();
    const int32_t got = __builtin_amdgcn_readfirstlane(s_red[1]);
    if (got >= 0) return got;
  }
  __syncthreads();
  if (wave0) {
    if (tid == 0) {
      const uint64_t t = atomicAdd(reinterpret_cast<unsigned long long*>(f.counter), 1ull) - ticket_base;
      s_red[1] = t < static_cast<uint64_t>(f.n_tickets - f.n_static) ? f.n_static + static_cast<int32_t>(t) : -1;
    }
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(s_red[1]);
}

}  // namespace dev
}  // namespace race
