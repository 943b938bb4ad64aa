// Attainable-bandwidth kernels: a read-only stream and a copy over large
// arrays with 16-byte loads and stores.  They measure the memory bandwidth
// a kernel can reach on this device, the input of the roofline bound (the
// paper measures load-only and copy bandwidths for the same purpose,
// Table 1 and Eq. upper_performance).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/race.h"
#include "errors.hpp"

namespace race {
namespace dev {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kInFlight = 8;  // 16-byte loads per thread per round

// Non-temporal 16-byte load and store: streamed data is used once, and
// keeping it out of the caches measured 10-15% faster than plain accesses
// for a read over 4 GiB on this chip.
__device__ __forceinline__ u32x4 nt_load(const u32x4* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void nt_store(u32x4 v, u32x4* p) { __builtin_nontemporal_store(v, p); }

// Loads every 16-byte element of src once (grid-stride, kInFlight loads in
// flight per thread) and folds them into one word per thread; the word is
// stored only when it equals a fixed constant, so the loads stay live while
// almost nothing is written.
__global__ void __launch_bounds__(256) stream_read_kernel(const u32x4* __restrict__ src, int64_t n16,
                                                          uint32_t* __restrict__ sink) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (; i + (kInFlight - 1) * stride < n16; i += kInFlight * stride) {
    u32x4 v[kInFlight];
#pragma unroll
    for (int u = 0; u < kInFlight; ++u) v[u] = nt_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < kInFlight; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (; i < n16; i += stride) {
    const u32x4 a = nt_load(src + i);
    acc ^= a.x ^ a.y ^ a.z ^ a.w;
  }
  if (acc == 0x9e3779b9u) sink[0] = acc;
}

// dst = src, 16-byte elements, kInFlight in flight per thread.
__global__ void __launch_bounds__(256) stream_copy_kernel(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                          int64_t n16) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  for (; i + (kInFlight - 1) * stride < n16; i += kInFlight * stride) {
    u32x4 v[kInFlight];
#pragma unroll
    for (int u = 0; u < kInFlight; ++u) v[u] = nt_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < kInFlight; ++u) nt_store(v[u], dst + i + u * stride);
  }
  for (; i < n16; i += stride) nt_store(nt_load(src + i), dst + i);
}

}  // namespace dev

// a and b are the streamed arrays (b NULL for the read, whose sink needs
// no alignment)
static int check_stream_args(int64_t bytes, int32_t grid, const void* a, const void* b) {
  if (bytes < 0 || bytes % 16 != 0) return set_error(RACE_EINVAL, "bytes must be a non-negative multiple of 16");
  if (grid < 1 || grid > (1 << 20)) return set_error(RACE_EINVAL, "grid must be in 1..2^20 workgroups");
  if (bytes > 0 && !a) return set_error(RACE_EINVAL, "NULL device pointer");
  if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) % 16 != 0)
    return set_error(RACE_EINVAL, "streamed arrays must be 16-byte aligned");
  return RACE_OK;
}

}  // namespace race

extern "C" {

int race_stream_read(const void* src, int64_t bytes, uint32_t* sink, int32_t grid, void* stream) {
  int rc = race::check_stream_args(bytes, grid, src, nullptr);
  if (rc) return rc;
  if (bytes > 0 && !sink) return race::set_error(RACE_EINVAL, "sink is NULL");
  if (bytes == 0) return RACE_OK;
  hipLaunchKernelGGL(race::dev::stream_read_kernel, dim3(static_cast<uint32_t>(grid)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), static_cast<const race::dev::u32x4*>(src), bytes / 16, sink);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return race::set_hip_error(e, "stream read launch");
  return RACE_OK;
}

int race_stream_copy(const void* src, void* dst, int64_t bytes, int32_t grid, void* stream) {
  int rc = race::check_stream_args(bytes, grid, src, dst);
  if (rc) return rc;
  if (bytes > 0 && !dst) return race::set_error(RACE_EINVAL, "dst is NULL");
  if (bytes == 0) return RACE_OK;
  hipLaunchKernelGGL(race::dev::stream_copy_kernel, dim3(static_cast<uint32_t>(grid)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), static_cast<const race::dev::u32x4*>(src), static_cast<race::dev::u32x4*>(dst),
                     bytes / 16);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return race::set_hip_error(e, "stream copy launch");
  return RACE_OK;
}

}  // extern "C"
