// gfx950 Gauss-Seidel sweep over a distance-1 RACE schedule: one launch per
// phase, one wavefront per leaf (leaves of one phase share no edge, so they
// run at the same time), the rows of a leaf in order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gs_kernels.hpp"

namespace race {
namespace dev {

constexpr int kGsLanes = 64;
constexpr int kGsAhead = 8;  // rows whose entries are in flight ahead of the running row

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

// One row's first 64 off-diagonal entries as this lane holds them (lane l
// takes entry l; lanes past the row hold slot 0 and value 0), with the
// row's right-hand side, diagonal and entry range.
struct GsRow {
  double v = 0.0;
  uint32_t sl = 0;
  double b = 0.0, d = 1.0;
  int32_t e0 = 0, e1 = 0;
};

__device__ __forceinline__ void gs_load_row(const GsArgs& a, const double* __restrict__ bvec, int32_t i,
                                            int32_t lane, GsRow& r) {
  r.e0 = gs_uniform(a.row_ptr, i);
  r.e1 = gs_uniform(a.row_ptr, i + 1);
  r.b = gs_uniform(bvec, i);
  r.d = gs_uniform(a.diag, i);
  const int32_t e = r.e0 + lane;
  r.v = 0.0;
  r.sl = 0u;
  if (e < r.e1) {
    r.v = a.val[e];
    r.sl = a.slot[e];
  }
}

// One leaf: stage the window (own rows and halo) in LDS, update the rows in
// order (backward: last row first) with
//   x_i = (b_i - sum_j a_ij x_j) / a_ii
// reading every x_j from the window and writing x_i into it, then store the
// own rows back.  The entries of the next kGsAhead rows are in flight while
// a row is summed; they do not depend on x.
template <bool kBackward>
__global__ void __launch_bounds__(kGsLanes) gs_leaf_kernel(GsArgs a, int32_t leaf0, const double* __restrict__ bvec,
                                                          double* __restrict__ x) {
  extern __shared__ double xw[];
  const int32_t leaf = leaf0 + static_cast<int32_t>(blockIdx.x);
  const int32_t lane = static_cast<int32_t>(threadIdx.x);
  const int32_t lo = gs_uniform(a.leaf_lo, leaf), hi = gs_uniform(a.leaf_hi, leaf);
  const int32_t h0 = gs_uniform(a.halo_ptr, leaf), h1 = gs_uniform(a.halo_ptr, leaf + 1);
  const int32_t R = hi - lo, H = h1 - h0;
  for (int32_t s = lane; s < R; s += kGsLanes) xw[s] = x[lo + s];
  for (int32_t s = lane; s < H; s += kGsLanes) xw[R + s] = x[a.halo[h0 + s]];
  GsRow ring[kGsAhead];
#pragma unroll
  for (int p = 0; p < kGsAhead; ++p)
    if (p < R) gs_load_row(a, bvec, kBackward ? hi - 1 - p : lo + p, lane, ring[p]);
  __syncthreads();
  for (int32_t t0 = 0; t0 < R; t0 += kGsAhead) {
#pragma unroll
    for (int p = 0; p < kGsAhead; ++p) {
      const int32_t t = t0 + p;
      if (t < R) {
        const int32_t i = kBackward ? hi - 1 - t : lo + t;
        double s = ring[p].v * xw[ring[p].sl];
        // entries past the first 64 (long rows) are loaded when the row runs
        for (int32_t e = ring[p].e0 + kGsLanes + lane; e < ring[p].e1; e += kGsLanes) s += a.val[e] * xw[a.slot[e]];
        const double bi = ring[p].b, di = ring[p].d;
        const int32_t tn = t + kGsAhead;
        if (tn < R) gs_load_row(a, bvec, kBackward ? hi - 1 - tn : lo + tn, lane, ring[p]);
        const double xi = (bi - wave_sum(s)) / di;
        if (lane == 0) xw[i - lo] = xi;
        __syncthreads();
      }
    }
  }
  for (int32_t s = lane; s < R; s += kGsLanes) x[lo + s] = xw[s];
}

}  // namespace dev

hipError_t launch_gs_phase(const GsArgs& a, int32_t leaf0, int32_t count, int32_t wmax, bool backward,
                           const double* b, double* x, hipStream_t st) {
  if (count == 0) return hipSuccess;
  static bool attr_done[2] = {false, false};
  const void* fn = backward ? reinterpret_cast<const void*>(&dev::gs_leaf_kernel<true>)
                            : reinterpret_cast<const void*>(&dev::gs_leaf_kernel<false>);
  if (!attr_done[backward]) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kGsMaxWindowBytes);
    if (e != hipSuccess) return e;
    attr_done[backward] = true;
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
