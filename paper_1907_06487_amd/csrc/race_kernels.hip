// gfx950 kernels: RACE SymmSpMV / SymmSpMM, the full-CRS SpMV and the
// global-atomic SymmSpMV baselines, and the permutation kernel.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace race {
namespace dev {

constexpr int kSlice = 64;
constexpr uint16_t kNoRow = 0xFFFF;

// One workgroup runs one leaf of a phase: the leaf's units in order.  For a
// unit with own rows [lo, lo + R) and halo list h[0..H):
//   1. x window  xw[s] = x[row of slot s], y window yw[s] = 0   (LDS)
//   2. every 64-row slice is taken by one wavefront, one row per lane:
//        acc  = diag * x[r] + sum_j v_j * xw[slot_j]      (the gather)
//        yw[slot_j] += v_j * x[r]  for every j           (the scatter, LDS atomics)
//        yw[slot_r] += acc
//   3. flush the window: y[g] = yw[s] when this unit is the first writer of
//      y[g], else y[g] += yw[s].  Units of one phase never share an index
//      (distance-2 coloring), so the flush needs no global atomics.
template <typename ValT, int K>
__global__ void __launch_bounds__(1024) race_leaf_kernel(UnitArgs<ValT> a, int32_t leaf_base,
                                                         const double* __restrict__ x, double* __restrict__ y,
                                                         int32_t wmax) {
  extern __shared__ double smem[];
  double* xw = smem;
  double* yw = smem + static_cast<size_t>(wmax) * K;
  const int32_t leaf = leaf_base + static_cast<int32_t>(blockIdx.x);
  const int32_t u0 = a.leaf_unit_ptr[leaf], u1 = a.leaf_unit_ptr[leaf + 1];
  const int32_t tid = static_cast<int32_t>(threadIdx.x), nthr = static_cast<int32_t>(blockDim.x);
  const int32_t lane = tid & (kSlice - 1), wave = tid / kSlice, nwaves = nthr / kSlice;
  for (int32_t u = u0; u < u1; ++u) {
    const int32_t lo = a.unit_lo[u];
    const int32_t R = a.unit_hi[u] - lo;
    const int32_t h0 = a.unit_halo_ptr[u];
    const int32_t W = R + (a.unit_halo_ptr[u + 1] - h0);
    for (int32_t s = tid; s < W; s += nthr) {
      const int32_t g = s < R ? lo + s : static_cast<int32_t>(a.halo[h0 + s - R] & 0x7fffffffu);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        xw[s * K + k] = x[static_cast<size_t>(g) * K + k];
        yw[s * K + k] = 0.0;
      }
    }
    __syncthreads();
    const int32_t c1 = a.unit_chunk_ptr[u + 1];
    for (int32_t c = a.unit_chunk_ptr[u] + wave; c < c1; c += nwaves) {
      const uint16_t rs = a.lane_slot[static_cast<size_t>(c) * kSlice + lane];
      if (rs != kNoRow) {
        const int32_t meta = a.chunk_len[c];
        const int32_t len = meta & 0xFFFF, width = meta >> 16;
        const ValT* vp = a.sell_val + a.chunk_off[c] + lane;
        const uint16_t* sp = a.sell_slot + a.chunk_off[c] + lane;
        const double d = static_cast<double>(a.lane_diag[static_cast<size_t>(c) * kSlice + lane]);
        double xr[K], acc[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          xr[k] = xw[rs * K + k];
          acc[k] = d * xr[k];
        }
        for (int32_t j = 0; j < len; ++j) {
          const double v = static_cast<double>(vp[j * width]);
          const int32_t s = sp[j * width];
          if (v != 0.0) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
              acc[k] += v * xw[s * K + k];
              atomicAdd(&yw[s * K + k], v * xr[k]);
            }
          }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) atomicAdd(&yw[rs * K + k], acc[k]);
      }
    }
    __syncthreads();
    for (int32_t s = tid; s < W; s += nthr) {
      int32_t g;
      bool first;
      if (s < R) {
        g = lo + s;
        first = (a.row_first_bits[g >> 5] >> (g & 31)) & 1u;
      } else {
        const uint32_t h = a.halo[h0 + s - R];
        g = static_cast<int32_t>(h & 0x7fffffffu);
        first = (h >> 31) != 0u;
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        double* dst = y + static_cast<size_t>(g) * K + k;
        *dst = first ? yw[s * K + k] : *dst + yw[s * K + k];
      }
    }
    __syncthreads();
  }
}

// Full-matrix CRS SpMV (Algorithm "SpMV"), LPR lanes per row.
template <int LPR>
__global__ void __launch_bounds__(256) csr_spmv_kernel(int32_t n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col, const double* __restrict__ val,
                                                       const double* __restrict__ x, double* __restrict__ y) {
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t row = gid / LPR;
  const int32_t l = static_cast<int32_t>(gid % LPR);
  if (row >= n) return;  // whole lane groups leave together
  double s = 0.0;
  const int32_t e = rp[row + 1];
  for (int32_t i = rp[row] + l; i < e; i += LPR) s += val[i] * x[col[i]];
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) s += __shfl_down(s, o, LPR);
  if (l == 0) y[row] = s;
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
static hipError_t launch_leaf(const UnitArgs<ValT>& a, int32_t leaf_base, int32_t n_leaves, const double* x, double* y,
                              int32_t wmax, int32_t threads, hipStream_t st) {
  const size_t lds = 2 * static_cast<size_t>(wmax) * K * sizeof(double);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&dev::race_leaf_kernel<ValT, K>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((dev::race_leaf_kernel<ValT, K>), dim3(n_leaves), dim3(threads), lds, st, a, leaf_base, x, y,
                     wmax);
  return hipGetLastError();
}

template <typename ValT>
hipError_t launch_race_phase(const UnitArgs<ValT>& a, int32_t leaf_base, int32_t n_leaves, int32_t k, const double* x,
                             double* y, int32_t wmax, int32_t threads, hipStream_t st) {
  switch (k) {
#define RACE_K(KK) \
  case KK:         \
    return launch_leaf<ValT, KK>(a, leaf_base, n_leaves, x, y, wmax, threads, st);
    RACE_K(1) RACE_K(2) RACE_K(3) RACE_K(4) RACE_K(5) RACE_K(6) RACE_K(7) RACE_K(8)
    RACE_K(9) RACE_K(10) RACE_K(11) RACE_K(12) RACE_K(13) RACE_K(14) RACE_K(15) RACE_K(16)
#undef RACE_K
    default:
      return hipErrorInvalidValue;
  }
}

template hipError_t launch_race_phase<double>(const UnitArgs<double>&, int32_t, int32_t, int32_t, const double*,
                                              double*, int32_t, int32_t, hipStream_t);
template hipError_t launch_race_phase<float>(const UnitArgs<float>&, int32_t, int32_t, int32_t, const double*,
                                             double*, int32_t, int32_t, hipStream_t);

hipError_t launch_csr_spmv(int32_t n, const int32_t* rp, const int32_t* col, const double* val, const double* x,
                           double* y, int32_t lpr, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t threads = static_cast<int64_t>(n) * lpr;
  const dim3 grid(static_cast<uint32_t>((threads + 255) / 256));
  switch (lpr) {
#define CSR_L(L)                                                                                   \
  case L:                                                                                          \
    hipLaunchKernelGGL(dev::csr_spmv_kernel<L>, grid, dim3(256), 0, st, n, rp, col, val, x, y); \
    break;
    CSR_L(1) CSR_L(2) CSR_L(4) CSR_L(8) CSR_L(16) CSR_L(32) CSR_L(64)
#undef CSR_L
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
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

hipError_t launch_permute(int32_t n, int32_t k, const int32_t* new2old, const double* in, double* out,
                          int32_t to_permuted, hipStream_t st) {
  const int64_t total = static_cast<int64_t>(n) * k;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::permute_kernel, dim3(static_cast<uint32_t>((total + 255) / 256)), dim3(256), 0, st, n, k,
                     new2old, in, out, to_permuted);
  return hipGetLastError();
}

}  // namespace race
