// gfx950 CRS kernels: the full-matrix SpMV yardsticks (lane per row group
// and row blocks), the expanded low-locality product (SpMV, SpMM, batch),
// and the SymmSpMV with device-wide atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "kernels.hpp"
#include "unit_device.hpp"

namespace race {
namespace dev {

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

// Full-matrix CRS SpMM over row blocks (X, Y row-major n x k, 2 <= k <=
// 16): blocks of at most 256 * PER entries (PER per thread).  The columns
// go in chunks of KB (KB = 2, 4 or 8): each entry's products with a chunk
// are kept in LDS (entry-major, KB per entry), then one thread per (row,
// column) adds its row's products in entry order; the entries' values and
// columns are loaded once for all chunks.  A full chunk with an even k
// reads an entry's X segment as 16-byte pieces; columns past k are computed
// on column k - 1 and never stored (the 16-byte reads also need X itself
// 16-byte aligned).  A block of one row longer than 256 * PER entries
// strides over it and reduces across the workgroup per column.  Blocks go
// to the XCDs in contiguous eighths.  kChunks: k may exceed KB (else the
// column loop runs once and compiles away).
template <typename ValT, int KB, int PER, bool kChunks>
__global__ void __launch_bounds__(256) csr_block_spmm_kernel(const int32_t* __restrict__ blk,
                                                             const int32_t* __restrict__ rp,
                                                             const int32_t* __restrict__ col,
                                                             const ValT* __restrict__ val,
                                                             const double* __restrict__ X, double* __restrict__ Y,
                                                             int32_t k, int32_t n_blocks) {
  constexpr int32_t kCap = 256 * PER;
  __shared__ double prod[kCap * KB];
  const int32_t t = static_cast<int32_t>(threadIdx.x);
  const int32_t b = xcd_block();
  if (b >= n_blocks) return;  // padding of the grid (uniform per workgroup)
  const int32_t r0 = uniform_load(blk, b), r1 = uniform_load(blk, b + 1);
  const int32_t e0 = uniform_load(rp, r0);
  const int32_t ne = uniform_load(rp, r1) - e0;
  const int32_t c_end = kChunks ? k : 1;
  if (ne > kCap) {
    for (int32_t c0 = 0; c0 < c_end; c0 += KB) {
      double s[KB];
#pragma unroll
      for (int j = 0; j < KB; ++j) s[j] = 0.0;
      for (int32_t i = e0 + t; i < e0 + ne; i += 256) {
        const double a = static_cast<double>(val[i]);
        const int64_t c = static_cast<int64_t>(col[i]) * k + c0;
#pragma unroll
        for (int j = 0; j < KB; ++j) s[j] += a * X[c + (c0 + j < k ? j : k - 1 - c0)];
      }
#pragma unroll
      for (int j = 0; j < KB; ++j)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s[j] += __shfl_xor(s[j], o, 64);
      if ((t & 63) == 0)
#pragma unroll
        for (int j = 0; j < KB; ++j) prod[(t >> 6) * KB + j] = s[j];
      __syncthreads();
      if (t < KB && c0 + t < k)
        Y[static_cast<int64_t>(r0) * k + c0 + t] = (prod[t] + prod[KB + t]) + (prod[2 * KB + t] + prod[3 * KB + t]);
      __syncthreads();
    }
    return;
  }
  int32_t c[PER];
  ValT v[PER];
  if (ne > 0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int32_t i = e0 + min(t + u * 256, ne - 1);
      c[u] = stream_load(col + i);
      v[u] = stream_load(val + i);
    }
  }
  const int32_t pairs = (r1 - r0) * KB;
  for (int32_t c0 = 0; c0 < c_end; c0 += KB) {
    if (ne > 0) {
      double xv[PER][KB];
      if (c0 + KB <= k && (k & 1) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0) {
        typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          const d2* xr = reinterpret_cast<const d2*>(X + static_cast<int64_t>(c[u]) * k + c0);
#pragma unroll
          for (int j = 0; j < KB / 2; ++j) {
            const d2 w = xr[j];
            xv[u][2 * j] = w.x;
            xv[u][2 * j + 1] = w.y;
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < PER; ++u)
#pragma unroll
          for (int j = 0; j < KB; ++j)
            xv[u][j] = X[static_cast<int64_t>(c[u]) * k + (c0 + j < k ? c0 + j : k - 1)];
      }
#pragma unroll
      for (int u = 0; u < PER; ++u)
        if (t + u * 256 < ne)
#pragma unroll
          for (int j = 0; j < KB; ++j) prod[(t + u * 256) * KB + j] = static_cast<double>(v[u]) * xv[u][j];
    }
    __syncthreads();
    for (int32_t p = t; p < pairs; p += 256) {
      const int32_t r = r0 + p / KB, j = p % KB;
      if (c0 + j >= k) continue;
      const int32_t a = rp[r] - e0, e = rp[r + 1] - e0;
      double s = 0.0;
      for (int32_t q = a; q < e; ++q) s += prod[q * KB + j];
      Y[static_cast<int64_t>(r) * k + c0 + j] = s;
    }
    __syncthreads();  // the next chunk overwrites the products
  }
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

}  // namespace dev

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
hipError_t launch_csr_block_spmm(int32_t n_blocks, const int32_t* blk, const int32_t* rp, const int32_t* col,
                                 const ValT* val, const double* X, double* Y, int32_t k, hipStream_t st) {
  if (n_blocks == 0) return hipSuccess;
  if (k < 2 || k > 16) return hipErrorInvalidValue;
  const dim3 grid(static_cast<uint32_t>((static_cast<int64_t>(n_blocks) + 7) / 8 * 8));
  // blocks of 512 entries up to 4 columns, of 256 from 5 (csr_spmm_block_per)
  if (k == 2)
    hipLaunchKernelGGL((dev::csr_block_spmm_kernel<ValT, 2, 2, false>), grid, dim3(256), 0, st, blk, rp, col, val, X,
                       Y, k, n_blocks);
  else if (k <= 4)
    hipLaunchKernelGGL((dev::csr_block_spmm_kernel<ValT, 4, 2, false>), grid, dim3(256), 0, st, blk, rp, col, val, X,
                       Y, k, n_blocks);
  else if (k <= 8)
    hipLaunchKernelGGL((dev::csr_block_spmm_kernel<ValT, 8, 1, false>), grid, dim3(256), 0, st, blk, rp, col, val, X,
                       Y, k, n_blocks);
  else  // chunks of 8 columns
    hipLaunchKernelGGL((dev::csr_block_spmm_kernel<ValT, 8, 1, true>), grid, dim3(256), 0, st, blk, rp, col, val, X,
                       Y, k, n_blocks);
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

}  // namespace race
