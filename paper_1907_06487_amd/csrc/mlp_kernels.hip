// gfx950 kernels of the cost-model network (12 -> 64 -> 64 -> 1, ReLU,
// float32): batched inference, mean-squared-error gradient, Adam.
//
// The network is tiny (5057 parameters, about 5k multiply-adds per sample)
// and every sample is independent, so one lane owns one sample: the weights
// are read at wave-uniform addresses (scalar loads, shared by the whole
// wavefront) and the activations stay in registers.  The gradient is a sum
// over samples of outer products; each workgroup of 256 samples stages the
// per-sample factors in LDS (sample-major, padded against bank conflicts)
// and reduces them to one partial gradient per workgroup; a second kernel
// adds the partials in a fixed order, so the result does not depend on
// scheduling.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "mlp.hpp"

namespace race {
namespace dev {

constexpr int kIn = kMlpIn, kHid = kMlpHid;
constexpr int kBlock = 256;   // samples per workgroup of the gradient kernel
constexpr int kPadH = kHid + 1;
constexpr int kPadX = kIn + 1;

struct Net {
  const float* W1;
  const float* b1;
  const float* W2;
  const float* b2;
  const float* w3;
  float b3;
};

__device__ __forceinline__ Net net(const float* __restrict__ theta) {
  Net p;
  p.W1 = theta;
  p.b1 = p.W1 + kHid * kIn;
  p.W2 = p.b1 + kHid;
  p.b2 = p.W2 + kHid * kHid;
  p.w3 = p.b2 + kHid;
  p.b3 = p.w3[kHid];
  return p;
}

// h1 = relu(W1 x + b1)
__device__ __forceinline__ void layer1(const Net& p, const float* x, float* h1) {
#pragma unroll
  for (int j = 0; j < kHid; ++j) {
    float z = p.b1[j];
#pragma unroll
    for (int i = 0; i < kIn; ++i) z = __builtin_fmaf(p.W1[j * kIn + i], x[i], z);
    h1[j] = z > 0.0f ? z : 0.0f;
  }
}

// z2 row o = W2[o] . h1 + b2[o]
__device__ __forceinline__ float layer2_row(const Net& p, const float* h1, int o) {
  float z = p.b2[o];
#pragma unroll
  for (int j = 0; j < kHid; ++j) z = __builtin_fmaf(p.W2[o * kHid + j], h1[j], z);
  return z;
}

__global__ void __launch_bounds__(256) mlp_forward_kernel(const float* __restrict__ theta,
                                                          const float* __restrict__ X, int64_t n,
                                                          float* __restrict__ y) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const Net p = net(theta);
  float x[kIn], h1[kHid];
  const bool valid = s < n;
#pragma unroll
  for (int i = 0; i < kIn; ++i) x[i] = valid ? X[s * kIn + i] : 0.0f;
  layer1(p, x, h1);
  float f = p.b3;
  for (int o = 0; o < kHid; ++o) {
    const float z = layer2_row(p, h1, o);
    if (z > 0.0f) f = __builtin_fmaf(p.w3[o], z, f);
  }
  if (valid) y[s] = f;
}

// One workgroup: 256 samples.  partial[blockIdx.x * (P + 1) + q] receives
// the workgroup's share of dL/dtheta_q (q < P) and of the loss (q = P), with
// L = (1/n) sum (f - t)^2.
__global__ void __launch_bounds__(kBlock) mlp_grad_kernel(const float* __restrict__ theta,
                                                          const float* __restrict__ X,
                                                          const float* __restrict__ t, int64_t n,
                                                          float* __restrict__ partial) {
  __shared__ float A[kBlock * kPadH];
  __shared__ float B[kBlock * kPadH];
  __shared__ float Xs[kBlock * kPadX];
  __shared__ float gs[kBlock];
  __shared__ float es[kBlock];
  const int tid = static_cast<int>(threadIdx.x);
  const int64_t s = static_cast<int64_t>(blockIdx.x) * kBlock + tid;
  const bool valid = s < n;
  const Net p = net(theta);
  float* out = partial + static_cast<size_t>(blockIdx.x) * (kMlpParams + 1);
  float* oW1 = out;
  float* ob1 = oW1 + kHid * kIn;
  float* oW2 = ob1 + kHid;
  float* ob2 = oW2 + kHid * kHid;
  float* ow3 = ob2 + kHid;

  float x[kIn], h1[kHid], h2[kHid];
#pragma unroll
  for (int i = 0; i < kIn; ++i) x[i] = valid ? X[s * kIn + i] : 0.0f;
  layer1(p, x, h1);
  float f = p.b3;
#pragma unroll
  for (int o = 0; o < kHid; ++o) {
    const float z = layer2_row(p, h1, o);
    h2[o] = z > 0.0f ? z : 0.0f;
    f = __builtin_fmaf(p.w3[o], h2[o], f);
  }
  const float r = valid ? f - t[s] : 0.0f;
  const float g = 2.0f * r / static_cast<float>(n);  // dL/df of this sample

  // stage 0: dL/dw3 = sum g h2, dL/db3 = sum g, loss = sum r^2 / n
#pragma unroll
  for (int o = 0; o < kHid; ++o) A[tid * kPadH + o] = g * h2[o];
  gs[tid] = g;
  es[tid] = r * r;
  __syncthreads();
  if (tid < kHid) {
    float acc = 0.0f;
    for (int q = 0; q < kBlock; ++q) acc += A[q * kPadH + tid];
    ow3[tid] = acc;
  } else if (tid == kHid) {
    float acc = 0.0f;
    for (int q = 0; q < kBlock; ++q) acc += gs[q];
    out[kMlpParams - 1] = acc;
  } else if (tid == kHid + 1) {
    float acc = 0.0f;
    for (int q = 0; q < kBlock; ++q) acc += es[q];
    out[kMlpParams] = acc / static_cast<float>(n);
  }
  __syncthreads();

  // stage 1: dz2 = g w3 [z2 > 0]; dL/dW2 = sum dz2 h1^T, dL/db2 = sum dz2
#pragma unroll
  for (int o = 0; o < kHid; ++o) h2[o] = h2[o] > 0.0f ? g * p.w3[o] : 0.0f;  // h2 now holds dz2
#pragma unroll
  for (int j = 0; j < kHid; ++j) {
    A[tid * kPadH + j] = h1[j];
    B[tid * kPadH + j] = h2[j];
  }
  __syncthreads();
  {
    const int o = tid >> 2, j0 = (tid & 3) * 16;
    float acc[16];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) acc[jj] = 0.0f;
    float accb = 0.0f;
    for (int q = 0; q < kBlock; ++q) {
      const float d = B[q * kPadH + o];
      accb += d;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) acc[jj] = __builtin_fmaf(d, A[q * kPadH + j0 + jj], acc[jj]);
    }
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) oW2[o * kHid + j0 + jj] = acc[jj];
    if ((tid & 3) == 0) ob2[o] = accb;
  }
  __syncthreads();

  // stage 2: dz1 = (W2^T dz2) [z1 > 0]; dL/dW1 = sum dz1 x^T, dL/db1 = sum dz1
#pragma unroll
  for (int j = 0; j < kHid; ++j) {
    float d = 0.0f;
    if (h1[j] > 0.0f) {
#pragma unroll
      for (int o = 0; o < kHid; ++o) d = __builtin_fmaf(p.W2[o * kHid + j], h2[o], d);
    }
    B[tid * kPadH + j] = d;
  }
#pragma unroll
  for (int i = 0; i < kIn; ++i) Xs[tid * kPadX + i] = x[i];
  __syncthreads();
  {
    const int j = tid >> 2, i0 = (tid & 3) * 3;
    float acc[3] = {0.0f, 0.0f, 0.0f};
    float accb = 0.0f;
    for (int q = 0; q < kBlock; ++q) {
      const float d = B[q * kPadH + j];
      accb += d;
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) acc[ii] = __builtin_fmaf(d, Xs[q * kPadX + i0 + ii], acc[ii]);
    }
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) oW1[j * kIn + i0 + ii] = acc[ii];
    if ((tid & 3) == 0) ob1[j] = accb;
  }
}

// grad[q] = sum over workgroups of partial[.][q], in workgroup order; the
// loss is entry P.
__global__ void __launch_bounds__(256) mlp_reduce_kernel(const float* __restrict__ partial, int32_t blocks,
                                                         float* __restrict__ grad, float* __restrict__ loss) {
  const int q = static_cast<int>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q > kMlpParams) return;
  float acc = 0.0f;
  for (int32_t b = 0; b < blocks; ++b) acc += partial[static_cast<size_t>(b) * (kMlpParams + 1) + q];
  if (q < kMlpParams) grad[q] = acc;
  else if (loss) *loss = acc;
}

// Adam (Kingma and Ba, Algorithm 1) with the bias corrections folded into
// c1 = 1 / (1 - beta1^step) and c2 = 1 / (1 - beta2^step).
__global__ void __launch_bounds__(256) mlp_adam_kernel(float* __restrict__ theta, const float* __restrict__ grad,
                                                       float* __restrict__ m, float* __restrict__ v, float lr,
                                                       float beta1, float beta2, float eps, float c1, float c2) {
  const int q = static_cast<int>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= kMlpParams) return;
  const float gq = grad[q];
  const float mq = beta1 * m[q] + (1.0f - beta1) * gq;
  const float vq = beta2 * v[q] + (1.0f - beta2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  theta[q] -= lr * (mq * c1) / (__builtin_sqrtf(vq * c2) + eps);
}

}  // namespace dev

int64_t mlp_workspace_floats(int64_t n) { return ((n + dev::kBlock - 1) / dev::kBlock) * (kMlpParams + 1); }

hipError_t launch_mlp_forward(const float* theta, const float* X, int64_t n, float* y, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::mlp_forward_kernel, dim3(static_cast<uint32_t>((n + 255) / 256)), dim3(256), 0, st, theta,
                     X, n, y);
  return hipGetLastError();
}

hipError_t launch_mlp_loss_grad(const float* theta, const float* X, const float* t, int64_t n, float* workspace,
                                float* grad, float* loss, hipStream_t st) {
  const int32_t blocks = static_cast<int32_t>((n + dev::kBlock - 1) / dev::kBlock);
  hipLaunchKernelGGL(dev::mlp_grad_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(dev::kBlock), 0, st, theta, X,
                     t, n, workspace);
  hipLaunchKernelGGL(dev::mlp_reduce_kernel, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, st, workspace, blocks,
                     grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* theta, const float* grad, float* m, float* v, float lr, float beta1, float beta2,
                           float eps, float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(dev::mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, theta, grad, m, v, lr,
                     beta1, beta2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace race
