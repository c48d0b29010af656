// Fitting-loop kernels: MSE loss with its upstream gradient (Sec. 4.3) and a
// fused Adam update (the paper optimises with Adam).
#include "common.h"

namespace gpf {
namespace {

__global__ void __launch_bounds__(256) mse_kernel(const float* __restrict__ L,
                                                  const float* __restrict__ T, int64_t q,
                                                  double* __restrict__ loss,
                                                  float* __restrict__ dL) {
  const float scale = (float)(2.0 / (double)q);
  double local = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < q * 3;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float d = L[i] - T[i];
    dL[i] = scale * d;
    local += (double)d * (double)d;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) local += __shfl_xor(local, off, 64);
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, part[0] + part[1] + part[2] + part[3]);
}

__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ p,
                                                   const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   int64_t n, float lr, float b1, float b2,
                                                   float eps, float bc1, float bc2,
                                                   const double* __restrict__ guard) {
  if (guard && !isfinite(*guard)) return;   // a non-finite loss leaves the state as it was
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

int blocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

gpf_status launch_mse(const float* L, const float* T, int64_t q, double* loss, float* dL,
                      hipStream_t s) {
  hipLaunchKernelGGL(mse_kernel, dim3(blocks_for(q * 3)), dim3(256), 0, s, L, T, q, loss, dL);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

gpf_status launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, int64_t step, const double* guard, hipStream_t s) {
  const float bc1 = (float)(1.0 - std::pow((double)b1, (double)step));
  const float bc2 = (float)(1.0 - std::pow((double)b2, (double)step));
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2,
                     eps, bc1, bc2, guard);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

}  // namespace gpf
