// Photon-to-Gaussian initialisation: photon grid, k nearest neighbours,
// network features, the parameter mapping, and network training targets.
#include <rocprim/device/device_scan.hpp>

#include <cmath>

#include "common.h"
#include "mlp.h"
#include "pointgrid.h"

namespace gpf {
namespace {

constexpr int kMaxK = 32;
constexpr int kPhotonDim = 256;  // cells per axis (max)

// One thread per photon: rings of cells around its own cell until the k-th
// best distance is below the distance to any unvisited cell.
template <int K>
__global__ void __launch_bounds__(256) knn_kernel(const float* __restrict__ pos, int64_t n, PGrid g,
                                                  const int* __restrict__ start,
                                                  const int* __restrict__ sorted,
                                                  int* __restrict__ out_idx,
                                                  float* __restrict__ out_d2, int k) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float px = pos[i * 3], py = pos[i * 3 + 1], pz = pos[i * 3 + 2];
  const int3 c = pcell(g, px, py, pz);
  float bd[K];
  int bi[K];
#pragma unroll
  for (int a = 0; a < K; ++a) {
    bd[a] = INFINITY;
    bi[a] = 0x7fffffff;
  }
  const int maxr = max(g.dx, max(g.dy, g.dz));
  for (int rr = 0; rr <= maxr; ++rr) {
    for (int z = c.z - rr; z <= c.z + rr; ++z) {
      if (z < 0 || z >= g.dz) continue;
      for (int y = c.y - rr; y <= c.y + rr; ++y) {
        if (y < 0 || y >= g.dy) continue;
        for (int x = c.x - rr; x <= c.x + rr; ++x) {
          if (x < 0 || x >= g.dx) continue;
          if (max(abs(x - c.x), max(abs(y - c.y), abs(z - c.z))) != rr) continue;
          const int cell = (z * g.dy + y) * g.dx + x;
          for (int s = start[cell]; s < start[cell + 1]; ++s) {
            const int j = sorted[s];
            if (j == (int)i) continue;
            const float d = sqd(px, py, pz, pos[(int64_t)j * 3], pos[(int64_t)j * 3 + 1],
                                pos[(int64_t)j * 3 + 2]);
            if (!before(d, j, bd[K - 1], bi[K - 1])) continue;
            bd[K - 1] = d;
            bi[K - 1] = j;
#pragma unroll
            for (int a = K - 1; a > 0; --a) {
              if (before(bd[a], bi[a], bd[a - 1], bi[a - 1])) {
                const float td = bd[a];
                bd[a] = bd[a - 1];
                bd[a - 1] = td;
                const int ti = bi[a];
                bi[a] = bi[a - 1];
                bi[a - 1] = ti;
              }
            }
          }
        }
      }
    }
    // any photon outside rings 0..rr is at least rr * h away
    float kth = bd[0];
#pragma unroll
    for (int a = 1; a < K; ++a)
      if (a == k - 1) kth = bd[a];
    const float reach = (float)rr * g.h;
    if (kth < reach * reach * (1.f - 1e-5f)) break;
  }
#pragma unroll
  for (int a = 0; a < K; ++a)
    if (a < k) {
      out_idx[i * k + a] = bi[a];
      out_d2[i * k + a] = bd[a];
    }
}

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// features [n][96] (bfloat16): per neighbour (offset / r16, log power ratio)
__global__ void __launch_bounds__(256) features_kernel(const float* __restrict__ pos,
                                                       const float* __restrict__ power, int64_t n,
                                                       const int* __restrict__ idx,
                                                       const float* __restrict__ d2,
                                                       uint16_t* __restrict__ X) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float r16 = fmaxf(sqrtf(d2[i * 16 + 15]), 1e-12f);
  const float inv = 1.f / r16;
  const float px = pos[i * 3], py = pos[i * 3 + 1], pz = pos[i * 3 + 2];
  const float lp0 = logf(fmaxf(power[i * 3], 1e-30f)), lp1 = logf(fmaxf(power[i * 3 + 1], 1e-30f)),
              lp2 = logf(fmaxf(power[i * 3 + 2], 1e-30f));
  for (int a = 0; a < 16; ++a) {
    const int64_t j = idx[i * 16 + a];
    uint16_t* o = X + i * kIn + 6 * a;
    o[0] = f2bf((pos[j * 3] - px) * inv);
    o[1] = f2bf((pos[j * 3 + 1] - py) * inv);
    o[2] = f2bf((pos[j * 3 + 2] - pz) * inv);
    o[3] = f2bf(logf(fmaxf(power[j * 3], 1e-30f)) - lp0);
    o[4] = f2bf(logf(fmaxf(power[j * 3 + 1], 1e-30f)) - lp1);
    o[5] = f2bf(logf(fmaxf(power[j * 3 + 2], 1e-30f)) - lp2);
  }
}

constexpr float kSMin = 1e-4f, kSMax = 0.1f;

// Gaussian parameters: plain initialisation (Y == nullptr) or corrected by the
// network outputs Y [n][10].
__global__ void __launch_bounds__(256) params_kernel(const float* __restrict__ pos,
                                                     const float* __restrict__ power, int64_t n,
                                                     const float* __restrict__ d2, int k,
                                                     const float* __restrict__ Y,
                                                     gpf_field_out out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  float o[kOut];
#pragma unroll
  for (int a = 0; a < kOut; ++a) o[a] = Y ? Y[i * kOut + a] : 0.f;
  const float r3 = sqrtf(d2[i * k + 2]);
  const float base = logf(fminf(fmaxf(r3, kSMin), kSMax));
  float q[4] = {1.f + o[0], o[1], o[2], o[3]};
  const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if (qn > 0.f) {
#pragma unroll
    for (int a = 0; a < 4; ++a) q[a] /= qn;
  } else {
    q[0] = 1.f;
    q[1] = q[2] = q[3] = 0.f;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    out.mu[i * 3 + a] = pos[i * 3 + a];
    out.log_scale[i * 3 + a] = base + o[4 + a];
    out.rgb[i * 3 + a] = power[i * 3 + a] * __expf(o[7 + a]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) out.quat[i * 4 + a] = q[a];
}

// Network targets from a fitted field whose i-th Gaussian started at photon i.
__global__ void __launch_bounds__(256) targets_kernel(const float* __restrict__ power, int64_t n,
                                                      const float* __restrict__ d2, int k,
                                                      const float* __restrict__ quat,
                                                      const float* __restrict__ ls,
                                                      const float* __restrict__ rgb,
                                                      float* __restrict__ T) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  float q[4] = {quat[i * 4], quat[i * 4 + 1], quat[i * 4 + 2], quat[i * 4 + 3]};
  const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const float sg = q[0] < 0.f ? -1.f : 1.f;
  const float iq = qn > 0.f ? sg / qn : 0.f;
  T[i * kOut + 0] = q[0] * iq - 1.f;
  T[i * kOut + 1] = q[1] * iq;
  T[i * kOut + 2] = q[2] * iq;
  T[i * kOut + 3] = q[3] * iq;
  const float base = logf(fminf(fmaxf(sqrtf(d2[i * k + 2]), kSMin), kSMax));
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T[i * kOut + 4 + a] = ls[i * 3 + a] - base;
    const float P = fmaxf(power[i * 3 + a], 1e-30f);
    T[i * kOut + 7 + a] = logf(fmaxf(rgb[i * 3 + a], 1e-6f * P) / P);
  }
}

}  // namespace

gpf_status photon_knn(const float* pos, int64_t n, int k, int* idx, float* d2, hipStream_t s) {
  // bounding box -> cubic cells holding about one photon per cell in volume
  const int nb = kPointBoxBlocks;
  float* part = nullptr;
  gpf_status st = dev_alloc((void**)&part, nb * 6 * sizeof(float), "photon box");
  if (st != GPF_OK) return st;
  hipLaunchKernelGGL(pbox_kernel, dim3(nb), dim3(256), 0, s, pos, n, part);
  float hp[nb * 6];
  hipError_t e = hipMemcpyAsync(hp, part, sizeof(hp), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free(part, nb * 6 * sizeof(float));
  if (e != hipSuccess) return hip_fail(e, "photon box");
  PGrid g;
  st = point_grid_geometry(hp, n, kPhotonDim, &g);
  if (st != GPF_OK) return st;
  const int64_t cells = (int64_t)g.dx * g.dy * g.dz;
  int *cnt = nullptr, *start = nullptr, *sorted = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  auto cleanup = [&]() {
    dev_free(cnt, (cells + 1) * 4);
    dev_free(start, (cells + 1) * 4);
    dev_free(sorted, n * 4);
    dev_free(tmp, tmp_bytes);
  };
  if ((st = dev_alloc((void**)&cnt, (cells + 1) * 4, "photon cells")) != GPF_OK ||
      (st = dev_alloc((void**)&start, (cells + 1) * 4, "photon cells")) != GPF_OK ||
      (st = dev_alloc((void**)&sorted, n * 4, "photon order")) != GPF_OK) {
    cleanup();
    return st;
  }
  e = hipMemsetAsync(cnt, 0, (cells + 1) * 4, s);
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(pcount_kernel, dim3(blocks), dim3(256), 0, s, pos, n, g, cnt);
  if (e == hipSuccess)
    e = rocprim::exclusive_scan(nullptr, tmp_bytes, cnt, start, 0, (size_t)(cells + 1),
                                rocprim::plus<int>(), s);
  if (e == hipSuccess && (st = dev_alloc(&tmp, tmp_bytes, "scan scratch")) != GPF_OK) {
    cleanup();
    return st;
  }
  if (e == hipSuccess)
    e = rocprim::exclusive_scan(tmp, tmp_bytes, cnt, start, 0, (size_t)(cells + 1),
                                rocprim::plus<int>(), s);
  if (e == hipSuccess) e = hipMemsetAsync(cnt, 0, (cells + 1) * 4, s);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "photon grid");
  }
  hipLaunchKernelGGL(pscatter_kernel, dim3(blocks), dim3(256), 0, s, pos, n, g, start, cnt, sorted);
  if (k <= 16)
    hipLaunchKernelGGL(knn_kernel<16>, dim3(blocks), dim3(256), 0, s, pos, n, g, start, sorted, idx, d2, k);
  else
    hipLaunchKernelGGL(knn_kernel<kMaxK>, dim3(blocks), dim3(256), 0, s, pos, n, g, start, sorted, idx, d2, k);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  cleanup();
  if (e != hipSuccess) return hip_fail(e, "photon knn");
  return GPF_OK;
}

gpf_status photon_features(const float* pos, const float* power, int64_t n, const int* idx,
                           const float* d2, uint16_t* X, hipStream_t s) {
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pos, power,
                     n, idx, d2, X);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

gpf_status photon_params(const float* pos, const float* power, int64_t n, const float* d2, int k,
                         const float* Y, gpf_field_out out, hipStream_t s) {
  hipLaunchKernelGGL(params_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pos, power,
                     n, d2, k, Y, out);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

gpf_status photon_targets(const float* power, int64_t n, const float* d2, int k, const float* quat,
                          const float* ls, const float* rgb, float* T, hipStream_t s) {
  hipLaunchKernelGGL(targets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, power, n,
                     d2, k, quat, ls, rgb, T);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

}  // namespace gpf
