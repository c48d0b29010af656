// Measurement helper: FP32 FMA issue-rate probe.  Gives the VALU ceiling the
// radiance kernels are measured against on the machine at hand (a
// non-packed FP32 FMA stream at full occupancy).
#include "common.h"

namespace gpf {
namespace {

constexpr int kProbeChains = 8;  // independent FMA chains per lane

__global__ void __launch_bounds__(256) valu_probe_kernel(float* __restrict__ out, int iters) {
  const int t = threadIdx.x;
  const float a = 1.0f + t * 1e-6f, b = 0.5f - t * 1e-7f;
  float v[kProbeChains];
#pragma unroll
  for (int i = 0; i < kProbeChains; ++i) v[i] = t * 1e-3f + i;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 64 / kProbeChains; ++r)
#pragma unroll
      for (int i = 0; i < kProbeChains; ++i) v[i] = fmaf(v[i], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < kProbeChains; ++i) s += v[i];
  out[(int64_t)blockIdx.x * 256 + t] = s;
}

}  // namespace

gpf_status launch_valu_probe(float* out, int blocks, int iters, hipStream_t s) {
  hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(256), 0, s, out, iters);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

}  // namespace gpf
