// Measurement helper, built as its own library (libgpf_probe.so) and kept out
// of the radiance library's C ABI: an FP32 FMA issue-rate probe that gives
// the VALU ceiling the radiance kernels are measured against on the machine
// at hand (a non-packed FP32 FMA stream at full occupancy).
//
//   int gpf_probe_valu(float *out, int64_t out_len, int blocks, int iters,
//                      void *stream);
//
// Enqueues `blocks` workgroups of 256 threads on `stream`; each thread runs
// iters x 64 independent FP32 fused multiply-adds (8 chains) and writes one
// float to out[blocks * 256] (device, caller-owned).  The work is
// blocks * 256 * iters * 128 flops.  Returns 0, 1 for a bad argument
// (out NULL, blocks < 1, iters < 1, out_len < blocks * 256) or 2 when the
// launch fails.
#include <hip/hip_runtime.h>

#include <cstdint>

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

extern "C" int gpf_probe_valu(float* out, int64_t out_len, int blocks, int iters, void* stream) {
  if (!out || blocks < 1 || iters < 1 || out_len < (int64_t)blocks * 256) return 1;
  hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, out,
                     iters);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}
