// Measurement helper, built as its own library (libgpf_probe.so) and kept out
// of the radiance library's C ABI: an FP32 FMA issue-rate probe that gives
// the VALU ceiling the radiance kernels are measured against on the machine
// at hand (a non-packed FP32 FMA stream at full occupancy).
//
//   int gpf_probe_valu(float *out, int64_t out_len, int blocks, int iters,
//                      void *stream);
//
// Enqueues `blocks` workgroups of 256 threads on `stream`; each thread runs
// iters x 64 FP32 fused multiply-adds over 8 independent chains, every
// operand a vector register (form 0 below: the fastest form, so the ceiling),
// and writes one float to out[blocks * 256] (device, caller-owned).  The work is
// blocks * 256 * iters * 128 flops.  Returns 0, 1 for a bad argument
// (out NULL, blocks < 1, iters < 1, out_len < blocks * 256) or 2 when the
// launch fails.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

// Operand-form probes: 8 independent chains per lane, 64 instructions of the
// form per iteration.  x and y are per-lane (vector registers); a and b are
// kernel arguments (scalar registers).
#define GPF_PROBE_INIT                                               \
  float v[8], x[8], y[8];                                            \
  for (int i = 0; i < 8; ++i) {                                      \
    v[i] = threadIdx.x * 1e-3f + i;                                  \
    x[i] = a + (i + 1) * 1e-3f * threadIdx.x;                        \
    y[i] = b - (i + 1) * 1e-4f * threadIdx.x;                        \
  }
#define GPF_PROBE_STORE                                              \
  float s = 0.f;                                                     \
  for (int i = 0; i < 8; ++i) s += v[i] + x[i] + y[i];               \
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;

__global__ void __launch_bounds__(256) form_vvv(float* __restrict__ out, int iters, float a, float b) {
  GPF_PROBE_INIT
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = fmaf(v[i], x[i], y[(i + r) & 7]);
  GPF_PROBE_STORE
}

__global__ void __launch_bounds__(256) form_vsv(float* __restrict__ out, int iters, float a, float b) {
  GPF_PROBE_INIT
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = fmaf(x[i], a, v[i]);
  GPF_PROBE_STORE
}

__global__ void __launch_bounds__(256) form_lit(float* __restrict__ out, int iters, float a, float b) {
  GPF_PROBE_INIT
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = fmaf(x[i], 1.2345f, v[i]);
  GPF_PROBE_STORE
}

__global__ void __launch_bounds__(256) form_exp(float* __restrict__ out, int iters, float a, float b) {
  GPF_PROBE_INIT
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = __builtin_amdgcn_exp2f(v[i]);
  GPF_PROBE_STORE
}

__global__ void __launch_bounds__(256) form_sel(float* __restrict__ out, int iters, float a, float b) {
  GPF_PROBE_INIT
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = (v[i] <= x[i]) ? y[i] : v[i];
  GPF_PROBE_STORE
}

}  // namespace

extern "C" int gpf_probe_valu_form(float* out, int64_t out_len, int blocks, int iters, int form,
                                   float a, float b, void* stream) {
  if (!out || blocks < 1 || iters < 1 || out_len < (int64_t)blocks * 256) return 1;
  void (*k)(float*, int, float, float) = nullptr;
  switch (form) {
    case 0: k = form_vvv; break;
    case 1: k = form_vsv; break;
    case 2: k = form_lit; break;
    case 3: k = form_exp; break;
    case 4: k = form_sel; break;
    default: return 1;
  }
  hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, (hipStream_t)stream, out, iters, a, b);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

extern "C" int gpf_probe_valu(float* out, int64_t out_len, int blocks, int iters, void* stream) {
  return gpf_probe_valu_form(out, out_len, blocks, iters, 0, 1.0001f, 1e-7f, stream);
}
