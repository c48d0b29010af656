// Single-workgroup exclusive scan of int32 counts; used for per-cell and
// per-tile offsets (tens of thousands of elements, so one workgroup suffices).
#pragma once
#include <hip/hip_runtime.h>

namespace gpf {
namespace {

constexpr int kScanThreads = 1024;

// out[i] = sum_{j<i} in[i]; out[n] = total.  in and out may alias.
// Launch with one workgroup of kScanThreads threads.
__global__ void __launch_bounds__(kScanThreads) scan_exclusive_kernel(const int* in, int* out,
                                                                      int n) {
  __shared__ int wave_sums[kScanThreads / 64];
  __shared__ int carry_s;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  if (tid == 0) carry_s = 0;
  __syncthreads();
  for (int base = 0; base < n; base += kScanThreads * 4) {
    int v[4];
    int local = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int i = base + tid * 4 + k;
      v[k] = (i < n) ? in[i] : 0;
      local += v[k];
    }
    // inclusive wave scan of `local`
    int incl = local;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      int t = __shfl_up(incl, off, 64);
      if (lane >= off) incl += t;
    }
    if (lane == 63) wave_sums[wid] = incl;
    __syncthreads();
    if (wid == 0) {
      int s = (lane < kScanThreads / 64) ? wave_sums[lane] : 0;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        int t = __shfl_up(s, off, 64);
        if (lane >= off) s += t;
      }
      if (lane < kScanThreads / 64) wave_sums[lane] = s;  // inclusive over waves
    }
    __syncthreads();
    int carry = carry_s;
    int run = carry + (wid > 0 ? wave_sums[wid - 1] : 0) + incl - local;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int i = base + tid * 4 + k;
      if (i < n) out[i] = run;
      run += v[k];
    }
    __syncthreads();
    if (tid == 0) carry_s = carry + wave_sums[kScanThreads / 64 - 1];
    __syncthreads();
  }
  if (tid == 0) out[n] = carry_s;
}

}  // namespace
}  // namespace gpf
