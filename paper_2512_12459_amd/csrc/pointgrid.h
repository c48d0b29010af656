// Uniform grid over a point set (counting sort by cell) and the
// single-precision distance order used for nearest-neighbour decisions.
// Shared by the photon kNN (init.hip) and the nearest-centre top-up of the
// hybrid query (hybrid.hip).
#pragma once

#include <cmath>

#include "common.h"

namespace gpf {
namespace {

struct PGrid {
  float ox, oy, oz, h;
  int dx, dy, dz;
};

__device__ __forceinline__ int3 pcell(const PGrid& g, float x, float y, float z) {
  int3 c;
  c.x = min(max((int)floorf((x - g.ox) / g.h), 0), g.dx - 1);
  c.y = min(max((int)floorf((y - g.oy) / g.h), 0), g.dy - 1);
  c.z = min(max((int)floorf((z - g.oz) / g.h), 0), g.dz - 1);
  return c;
}

// min / max that keep a NaN once seen (fminf / fmaxf would drop it), so
// that a NaN coordinate reaches the host-side finiteness check.
__device__ __forceinline__ float nan_min(float a, float b) { return (b < a || b != b) ? b : a; }
__device__ __forceinline__ float nan_max(float a, float b) { return (b > a || b != b) ? b : a; }

__global__ void pbox_kernel(const float* __restrict__ pos, int64_t n, float* part) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = nan_min(lo[a], pos[i * 3 + a]);
      hi[a] = nan_max(hi[a], pos[i * 3 + a]);
    }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = nan_min(lo[a], __shfl_xor(lo[a], off, 64));
      hi[a] = nan_max(hi[a], __shfl_xor(hi[a], off, 64));
    }
  __shared__ float s[4][6];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int a = 0; a < 3; ++a) {
      s[w][a] = lo[a];
      s[w][3 + a] = hi[a];
    }
  __syncthreads();
  if (threadIdx.x < 6) {
    float v = s[0][threadIdx.x];
    for (int k = 1; k < 4; ++k)
      v = threadIdx.x < 3 ? nan_min(v, s[k][threadIdx.x]) : nan_max(v, s[k][threadIdx.x]);
    part[blockIdx.x * 6 + threadIdx.x] = v;
  }
}

__global__ void pcount_kernel(const float* __restrict__ pos, int64_t n, PGrid g,
                              int* __restrict__ cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int3 c = pcell(g, pos[i * 3], pos[i * 3 + 1], pos[i * 3 + 2]);
  atomicAdd(&cnt[(c.z * g.dy + c.y) * g.dx + c.x], 1);
}

__global__ void pscatter_kernel(const float* __restrict__ pos, int64_t n, PGrid g,
                                const int* __restrict__ start, int* __restrict__ fill,
                                int* __restrict__ sorted) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int3 c = pcell(g, pos[i * 3], pos[i * 3 + 1], pos[i * 3 + 2]);
  const int cell = (c.z * g.dy + c.y) * g.dx + c.x;
  const int slot = atomicAdd(&fill[cell], 1);
  sorted[start[cell] + slot] = (int)i;
}

// Cell of each point (sort key) and its index (sort value), for a stable
// radix sort that lists every cell's points in index order without atomics.
__global__ void point_key_kernel(const float* __restrict__ pos, int64_t n, PGrid g,
                                 unsigned* __restrict__ key, int* __restrict__ val) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int3 c = pcell(g, pos[i * 3], pos[i * 3 + 1], pos[i * 3 + 2]);
  key[i] = (unsigned)((c.z * g.dy + c.y) * g.dx + c.x);
  val[i] = (int)i;
}

// start[c] = first position of cell c in the sorted keys (c = 0 .. cells;
// start[cells] = n): a binary search per cell.
__global__ void sorted_cell_starts_kernel(const unsigned* __restrict__ key_s, int64_t n,
                                          int64_t cells, int* __restrict__ start) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c > cells) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)key_s[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  start[c] = (int)lo;
}

// Bits of a radix sort over cell keys 0 .. cells - 1.
inline int cell_key_bits(int64_t cells) {
  int bits = 1;
  while (bits < 32 && ((int64_t)1 << bits) < cells) ++bits;
  return bits;
}

// (d2, index) order; FP32 squared distance without fused multiply-add
__device__ __forceinline__ float sqd(float ax, float ay, float az, float bx, float by, float bz) {
#pragma clang fp contract(off)
  const float dx = bx - ax, dy = by - ay, dz = bz - az;
  return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ bool before(float da, int ia, float db, int ib) {
  return da < db || (da == db && ia < ib);
}

constexpr int kPointBoxBlocks = 64;  // blocks of pbox_kernel (partial boxes)

// Geometry of a point grid from the partial boxes pbox_kernel wrote: cubic
// cells holding about one point each in the box's volume (or of edge `cell`
// when cell > 0), at most maxdim per axis.  Fails on non-finite coordinates.
inline gpf_status point_grid_geometry(const float* hp, int64_t n, int maxdim, PGrid* g,
                                      double cell = 0.0) {
  float lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = hp[a];
    hi[a] = hp[3 + a];
    for (int b = 1; b < kPointBoxBlocks; ++b) {
      const float l = hp[b * 6 + a], h = hp[b * 6 + 3 + a];
      lo[a] = (l < lo[a] || l != l) ? l : lo[a];
      hi[a] = (h > hi[a] || h != h) ? h : hi[a];
    }
    if (!std::isfinite(lo[a]) || !std::isfinite(hi[a]))
      return set_error(GPF_ERR_INVALID_ARGUMENT, "positions contain NaN or Inf");
  }
  double ext = 0;
  for (int a = 0; a < 3; ++a) ext = std::fmax(ext, (double)hi[a] - lo[a]);
  double vol = 1;
  for (int a = 0; a < 3; ++a) vol *= std::fmax((double)hi[a] - lo[a], ext * 1e-3 + 1e-12);
  double h = cell > 0.0 ? cell : std::cbrt(vol / (double)n);
  h = std::fmax(h, ext / maxdim + 1e-12);
  *g = PGrid{lo[0], lo[1], lo[2], (float)h, 1, 1, 1};
  int* dims[3] = {&g->dx, &g->dy, &g->dz};
  for (int a = 0; a < 3; ++a)
    *dims[a] = std::min(maxdim, (int)std::floor(((double)hi[a] - lo[a]) / h) + 1);
  return GPF_OK;
}

}  // namespace
}  // namespace gpf
