// Query binning: sort the (static) visible points by grid cell and by a Morton
// code inside the cell, then cut every cell's run into tiles of <= 64 points
// with a tight bounding box each.  Runs once per query set.
#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cmath>

#include "common.h"
#include <rocprim/device/device_scan.hpp>

#include "scan.h"

namespace gpf {
namespace {

constexpr int kRedBlocks = 256;
constexpr int kMaxDim = 1024;            // cells per axis (10-bit Morton)
constexpr int64_t kMaxDense = 1 << 26;   // dense cell table entries

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x3ff;
  x = (x | (x << 16)) & 0x030000FFull;
  x = (x | (x << 8)) & 0x0300F00Full;
  x = (x | (x << 4)) & 0x030C30C3ull;
  x = (x | (x << 2)) & 0x09249249ull;
  return x;
}

__device__ __forceinline__ uint64_t morton3(uint32_t a, uint32_t b, uint32_t c) {
  return spread3(a) | (spread3(b) << 1) | (spread3(c) << 2);
}

// min / max that keep a NaN once seen (fminf / fmaxf would drop it), so a
// non-finite point always reaches the host check of the box
__device__ __forceinline__ float min_keep_nan(float a, float b) { return (b < a || b != b) ? b : a; }
__device__ __forceinline__ float max_keep_nan(float a, float b) { return (b > a || b != b) ? b : a; }

__global__ void bbox_partial_kernel(const float* __restrict__ x, int64_t q, float* part) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < q;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float v = x[i * 3 + a];
      lo[a] = min_keep_nan(lo[a], v);
      hi[a] = max_keep_nan(hi[a], v);
    }
  }
  __shared__ float s[6][256];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    s[a][threadIdx.x] = lo[a];
    s[3 + a][threadIdx.x] = hi[a];
  }
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = min_keep_nan(s[a][threadIdx.x], s[a][threadIdx.x + st]);
        s[3 + a][threadIdx.x] = max_keep_nan(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + st]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

// One wave: lane l folds partials l, l + 64, ... (independent loads), then a
// butterfly over the wave.
__global__ void __launch_bounds__(64) bbox_final_kernel(const float* part, int nparts, float* out) {
  const int lane = threadIdx.x;
  float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int b = lane; b < nparts; b += 64) {
#pragma unroll
    for (int a = 0; a < 6; ++a)
      v[a] = a < 3 ? min_keep_nan(v[a], part[b * 6 + a]) : max_keep_nan(v[a], part[b * 6 + a]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      const float o = __shfl_xor(v[a], off, 64);
      v[a] = a < 3 ? min_keep_nan(v[a], o) : max_keep_nan(v[a], o);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < 6; ++a) out[a] = v[a];
  }
}

struct GridGeom {
  float ox, oy, oz, inv;
  int dx, dy, dz;
};

__device__ __forceinline__ void cell_of(const GridGeom& g, float x, float y, float z, int* c,
                                        float* f) {
  float p[3] = {(x - g.ox) * g.inv, (y - g.oy) * g.inv, (z - g.oz) * g.inv};
  int d[3] = {g.dx, g.dy, g.dz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int ci = (int)floorf(p[a]);
    ci = min(max(ci, 0), d[a] - 1);
    c[a] = ci;
    f[a] = fminf(fmaxf(p[a] - (float)ci, 0.f), 0.99999994f);
  }
}

__global__ void key_kernel(const float* __restrict__ x, int64_t q, GridGeom g, uint64_t* keys,
                           int* idx) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= q) return;
  int c[3];
  float f[3];
  cell_of(g, x[i * 3], x[i * 3 + 1], x[i * 3 + 2], c, f);
  uint64_t cm = morton3(c[0], c[1], c[2]);
  uint64_t sm = morton3((uint32_t)(f[0] * 1024.f), (uint32_t)(f[1] * 1024.f), (uint32_t)(f[2] * 1024.f));
  keys[i] = (cm << 30) | sm;
  idx[i] = (int)i;
}

__global__ void gather_kernel(const float* __restrict__ x, const uint64_t* __restrict__ keys,
                              const int* __restrict__ perm, int64_t q, float4* xs, int* flag) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= q) return;
  int i = perm[k];
  xs[k] = make_float4(x[(int64_t)i * 3], x[(int64_t)i * 3 + 1], x[(int64_t)i * 3 + 2], 0.f);
  flag[k] = (k == 0 || (keys[k] >> 30) != (keys[k - 1] >> 30)) ? 1 : 0;
}

// scanned[] is the exclusive scan of the run-start flags: slot of point k =
// scanned[k] for a run start.  Records the first point and dense cell of each occupied slot.
__global__ void cell_runs_kernel(const float4* __restrict__ xs, const uint64_t* __restrict__ keys,
                                 const int* __restrict__ scanned, int64_t q, GridGeom g,
                                 int* cell_first, int* occ_dense) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= q) return;
  bool start = (k == 0 || (keys[k] >> 30) != (keys[k - 1] >> 30));
  if (!start) return;
  int slot = scanned[k];
  float4 p = xs[k];
  int c[3];
  float f[3];
  cell_of(g, p.x, p.y, p.z, c, f);
  cell_first[slot] = (int)k;
  occ_dense[slot] = (c[2] * g.dy + c[1]) * g.dx + c[0];
}

__global__ void occ_table_kernel(const int* __restrict__ occ_dense, int ncells, int* occ_of_dense,
                                 uint32_t* occ_bits) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ncells) return;
  const int d = occ_dense[s];
  occ_of_dense[d] = s;
  atomicOr(occ_bits + (d >> 5), 1u << (d & 31));
}

// Tiles of kTile points and groups of kGroupTiles tiles per occupied cell,
// both from the cell's point count (so both scans run before one read-back).
__global__ void tiles_per_cell_kernel(const int* __restrict__ cell_first, int ncells, int q,
                                      int* ntile, int* ngroup) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ncells) return;
  int end = (s + 1 < ncells) ? cell_first[s + 1] : q;
  int cnt = end - cell_first[s];
  const int nt = (cnt + kTile - 1) / kTile;
  ntile[s] = nt;
  ngroup[s] = (nt + kGroupTiles - 1) / kGroupTiles;
}

// Largest s in [0, n) with off[s] <= i, for strictly increasing offsets
// (every occupied cell has at least one tile and one group).
__device__ __forceinline__ int owner_of(const int* __restrict__ off, int n, int i) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One thread per tile: tile t - toff[s] of cell s covers kTile points from
// the cell's first point on (the last one of a cell may be ragged).
__global__ void tiles_fill_kernel(const int* __restrict__ cell_first, const int* __restrict__ toff,
                                  int ncells, int ntiles, int q, TileInfo* tiles) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  const int s = owner_of(toff, ncells, t);
  const int end = (s + 1 < ncells) ? cell_first[s + 1] : q;
  TileInfo ti;
  ti.start = cell_first[s] + (t - toff[s]) * kTile;
  ti.count = min(kTile, end - ti.start);
  ti.cell = s;
  ti.pad = 0;
  tiles[t] = ti;
}

// One wave per tile: tight box of its points.
__global__ void __launch_bounds__(256) tile_box_kernel(const float4* __restrict__ xs,
                                                       const TileInfo* __restrict__ tiles,
                                                       int ntiles, float4* lo, float4* hi) {
  int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (t >= ntiles) return;
  TileInfo ti = tiles[t];
  float4 p = xs[ti.start + min(lane, ti.count - 1)];
  float l[3] = {p.x, p.y, p.z}, h[3] = {p.x, p.y, p.z};
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      l[a] = fminf(l[a], __shfl_xor(l[a], off, 64));
      h[a] = fmaxf(h[a], __shfl_xor(h[a], off, 64));
    }
  }
  if (lane == 0) {
    lo[t] = make_float4(l[0], l[1], l[2], 0.f);
    hi[t] = make_float4(h[0], h[1], h[2], 0.f);
  }
}

// One thread per group: group g - goff[s] of cell s takes the next
// kGroupTiles tiles of the cell (fewer at the cell's end).
__global__ void groups_fill_kernel(const int* __restrict__ toff, const int* __restrict__ goff,
                                   const TileInfo* __restrict__ tiles, int ncells, int ngroups,
                                   GroupInfo* groups) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroups) return;
  const int s = owner_of(goff, ncells, g);
  const int t = toff[s] + (g - goff[s]) * kGroupTiles;
  const int tl = min(t + kGroupTiles, toff[s + 1]) - 1;
  GroupInfo gi;
  gi.start = tiles[t].start;
  gi.count = tiles[tl].start + tiles[tl].count - gi.start;
  gi.cell = s;
  gi.first_tile = t;
  groups[g] = gi;
}

__global__ void group_box_kernel(const GroupInfo* __restrict__ groups, int ngroups,
                                 const float4* __restrict__ tlo, const float4* __restrict__ thi,
                                 float4* glo, float4* ghi) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroups) return;
  GroupInfo gi = groups[g];
  float4 lo = tlo[gi.first_tile], hi = thi[gi.first_tile];
  int nt = (gi.count + kTile - 1) / kTile;
  for (int t = gi.first_tile + 1; t < gi.first_tile + nt; ++t) {
    float4 a = tlo[t], b = thi[t];
    lo.x = fminf(lo.x, a.x); lo.y = fminf(lo.y, a.y); lo.z = fminf(lo.z, a.z);
    hi.x = fmaxf(hi.x, b.x); hi.y = fmaxf(hi.y, b.y); hi.z = fmaxf(hi.z, b.z);
  }
  glo[g] = lo;
  ghi[g] = hi;
}

}  // namespace

// (Re)allocates p to hold `want` bytes unless its current `cap` suffices.
template <class T>
static gpf_status grow(T*& p, size_t& cap, size_t want, const char* what) {
  if (p && cap >= want) return GPF_OK;
  dev_free((void*)p, cap);
  p = nullptr;
  cap = 0;
  void* v = nullptr;
  const gpf_status st = dev_alloc(&v, want, what);
  if (st != GPF_OK) return st;
  p = (T*)v;
  cap = want;
  return GPF_OK;
}

template <class T>
static void release(T*& p, size_t& cap) {
  dev_free((void*)p, cap);
  p = nullptr;
  cap = 0;
}

void release_bin_scratch(gpf_queries* qs) {
  release(qs->keys, qs->keys_cap);
  release(qs->keys_s, qs->keys_s_cap);
  release(qs->idx, qs->idx_cap);
  release(qs->flag, qs->flag_cap);
  release(qs->flag_s, qs->flag_s_cap);
  release(qs->cell_first, qs->cell_first_cap);
  release(qs->ntile, qs->ntile_cap);
  release(qs->cell_first_g, qs->cell_first_g_cap);
  release(qs->part, qs->part_cap);
  release(qs->tmp, qs->tmp_cap);
}

void release_bin_outputs(gpf_queries* qs) {
  release(qs->xs, qs->xs_cap);
  release(qs->perm, qs->perm_cap);
  release(qs->occ_of_dense, qs->occ_of_dense_cap);
  release(qs->occ_dense, qs->occ_dense_cap);
  release(qs->occ_bits, qs->occ_bits_cap);
  release(qs->tiles, qs->tiles_cap);
  release(qs->tile_lo, qs->tile_lo_cap);
  release(qs->tile_hi, qs->tile_hi_cap);
  release(qs->groups, qs->groups_cap);
  release(qs->group_lo, qs->group_lo_cap);
  release(qs->group_hi, qs->group_hi_cap);
}

// Bins x into `out`, reusing every buffer that is already large enough (a
// rebin of a handle allocates only when the new points need more room).  The
// scratch is released at the end unless keep_scratch.  On failure the handle
// holds no valid binning (q = 0).
gpf_status launch_bin_queries(const float* x, int64_t q, float cell, bool keep_scratch,
                              hipStream_t s, gpf_queries* out) {
  ++out->gen;  // grids built on the previous binning are stale from here on
  out->q = 0;
  out->ncells = out->ntiles = out->ngroups = 0;
  gpf_status st;
#define TRY(x)                                          \
  do {                                                  \
    gpf_status s_ = (x);                                \
    if (s_ != GPF_OK) {                                 \
      if (!keep_scratch) release_bin_scratch(out);      \
      return s_;                                        \
    }                                                   \
  } while (0)
#define TRYH(x, what)                                   \
  do {                                                  \
    hipError_t e_ = (x);                                \
    if (e_ != hipSuccess) {                             \
      if (!keep_scratch) release_bin_scratch(out);      \
      return hip_fail(e_, what);                        \
    }                                                   \
  } while (0)
  // 1. bounding box
  TRY(grow(out->part, out->part_cap, (kRedBlocks * 6 + 6) * sizeof(float), "bbox"));
  hipLaunchKernelGGL(bbox_partial_kernel, dim3(kRedBlocks), dim3(256), 0, s, x, q, out->part);
  hipLaunchKernelGGL(bbox_final_kernel, dim3(1), dim3(64), 0, s, out->part, kRedBlocks,
                     out->part + kRedBlocks * 6);
  float box[6];
  TRYH(hipMemcpyAsync(box, out->part + kRedBlocks * 6, sizeof(box), hipMemcpyDeviceToHost, s),
       "bin_queries bbox");
  TRYH(hipStreamSynchronize(s), "bin_queries bbox");
  for (int a = 0; a < 6; ++a)
    if (!std::isfinite(box[a])) TRY(set_error(GPF_ERR_INVALID_ARGUMENT, "query points contain NaN or Inf"));
  int64_t dense = 1;
  for (int a = 0; a < 3; ++a) {
    out->origin[a] = box[a];
    double ext = (double)box[3 + a] - (double)box[a];
    int64_t d = (int64_t)std::floor(ext / cell) + 1;
    if (d > kMaxDim)
      TRY(set_error(GPF_ERR_CAPACITY, "cell_size too small: more than 1024 cells per axis"));
    out->dims[a] = (int)d;
    dense *= d;
  }
  if (dense > kMaxDense) TRY(set_error(GPF_ERR_CAPACITY, "cell_size too small: more than 2^26 cells"));
  out->x_user = x;
  out->cell = cell;
  GridGeom g{out->origin[0], out->origin[1], out->origin[2], 1.f / cell, out->dims[0],
             out->dims[1], out->dims[2]};

  // 2. keys and sort
  TRY(grow(out->keys, out->keys_cap, q * 8, "keys"));
  TRY(grow(out->keys_s, out->keys_s_cap, q * 8, "keys"));
  TRY(grow(out->idx, out->idx_cap, q * 4, "idx"));
  TRY(grow(out->perm, out->perm_cap, q * 4, "perm"));
  TRY(grow(out->xs, out->xs_cap, q * sizeof(float4), "xs"));
  TRY(grow(out->flag, out->flag_cap, (q + 1) * 4, "flag"));
  TRY(grow(out->flag_s, out->flag_s_cap, (q + 1) * 4, "flag scan"));
  const int nb = (int)((q + 255) / 256);
  hipLaunchKernelGGL(key_kernel, dim3(nb), dim3(256), 0, s, x, q, g, out->keys, out->idx);
  size_t sort_bytes = 0, scan_bytes = 0;
  TRYH(rocprim::radix_sort_pairs(nullptr, sort_bytes, out->keys, out->keys_s, out->idx, out->perm,
                                 (size_t)q, 0, 60, s),
       "radix_sort size");
  TRYH(rocprim::exclusive_scan(nullptr, scan_bytes, out->flag, out->flag_s, 0, (size_t)(q + 1),
                               rocprim::plus<int>(), s),
       "scan size");
  TRY(grow(out->tmp, out->tmp_cap, std::max(sort_bytes, scan_bytes), "sort scratch"));
  TRYH(rocprim::radix_sort_pairs(out->tmp, sort_bytes, out->keys, out->keys_s, out->idx, out->perm,
                                 (size_t)q, 0, 60, s),
       "radix_sort");
  hipLaunchKernelGGL(gather_kernel, dim3(nb), dim3(256), 0, s, x, out->keys_s, out->perm, q,
                     out->xs, out->flag);
  // run starts -> occupied-cell slots: a device-wide scan over q + 1 flags
  // (flag[q] = 0, so the last entry is the number of occupied cells)
  TRYH(hipMemsetAsync(out->flag + q, 0, 4, s), "flag end");
  TRYH(rocprim::exclusive_scan(out->tmp, scan_bytes, out->flag, out->flag_s, 0, (size_t)(q + 1),
                               rocprim::plus<int>(), s),
       "scan");
  int ncells = 0;
  TRYH(hipMemcpyAsync(&ncells, out->flag_s + q, 4, hipMemcpyDeviceToHost, s), "ncells readback");
  TRYH(hipStreamSynchronize(s), "ncells sync");
  TRY(grow(out->cell_first, out->cell_first_cap, (int64_t)(ncells + 1) * 4, "cell_first"));
  TRY(grow(out->occ_dense, out->occ_dense_cap, (int64_t)ncells * 4, "occ_dense"));
  TRY(grow(out->occ_of_dense, out->occ_of_dense_cap, dense * 4, "occ_of_dense"));
  TRY(grow(out->occ_bits, out->occ_bits_cap, ((dense + 31) / 32) * 4, "occupancy bits"));
  hipLaunchKernelGGL(cell_runs_kernel, dim3(nb), dim3(256), 0, s, out->xs, out->keys_s, out->flag_s,
                     q, g, out->cell_first, out->occ_dense);
  TRYH(hipMemsetAsync(out->occ_of_dense, 0xff, dense * 4, s), "occ table clear");
  TRYH(hipMemsetAsync(out->occ_bits, 0, ((dense + 31) / 32) * 4, s), "occupancy bits clear");
  const int cb = (ncells + 255) / 256;
  hipLaunchKernelGGL(occ_table_kernel, dim3(cb), dim3(256), 0, s, out->occ_dense, ncells,
                     out->occ_of_dense, out->occ_bits);
  TRY(grow(out->ntile, out->ntile_cap, (int64_t)(ncells + 1) * 4, "ntile"));
  TRY(grow(out->cell_first_g, out->cell_first_g_cap, (int64_t)(ncells + 1) * 4, "group offsets"));
  hipLaunchKernelGGL(tiles_per_cell_kernel, dim3(cb), dim3(256), 0, s, out->cell_first, ncells,
                     (int)q, out->ntile, out->cell_first_g);
  hipLaunchKernelGGL(scan_exclusive_kernel, dim3(1), dim3(kScanThreads), 0, s, out->ntile,
                     out->ntile, ncells);
  hipLaunchKernelGGL(scan_exclusive_kernel, dim3(1), dim3(kScanThreads), 0, s, out->cell_first_g,
                     out->cell_first_g, ncells);
  int counts[2] = {0, 0};  // tiles, groups
  TRYH(hipMemcpyAsync(&counts[0], out->ntile + ncells, 4, hipMemcpyDeviceToHost, s),
       "ntiles readback");
  TRYH(hipMemcpyAsync(&counts[1], out->cell_first_g + ncells, 4, hipMemcpyDeviceToHost, s),
       "ngroups readback");
  TRYH(hipStreamSynchronize(s), "tile and group counts sync");
  const int ntiles = counts[0], ngroups = counts[1];
  TRY(grow(out->tiles, out->tiles_cap, (int64_t)ntiles * sizeof(TileInfo), "tiles"));
  TRY(grow(out->tile_lo, out->tile_lo_cap, (int64_t)ntiles * sizeof(float4), "tile_lo"));
  TRY(grow(out->tile_hi, out->tile_hi_cap, (int64_t)ntiles * sizeof(float4), "tile_hi"));
  hipLaunchKernelGGL(tiles_fill_kernel, dim3((ntiles + 255) / 256), dim3(256), 0, s,
                     out->cell_first, out->ntile, ncells, ntiles, (int)q, out->tiles);
  hipLaunchKernelGGL(tile_box_kernel, dim3((ntiles + 3) / 4), dim3(256), 0, s, out->xs, out->tiles,
                     ntiles, out->tile_lo, out->tile_hi);
  // groups of consecutive tiles per cell (ntile[] now holds the tile offsets)
  TRY(grow(out->groups, out->groups_cap, (int64_t)ngroups * sizeof(GroupInfo), "groups"));
  TRY(grow(out->group_lo, out->group_lo_cap, (int64_t)ngroups * sizeof(float4), "group_lo"));
  TRY(grow(out->group_hi, out->group_hi_cap, (int64_t)ngroups * sizeof(float4), "group_hi"));
  hipLaunchKernelGGL(groups_fill_kernel, dim3((ngroups + 255) / 256), dim3(256), 0, s, out->ntile,
                     out->cell_first_g, out->tiles, ncells, ngroups, out->groups);
  hipLaunchKernelGGL(group_box_kernel, dim3((ngroups + 255) / 256), dim3(256), 0, s, out->groups,
                     ngroups, out->tile_lo, out->tile_hi, out->group_lo, out->group_hi);
  TRYH(hipGetLastError(), "bin_queries launch");
  TRYH(hipStreamSynchronize(s), "bin_queries sync");
  if (!keep_scratch) release_bin_scratch(out);
#undef TRY
#undef TRYH
  out->q = q;
  out->ncells = ncells;
  out->ntiles = ntiles;
  out->ngroups = ngroups;
  out->bytes = out->xs_cap + out->perm_cap + out->occ_of_dense_cap + out->occ_dense_cap +
               out->occ_bits_cap + out->tiles_cap + out->tile_lo_cap + out->tile_hi_cap +
               out->groups_cap + out->group_lo_cap + out->group_hi_cap + out->keys_cap +
               out->keys_s_cap + out->idx_cap + out->flag_cap + out->flag_s_cap +
               out->cell_first_cap + out->ntile_cap + out->cell_first_g_cap + out->part_cap +
               out->tmp_cap;
  return GPF_OK;
}

}  // namespace gpf
