// Photon tracing (Sec. 3.2 photon pass: photons traced from the light and
// stored at every diffuse hit) and the photon density estimate (Sec. 3
// radiance estimation; Sec. 4.3 reference equation), for the box scene with a
// glass sphere that the caustic workloads use.
//
// Scene: the box [0,1]^3 with diffuse faces floor y=0 (0), ceiling y=1 (1),
// x=0 (2), x=1 (3), back z=0 (4), the side z=1 open; a glass sphere (index
// 1.5, radius 0.2, centre (0.5, 0.5, 0.5)).  Lambertian albedos: white
// (0.73, 0.73, 0.73) for 0, 1, 4, red (0.63, 0.06, 0.05) for 2, green
// (0.14, 0.45, 0.09) for 3.  Light: a square [lo, hi]^2 of the ceiling
// emitting a cosine distribution downwards with total power (12, 10, 8).
//
// One thread per photon path; uniforms from Philox4x64-10 (Salmon et al.,
// SC'11), key (seed, 0), counter (path, event, 0, 0), each word mapped to
// (w >> 40) * 2^-24.  Event 0 emits; events 1..E intersect the sphere and the
// box (the open side ends the path): the sphere reflects when u0 < F (exact
// unpolarised Fresnel, total internal reflection F = 1) and refracts
// otherwise; a face stores (position, power, face) in slot event-1, then
// continues when u0 < q = max(albedo) with power * albedo / q and a cosine
// direction about the normal (azimuth 2 pi u1, sin^2 of the polar angle u2).
#include <rocprim/device/device_scan.hpp>

#include <algorithm>

#include "common.h"
#include "sort.h"
#include "pointgrid.h"
#include "scene.h"

namespace gpf {
namespace {

constexpr int kPhotonGridDim = 256;
// Photon cells have edge >= r / kCellRings, so a disc of radius r around a
// point lies within kCellRings cells of the point's cell along each axis.
// Halving the edge (2 rings) shrinks the candidate region a tile of points
// scans from about 3.9 to 2.4 disc areas on the walls.
constexpr int kCellRings = 2;

__global__ void __launch_bounds__(256) trace_kernel(int64_t n, uint64_t seed, int E, float lo,
                                                    float hi, int sphere, float3 power0,
                                                    float* __restrict__ pos,
                                                    float* __restrict__ pw,
                                                    int* __restrict__ surf) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  // every slot is written: unused ones hold face -1 and zero position and power
  for (int j = 0; j < E; ++j) {
    const int64_t slot = i * E + j;
    surf[slot] = -1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      pos[slot * 3 + a] = 0.f;
      pw[slot * 3 + a] = 0.f;
    }
  }
  float u[4];
  uniforms((uint64_t)i, 0, 0, seed, u);
  float o[3] = {lo + (hi - lo) * u[0], 1.f, lo + (hi - lo) * u[1]};
  const float phi = 2.f * kPi * u[2];
  const float r = sqrtf(u[3]);
  float d[3] = {r * cosf(phi), -sqrtf(1.f - u[3]), r * sinf(phi)};
  float p[3] = {power0.x, power0.y, power0.z};
  for (int j = 1; j <= E; ++j) {
    uniforms((uint64_t)i, (uint64_t)j, 0, seed, u);
    int face;
    const float tb = box_crossing(o, d, face);
    const float ts = sphere ? sphere_crossing(o, d) : INFINITY;
    const bool hit_s = ts < tb;
    if (!hit_s && (face < 0 || face == 5)) break;  // escaped through the open side
    const float t = hit_s ? ts : tb;
    const float x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
    if (hit_s) {
      float fac[3];
      sphere_scatter(d, x, u[0], sphere, fac);
      if (sphere == kSphereMirror) {
#pragma unroll
        for (int a = 0; a < 3; ++a) p[a] *= fac[a];
      }
    } else {
      const int64_t slot = i * E + (j - 1);
      pos[slot * 3] = x[0];
      pos[slot * 3 + 1] = x[1];
      pos[slot * 3 + 2] = x[2];
      pw[slot * 3] = p[0];
      pw[slot * 3 + 1] = p[1];
      pw[slot * 3 + 2] = p[2];
      surf[slot] = face;
      const float q = fmaxf(kAlbedo[face][0], fmaxf(kAlbedo[face][1], kAlbedo[face][2]));
      if (!(u[0] < q)) break;
#pragma unroll
      for (int a = 0; a < 3; ++a) p[a] = p[a] * kAlbedo[face][a] / q;
      const float ph = 2.f * kPi * u[1];
      const float sr = sqrtf(u[2]), nz = sqrtf(1.f - u[2]);
      const float ct = sr * cosf(ph), st = sr * sinf(ph);
      float nd[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) nd[a] = ct * kTangT[face][a] + st * kTangB[face][a] + nz * kNormal[face][a];
      const float inv = 1.f / sqrtf(dot3(nd, nd));
#pragma unroll
      for (int a = 0; a < 3; ++a) d[a] = nd[a] * inv;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) o[a] = x[a];
  }
}

__global__ void __launch_bounds__(256) photon_flags_kernel(const int* __restrict__ surf, int64_t m,
                                                           int* __restrict__ flags) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < m) flags[i] = surf[i] >= 0 ? 1 : 0;
  else if (i == m) flags[m] = 0;
}

__global__ void __launch_bounds__(256) photon_scatter_kernel(
    const float* __restrict__ pos, const float* __restrict__ pw, const int* __restrict__ surf,
    int64_t m, const int* __restrict__ off, float* __restrict__ opos, float* __restrict__ opw,
    int* __restrict__ osurf, int64_t* __restrict__ oslot) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= m || surf[i] < 0) return;
  const int64_t k = off[i];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    opos[k * 3 + a] = pos[i * 3 + a];
    opw[k * 3 + a] = pw[i * 3 + a];
  }
  osurf[k] = surf[i];
  if (oslot) oslot[k] = i;
}

// Photon records gathered into cell order, two float4 per photon:
// (x, y, z, face bits) and (power, 0), so that a gather reads each cell's
// photons as one contiguous run and one photon as one 32-byte load.
__global__ void __launch_bounds__(256) photon_gather_kernel(
    const int* __restrict__ sorted, int64_t np, const float* __restrict__ ppos,
    const float* __restrict__ ppw, const int* __restrict__ psurf, float4* __restrict__ rec) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= np) return;
  const int64_t j = sorted[s];
  rec[2 * s] = make_float4(ppos[j * 3], ppos[j * 3 + 1], ppos[j * 3 + 2], __int_as_float(psurf[j]));
  rec[2 * s + 1] = make_float4(ppw[j * 3], ppw[j * 3 + 1], ppw[j * 3 + 2], 0.f);
}

// Density estimate at point i on face k: sum over the photons of face k
// within r (FP32 squared distance in the fixed order), times
// weight * albedo_k / pi / (pi r^2), stored or added.  Cells have edge
// >= r / kCellRings, so the cells within kCellRings of the point's cell cover
// the disc.  Photons are visited in (cell z, cell y, cell x, photon index)
// order.
__global__ void __launch_bounds__(256) kde_kernel(const float* __restrict__ x,
                                                  const int* __restrict__ xs, int64_t q, PGrid g,
                                                  const int* __restrict__ start,
                                                  const float4* __restrict__ rec, float r2,
                                                  float scale, int accumulate,
                                                  float* __restrict__ L, int* __restrict__ count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= q) return;
  const int k = xs[i];
  float s0 = 0.f, s1 = 0.f, s2 = 0.f;
  int cnt = 0;
  if (k >= 0 && k <= 4) {
    const float px = x[i * 3], py = x[i * 3 + 1], pz = x[i * 3 + 2];
    const int3 c = pcell(g, px, py, pz);
    for (int zc = max(c.z - kCellRings, 0); zc <= min(c.z + kCellRings, g.dz - 1); ++zc)
      for (int yc = max(c.y - kCellRings, 0); yc <= min(c.y + kCellRings, g.dy - 1); ++yc) {
        // the x-neighbours of a row are adjacent cells: one contiguous run
        const int row = (zc * g.dy + yc) * g.dx;
        const int e = start[row + min(c.x + kCellRings, g.dx - 1) + 1];
        for (int s = start[row + max(c.x - kCellRings, 0)]; s < e; ++s) {
          const float4 p = rec[2 * s];
          if (__float_as_int(p.w) != k) continue;
          float d2;
          {
#pragma clang fp contract(off)
            const float dx = px - p.x, dy = py - p.y, dz = pz - p.z;
            d2 = (dx * dx + dy * dy) + dz * dz;
          }
          if (d2 <= r2) {
            const float4 w = rec[2 * s + 1];
            s0 += w.x;
            s1 += w.y;
            s2 += w.z;
            ++cnt;
          }
        }
      }
    s0 *= kAlbedo[k][0] * scale;
    s1 *= kAlbedo[k][1] * scale;
    s2 *= kAlbedo[k][2] * scale;
  }
  if (accumulate) {
    L[i * 3] += s0;
    L[i * 3 + 1] += s1;
    L[i * 3 + 2] += s2;
  } else {
    L[i * 3] = s0;
    L[i * 3 + 1] = s1;
    L[i * 3 + 2] = s2;
  }
  if (count) count[i] = cnt;
}

// The same estimate over binned points: one wave per tile of <= 64 points
// (lane = point), the photon cells covering the tile's box widened by r
// visited in the same (z, y, x, index) order, each photon read once per wave
// with wave-uniform scalar loads.  Every photon within r of a point lies in
// both this range and the point's neighbourhood in kde_kernel (photons in one
// and not the other are farther than r and add nothing), and both visit
// cells in the same global order, so every point sums the same photons in
// the same order as kde_kernel: the results are bit-identical.
constexpr int kKdeWaves = 4;

__global__ void __launch_bounds__(kKdeWaves * 64) kde_tile_kernel(
    const float4* __restrict__ xq, const int* __restrict__ perm,
    const TileInfo* __restrict__ tiles, const float4* __restrict__ tlo,
    const float4* __restrict__ thi, int ntiles, const int* __restrict__ xsurf, PGrid g,
    const int* __restrict__ start, const float4* __restrict__ rec, float reach, float r2,
    float scale, int accumulate, float* __restrict__ L, int* __restrict__ count) {
  const int lane = threadIdx.x & 63;
  // wave-uniform tile index, so that the tile's data and the photon records
  // are read with scalar loads
  const int t = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x) * kKdeWaves +
                                               (int)(threadIdx.x >> 6));
  if (t >= ntiles) return;
  const TileInfo ti = tiles[t];
  const int qi = ti.start + min(lane, ti.count - 1);
  const float4 p = xq[qi];
  const int o = perm[qi];
  const int k = xsurf[o];
  const float4 lo = tlo[t], hi = thi[t];
  const int3 c0 = pcell(g, lo.x - reach, lo.y - reach, lo.z - reach);
  const int3 c1 = pcell(g, hi.x + reach, hi.y + reach, hi.z + reach);
  float s0 = 0.f, s1 = 0.f, s2 = 0.f;
  int cnt = 0;
  auto visit = [&](const float4& ph, const float4& w) {
    float d2;
    {
#pragma clang fp contract(off)
      const float dx = p.x - ph.x, dy = p.y - ph.y, dz = p.z - ph.z;
      d2 = (dx * dx + dy * dy) + dz * dz;
    }
    const bool in = (__float_as_int(ph.w) == k) & (d2 <= r2);
    // fma(1, w, s) rounds like s + w and fma(0, w, s) = s: the same sums as a
    // branch, one instruction per channel
    const float mf = in ? 1.f : 0.f;
    s0 = fmaf(mf, w.x, s0);
    s1 = fmaf(mf, w.y, s1);
    s2 = fmaf(mf, w.z, s2);
    cnt += in ? 1 : 0;
  };
  for (int zc = c0.z; zc <= c1.z; ++zc)
    for (int yc = c0.y; yc <= c1.y; ++yc) {
      const int row = (zc * g.dy + yc) * g.dx;
      const int a = start[row + c0.x], b = start[row + c1.x + 1];
      int s = a;
      // four records per round: their scalar loads are issued together
      for (; s + 4 <= b; s += 4) {
        const float4 q0 = rec[2 * s], w0 = rec[2 * s + 1];
        const float4 q1 = rec[2 * s + 2], w1 = rec[2 * s + 3];
        const float4 q2 = rec[2 * s + 4], w2 = rec[2 * s + 5];
        const float4 q3 = rec[2 * s + 6], w3 = rec[2 * s + 7];
        visit(q0, w0);
        visit(q1, w1);
        visit(q2, w2);
        visit(q3, w3);
      }
      for (; s < b; ++s) visit(rec[2 * s], rec[2 * s + 1]);
    }
  if (lane >= ti.count) return;
  if (k >= 0 && k <= 4) {
    s0 *= kAlbedo[k][0] * scale;
    s1 *= kAlbedo[k][1] * scale;
    s2 *= kAlbedo[k][2] * scale;
  } else {
    s0 = s1 = s2 = 0.f;
    cnt = 0;
  }
  const int64_t oi = (int64_t)o * 3;
  if (accumulate) {
    L[oi] += s0;
    L[oi + 1] += s1;
    L[oi + 2] += s2;
  } else {
    L[oi] = s0;
    L[oi + 1] = s1;
    L[oi + 2] = s2;
  }
  if (count) count[o] = cnt;
}

}  // namespace

gpf_status launch_trace_photons(int64_t n, uint64_t seed, int E, float lo, float hi, int sphere,
                                float* pos, float* pw, int* surf, hipStream_t s) {
  const float3 p0 = make_float3((float)(12.0 / (double)n), (float)(10.0 / (double)n),
                                (float)(8.0 / (double)n));
  hipLaunchKernelGGL(trace_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, seed, E,
                     lo, hi, sphere, p0, pos, pw, surf);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

gpf_status compact_photons(const float* pos, const float* pw, const int* surf, int64_t m,
                           float* opos, float* opw, int* osurf, int64_t* oslot, int64_t cap,
                           int64_t* count, hipStream_t s) {
  int *flags = nullptr, *off = nullptr;
  void* tmp = nullptr;
  size_t tb = 0;
  gpf_status st;
  if ((st = dev_alloc((void**)&flags, (m + 1) * sizeof(int), "photon flags")) != GPF_OK) return st;
  if ((st = dev_alloc((void**)&off, (m + 1) * sizeof(int), "photon offsets")) != GPF_OK) {
    dev_free(flags, (m + 1) * sizeof(int));
    return st;
  }
  auto cleanup = [&]() {
    dev_free(flags, (m + 1) * sizeof(int));
    dev_free(off, (m + 1) * sizeof(int));
    dev_free(tmp, tb);
  };
  const unsigned blocks = (unsigned)((m + 256) / 256);
  hipLaunchKernelGGL(photon_flags_kernel, dim3(blocks), dim3(256), 0, s, surf, m, flags);
  hipError_t e = rocprim::exclusive_scan(nullptr, tb, flags, off, 0, (size_t)(m + 1),
                                         rocprim::plus<int>(), s);
  if (e == hipSuccess && (st = dev_alloc(&tmp, tb, "photon scan")) != GPF_OK) {
    cleanup();
    return st;
  }
  if (e == hipSuccess)
    e = rocprim::exclusive_scan(tmp, tb, flags, off, 0, (size_t)(m + 1), rocprim::plus<int>(), s);
  int total = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&total, off + m, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "photon compaction");
  }
  if (total > cap) {
    cleanup();
    return set_error(GPF_ERR_CAPACITY, "more stored photons than the output capacity");
  }
  hipLaunchKernelGGL(photon_scatter_kernel, dim3(blocks), dim3(256), 0, s, pos, pw, surf, m, off,
                     opos, opw, osurf, oslot);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  cleanup();
  if (e != hipSuccess) return hip_fail(e, "photon compaction");
  *count = total;
  return GPF_OK;
}

}  // namespace gpf

// Photon map: the stored photons gathered into the cells of a uniform grid of
// edge >= r (records in cell order), built once and gathered any number of
// times.
struct gpf_photon_map {
  gpf::PGrid g;
  int64_t np = 0, cells = 0;
  float r = 0.f;
  int* start = nullptr;      // [cells + 1] first photon of each cell in cell order
  float4* rec = nullptr;     // [2 np] (x, y, z, face bits), (power, 0) in cell order
  // scratch kept between rebuilds (grown when a larger map comes)
  int64_t np_cap = 0, cells_cap = 0;
  size_t tmp_bytes = 0;
  float* part = nullptr;     // [64 * 6] partial boxes
  unsigned* key = nullptr;   // [2 np_cap] cell keys, then sorted keys
  int* val = nullptr;        // [np_cap] photon indices
  int* sorted = nullptr;     // [np_cap] photon indices in cell order
  void* tmp = nullptr;       // radix sort scratch
};

namespace gpf {

void photon_map_free(gpf_photon_map* m) {
  if (!m) return;
  dev_free(m->start, (m->cells_cap + 1) * 4);
  dev_free(m->rec, 2 * m->np_cap * sizeof(float4));
  dev_free(m->part, kPointBoxBlocks * 6 * sizeof(float));
  dev_free(m->key, 2 * m->np_cap * 4);
  dev_free(m->val, m->np_cap * 4);
  dev_free(m->sorted, m->np_cap * 4);
  dev_free(m->tmp, m->tmp_bytes);
  delete m;
}

// Bins the photons into m, growing its buffers when needed.  On failure the
// map holds no valid photons (np = 0) but stays releasable.
gpf_status photon_map_fill(gpf_photon_map* m, const float* ppos, const float* ppw,
                           const int* psurf, int64_t np, float r, hipStream_t s) {
  m->np = 0;
  gpf_status st;
  if (!m->part &&
      (st = dev_alloc((void**)&m->part, kPointBoxBlocks * 6 * sizeof(float), "photon box")) != GPF_OK)
    return st;
  hipLaunchKernelGGL(pbox_kernel, dim3(kPointBoxBlocks), dim3(256), 0, s, ppos, np, m->part);
  float hp[kPointBoxBlocks * 6];
  GPF_HIP(hipMemcpyAsync(hp, m->part, sizeof(hp), hipMemcpyDeviceToHost, s));
  GPF_HIP(hipStreamSynchronize(s));
  PGrid g;
  if ((st = point_grid_geometry(hp, np, kPhotonGridDim, &g, (double)r * (1.0 + 1e-4) / kCellRings)) != GPF_OK)
    return st;
  const int64_t cells = (int64_t)g.dx * g.dy * g.dz;
  if (m->cells_cap < cells) {
    dev_free(m->start, (m->cells_cap + 1) * 4);
    m->start = nullptr;
    m->cells_cap = 0;
    if ((st = dev_alloc((void**)&m->start, (cells + 1) * 4, "photon cells")) != GPF_OK) return st;
    m->cells_cap = cells;
  }
  if (m->np_cap < np) {
    // with headroom: the stored-photon count varies from iteration to
    // iteration, and freeing device memory waits for the whole device
    const int64_t want = np + np / 8 + 1024;
    dev_free(m->rec, 2 * m->np_cap * sizeof(float4));
    dev_free(m->key, 2 * m->np_cap * 4);
    dev_free(m->val, m->np_cap * 4);
    dev_free(m->sorted, m->np_cap * 4);
    m->rec = nullptr;
    m->key = nullptr;
    m->val = m->sorted = nullptr;
    m->np_cap = 0;
    if ((st = dev_alloc((void**)&m->rec, 2 * want * sizeof(float4), "photon records")) != GPF_OK ||
        (st = dev_alloc((void**)&m->key, 2 * want * 4, "photon keys")) != GPF_OK ||
        (st = dev_alloc((void**)&m->val, want * 4, "photon order")) != GPF_OK ||
        (st = dev_alloc((void**)&m->sorted, want * 4, "photon order")) != GPF_OK) {
      dev_free(m->rec, 2 * want * sizeof(float4));
      dev_free(m->key, 2 * want * 4);
      dev_free(m->val, want * 4);
      m->rec = nullptr;
      m->key = nullptr;
      m->val = nullptr;
      return st;
    }
    m->np_cap = want;
  }
  // photons by cell: a stable radix sort of (cell, index), so each cell lists
  // its photons in index order and the gather's summation order does not
  // depend on scheduling; cell starts by binary search (no atomics, so the
  // crowded cells of a caustic cost nothing extra)
  const int bits = cell_key_bits(cells);
  size_t tb = 0;
  GPF_HIP(sort_pairs(nullptr, tb, m->key, m->key + np, m->val, m->sorted, (size_t)np, 0, bits, s));
  if (m->tmp_bytes < tb) {
    size_t cap_bytes = 0;   // sized for the capacity, as the arrays above
    GPF_HIP(sort_pairs(nullptr, cap_bytes, m->key, m->key + np, m->val, m->sorted,
                       (size_t)m->np_cap, 0, bits, s));
    tb = std::max(tb, cap_bytes);
    dev_free(m->tmp, m->tmp_bytes);
    m->tmp = nullptr;
    m->tmp_bytes = 0;
    if ((st = dev_alloc(&m->tmp, tb, "photon sort")) != GPF_OK) return st;
    m->tmp_bytes = tb;
  }
  const unsigned pb = (unsigned)((np + 255) / 256);
  hipLaunchKernelGGL(point_key_kernel, dim3(pb), dim3(256), 0, s, ppos, np, g, m->key, m->val);
  tb = m->tmp_bytes;
  GPF_HIP(sort_pairs(m->tmp, tb, m->key, m->key + np, m->val, m->sorted, (size_t)np, 0, bits, s));
  hipLaunchKernelGGL(sorted_cell_starts_kernel, dim3((unsigned)((cells + 256) / 256)), dim3(256), 0,
                     s, m->key + np, np, cells, m->start);
  hipLaunchKernelGGL(photon_gather_kernel, dim3(pb), dim3(256), 0, s, m->sorted, np, ppos, ppw,
                     psurf, m->rec);
  GPF_HIP(hipGetLastError());
  // the caller may release its photon arrays once this returns
  GPF_HIP(hipStreamSynchronize(s));
  m->g = g;
  m->cells = cells;
  m->r = r;
  m->np = np;
  return GPF_OK;
}

gpf_status photon_map_build(const float* ppos, const float* ppw, const int* psurf, int64_t np,
                            float r, gpf_photon_map** out, hipStream_t s) {
  auto* m = new gpf_photon_map;
  const gpf_status st = photon_map_fill(m, ppos, ppw, psurf, np, r, s);
  if (st != GPF_OK) {
    photon_map_free(m);
    return st;
  }
  *out = m;
  return GPF_OK;
}

gpf_status photon_map_gather(const gpf_photon_map* m, const float* x, const int* xs, int64_t q,
                             float weight, bool accumulate, float* L, int* count, hipStream_t s) {
  if (m->np == 0) return set_error(GPF_ERR_INVALID_ARGUMENT, "photon map holds no photons");
  const float r = m->r;
  const float r2 = r * r;
  const float scale = (float)((double)weight / (M_PI * M_PI * (double)r * (double)r));
  hipLaunchKernelGGL(kde_kernel, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, x, xs, q, m->g,
                     m->start, m->rec, r2, scale, accumulate ? 1 : 0, L, count);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

gpf_status photon_map_gather_binned(const gpf_photon_map* m, const gpf_queries* qs,
                                    const int* xs, float weight, bool accumulate, float* L,
                                    int* count, hipStream_t s) {
  if (m->np == 0) return set_error(GPF_ERR_INVALID_ARGUMENT, "photon map holds no photons");
  if (qs->ntiles == 0) return GPF_OK;
  const float r = m->r;
  const float r2 = r * r;
  // the candidate range only needs to contain the discs; widening it adds
  // candidates, never results
  const float reach = r * 1.0001f + 1e-6f;
  const float scale = (float)((double)weight / (M_PI * M_PI * (double)r * (double)r));
  const int64_t blocks = (qs->ntiles + kKdeWaves - 1) / kKdeWaves;
  hipLaunchKernelGGL(kde_tile_kernel, dim3(xcd_grid(blocks)), dim3(kKdeWaves * 64), 0, s, qs->xs,
                     qs->perm, qs->tiles, qs->tile_lo, qs->tile_hi, (int)qs->ntiles, xs, m->g,
                     m->start, m->rec, reach, r2, scale, accumulate ? 1 : 0, L, count);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

}  // namespace gpf
