// Grid build: per-primitive frame (FP64 -> FP32 record), then registration of
// every primitive in the occupied query cells its cutoff ellipsoid may touch:
// count per primitive -> scan -> emit (cell, primitive) entries in primitive
// order -> stable radix sort by cell, so each cell lists its primitives in
// ascending index order (deterministic sums downstream).
#include <rocprim/device/device_scan.hpp>

#include <algorithm>
#include <cmath>

#include "common.h"
#include "sort.h"

namespace gpf {
namespace {

struct Geom {
  float ox, oy, oz, h;
  int dx, dy, dz;
};

// Threads per primitive in the count and emit passes: a cutoff box spans
// tens to hundreds of query cells, so one thread each leaves the launch
// latency-bound when n is a few hundred thousand.  Eight for cutoff boxes; for
// the hybrid query's ball boxes (whose cell span is known) about 16 cells per
// thread; fewer beyond 2^24 primitives so that the counts stay under 2^27.
int sub_threads(int64_t n, float ball, float cell) {
  int S = 8;
  if (ball > 0.f) {
    const double span = 2.0 * ball / cell + 2.0;  // cells per axis, at most
    S = 1;
    while (S < 8 && span * span * span >= 32.0 * S) S <<= 1;
  }
  while (S > 1 && n * S > ((int64_t)1 << 27) && n > ((int64_t)1 << 24)) S >>= 1;
  return S;
}

// Frame of primitive i in FP64 (Sec. 4.1): qhat = q/|q|, R(qhat) with the local
// axes as columns, s = exp(log_scale), W = diag(1/s) R^T.  Writes the FP32
// record and returns the half-extents of the cutoff ellipsoid's box; returns
// false for a degenerate primitive (zero or non-finite quaternion, non-finite
// scale, position or flux).
__device__ bool prim_frame(const float* __restrict__ mu, const float* __restrict__ quat,
                           const float* __restrict__ ls, const float* __restrict__ rgb, int i,
                           float cutoff, PrimRec* rec, float ext[3]) {
  double qw = quat[i * 4], qx = quat[i * 4 + 1], qy = quat[i * 4 + 2], qz = quat[i * 4 + 3];
  double nrm = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  double s[3] = {exp((double)ls[i * 3]), exp((double)ls[i * 3 + 1]), exp((double)ls[i * 3 + 2])};
  bool ok = nrm > 0.0 && isfinite(nrm) && isfinite(s[0]) && isfinite(s[1]) && isfinite(s[2]) &&
            s[0] > 0.0 && s[1] > 0.0 && s[2] > 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) ok = ok && isfinite(mu[i * 3 + a]) && isfinite(rgb[i * 3 + a]);
  if (!ok) {
    PrimRec z;
    z.r0 = make_float4(mu[i * 3], mu[i * 3 + 1], mu[i * 3 + 2], 0.f);
    z.r1 = z.r2 = make_float4(0.f, 0.f, 0.f, 0.f);
    z.r3 = make_float4(0.f, 0.f, 0.f, __int_as_float(i));
    *rec = z;
    return false;
  }
  qw /= nrm; qx /= nrm; qy /= nrm; qz /= nrm;
  double R[3][3];
  R[0][0] = 1 - 2 * (qy * qy + qz * qz);
  R[0][1] = 2 * (qx * qy - qw * qz);
  R[0][2] = 2 * (qx * qz + qw * qy);
  R[1][0] = 2 * (qx * qy + qw * qz);
  R[1][1] = 1 - 2 * (qx * qx + qz * qz);
  R[1][2] = 2 * (qy * qz - qw * qx);
  R[2][0] = 2 * (qx * qz - qw * qy);
  R[2][1] = 2 * (qy * qz + qw * qx);
  R[2][2] = 1 - 2 * (qx * qx + qy * qy);
  const double kap = sqrt(kKappa2);
  float W[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 3; ++j) W[k][j] = (float)(kap * R[j][k] / s[k]);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    double e2 = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) e2 += R[j][k] * R[j][k] * s[k] * s[k];
    ext[j] = (float)(cutoff * sqrt(e2) * (1.0 + 1e-5));
  }
  PrimRec r;
  r.r0 = make_float4(mu[i * 3], mu[i * 3 + 1], mu[i * 3 + 2], rgb[i * 3]);
  r.r1 = make_float4(W[0][0], W[0][1], W[0][2], rgb[i * 3 + 1]);
  r.r2 = make_float4(W[1][0], W[1][1], W[1][2], rgb[i * 3 + 2]);
  r.r3 = make_float4(W[2][0], W[2][1], W[2][2], __int_as_float(i));
  *rec = r;
  return true;
}

// Conservative test: may the ellipsoid {|W'(x-mu)|^2 <= c2} meet the box with
// centre b and half-edge hh?  Per whitened axis k, |u_k(x)| >= |u_k(b)| - r_k
// with r_k = hh * sum_j |W'_kj|; a sum of squared lower bounds above c2 rules
// the box out.  Slack keeps FP32 rounding on the safe side.
__device__ __forceinline__ bool box_may_touch(const PrimRec& r, float bx, float by, float bz,
                                              float hh, float c2) {
  float dx = bx - r.r0.x, dy = by - r.r0.y, dz = bz - r.r0.z;
  float4 w[3] = {r.r1, r.r2, r.r3};
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float u = w[k].x * dx + w[k].y * dy + w[k].z * dz;
    float rad = hh * (fabsf(w[k].x) + fabsf(w[k].y) + fabsf(w[k].z)) * 1.001f + 1e-4f;
    float lb = fmaxf(fabsf(u) - rad, 0.f);
    acc += lb * lb;
  }
  return acc <= c2 * 1.001f;
}

// Conservative test: may a point within distance `ball` of the centre lie in
// the box with centre b and half-edge hh?  (Hybrid query: ball query of
// radius r about each query point, Sec. 4.2 neighbourhood search.)
__device__ __forceinline__ bool ball_may_touch(const PrimRec& r, float bx, float by, float bz,
                                               float hh, float ball) {
  const float ex = fmaxf(fabsf(bx - r.r0.x) - hh, 0.f);
  const float ey = fmaxf(fabsf(by - r.r0.y) - hh, 0.f);
  const float ez = fmaxf(fabsf(bz - r.r0.z) - hh, 0.f);
  return ex * ex + ey * ey + ez * ez <= ball * ball * 1.001f + 1e-10f;
}

// Visits the occupied cells of the primitive's cutoff box (or, with ball > 0,
// of the box of its ball) that pass the whitened-frame (or ball) test; counts
// them, or (kEmit) writes (cell slot, primitive) entries from `base` on.  The
// box is taken row by row (one row = the cells of one (y, z) along x; rows in
// (z, y) order), sub-thread `sub` of S taking rows sub, sub + S, ...; within a
// row the occupancy bits are read 32 cells at a time and only occupied cells
// are tested, in ascending x.  Count and emit read the same stored record and
// extents with the same split, so they make identical decisions.
template <bool kEmit>
__device__ __forceinline__ int visit_cells(const PrimRec& r, const float ext[3], const Geom& g,
                                           const uint32_t* __restrict__ bits,
                                           const int* __restrict__ occ_of_dense, float c2,
                                           float ball, int pid, int sub, int S, int* __restrict__ keys,
                                           int* __restrict__ vals, int base, int limit) {
  const float inv = 1.f / g.h;
  const float m[3] = {r.r0.x, r.r0.y, r.r0.z};
  const float o[3] = {g.ox, g.oy, g.oz};
  const int d[3] = {g.dx, g.dy, g.dz};
  int lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float a0 = (m[a] - ext[a] - o[a]) * inv;
    const float a1 = (m[a] + ext[a] - o[a]) * inv;
    if (a1 < -1e-3f || a0 > (float)d[a] + 1e-3f) return 0;  // box misses the grid
    lo[a] = max(0, (int)floorf(a0 - 1e-3f));
    hi[a] = min(d[a] - 1, (int)floorf(a1 + 1e-3f));
    if (!(lo[a] <= hi[a])) return 0;   // a box starting on the grid's far face
  }
  const int ny = hi[1] - lo[1] + 1, rows = ny * (hi[2] - lo[2] + 1);
  const float hh = 0.5f * g.h;
  int cnt = 0;
  for (int row = sub; row < rows; row += S) {
    const int cy = lo[1] + row % ny, cz = lo[2] + row / ny;
    const int row0 = (cz * g.dy + cy) * g.dx;          // dense index of x = 0
    const int first = row0 + lo[0], last = row0 + hi[0];
    const float by = o[1] + (cy + 0.5f) * g.h, bz = o[2] + (cz + 0.5f) * g.h;
    for (int w = first >> 5; w <= (last >> 5); ++w) {
      const int w0 = w << 5;
      uint32_t word = bits[w];
      if (first > w0) word &= ~0u << (first - w0);          // shift in [1, 31]
      if (last < w0 + 31) word &= ~0u >> (w0 + 31 - last);  // shift in [1, 31]
      while (word) {
        const int dc = w0 + __builtin_ctz(word);
        word &= word - 1;
        const float bx = o[0] + (dc - row0 + 0.5f) * g.h;
        const bool touch = ball > 0.f ? ball_may_touch(r, bx, by, bz, hh, ball)
                                      : box_may_touch(r, bx, by, bz, hh, c2);
        if (touch) {
          if (kEmit && cnt < limit) {
            keys[base + cnt] = occ_of_dense[dc];
            vals[base + cnt] = pid;
          }
          ++cnt;
        }
      }
    }
  }
  return cnt;
}

// Pass 1: frame of every primitive (FP64 -> FP32 record, cutoff box);
// `bad` counts degenerate primitives.
__global__ void __launch_bounds__(256) frame_kernel(
    const float* __restrict__ mu, const float* __restrict__ quat, const float* __restrict__ ls,
    const float* __restrict__ rgb, int n, float cutoff, float ball, PrimRec* __restrict__ recs,
    float4* __restrict__ exts, int* __restrict__ bad, int* __restrict__ scan_pad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *scan_pad = 0;   // the count past the last one, so the scan yields the total
  if (i >= n) return;
  PrimRec r;
  float ext[3];
  const bool ok = prim_frame(mu, quat, ls, rgb, i, cutoff, &r, ext);
  if (ball > 0.f) ext[0] = ext[1] = ext[2] = ball * (1.f + 1e-5f);
  recs[i] = r;
  exts[i] = make_float4(ext[0], ext[1], ext[2], ok ? 1.f : 0.f);
  if (!ok) atomicAdd(bad, 1);
}

// Pass 2: per (primitive, sub-thread) the number of cells it registers in.
__global__ void __launch_bounds__(256) count_kernel(int n, int S, float cutoff, float ball, Geom g,
                                                    const uint32_t* __restrict__ bits,
                                                    const int* __restrict__ occ_of_dense,
                                                    const PrimRec* __restrict__ recs,
                                                    const float4* __restrict__ exts,
                                                    int* __restrict__ cnt) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * S) return;
  const int i = (int)(t / S), sub = (int)(t % S);
  const float4 e = exts[i];
  if (e.w == 0.f) {
    cnt[t] = 0;
    return;
  }
  const float ext[3] = {e.x, e.y, e.z};
  const float c2 = (float)(kKappa2 * cutoff * cutoff);
  cnt[t] = visit_cells<false>(recs[i], ext, g, bits, occ_of_dense, c2, ball, i, sub, S,
                              nullptr, nullptr, 0, 0);
}

// Pass 3: entries at the scanned offsets, primitive-major (and sub-thread
// order within a primitive).
__global__ void __launch_bounds__(256) emit_kernel(int n, int S, float cutoff, float ball, Geom g,
                                                   const uint32_t* __restrict__ bits,
                                                   const int* __restrict__ occ_of_dense,
                                                   const PrimRec* __restrict__ recs,
                                                   const float4* __restrict__ exts,
                                                   const int* __restrict__ off,
                                                   int* __restrict__ keys, int* __restrict__ vals) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * S) return;
  const int i = (int)(t / S), sub = (int)(t % S);
  const float4 e = exts[i];
  if (e.w == 0.f) return;
  const float ext[3] = {e.x, e.y, e.z};
  const float c2 = (float)(kKappa2 * cutoff * cutoff);
  const int base = off[t];
  // never write past this sub-thread's range, whatever the visit decides
  visit_cells<true>(recs[i], ext, g, bits, occ_of_dense, c2, ball, i, sub, S, keys, vals, base,
                    off[t + 1] - base);
}

// Records in cell-list order (entry e holds the record of cell_prims[e]), so
// that a cull reads a cell's candidates as one contiguous block.
__global__ void __launch_bounds__(256) gather_recs_kernel(const int* __restrict__ cell_prims,
                                                          const PrimRec* __restrict__ recs,
                                                          PrimRec* __restrict__ cell_recs, int E) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < E) cell_recs[e] = recs[cell_prims[e]];
}

// cell_start[c] = first sorted entry with key >= c (binary search).
__global__ void cell_start_kernel(const int* __restrict__ keys, int E, int ncells,
                                  int* __restrict__ cell_start) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > ncells) return;
  int lo = 0, hi = E;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (keys[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  cell_start[c] = lo;
}

}  // namespace

gpf_status launch_build_grid(gpf_grid* g, hipStream_t s) {
  g->surv_ready = false;  // the forward's survivor lists belong to the previous build
  const gpf_queries* qs = g->qs;
  const int n = (int)g->n;
  const int nc = (int)qs->ncells;
  const int S = sub_threads(n, g->ball, qs->cell);
  const int64_t m = (int64_t)n * S;  // (primitive, sub-thread) pairs
  if (g->rec_cap < n) {
    dev_free(g->rec, g->rec_cap * sizeof(PrimRec));
    dev_free(g->ext, g->rec_cap * sizeof(float4));
    g->rec = nullptr;
    g->ext = nullptr;
    g->rec_cap = 0;
    gpf_status st;
    if ((st = dev_alloc((void**)&g->rec, (size_t)n * sizeof(PrimRec), "grid records")) != GPF_OK ||
        (st = dev_alloc((void**)&g->ext, (size_t)n * sizeof(float4), "grid extents")) != GPF_OK) {
      dev_free(g->rec, (size_t)n * sizeof(PrimRec));
      g->rec = nullptr;
      return st;
    }
    g->rec_cap = n;
  }
  if (g->prim_off_len < 2 * m + 3) {
    dev_free(g->prim_off, (size_t)g->prim_off_len * sizeof(int));
    g->prim_off = nullptr;
    g->prim_off_len = 0;
    gpf_status st =
        dev_alloc((void**)&g->prim_off, (size_t)(2 * m + 3) * sizeof(int), "grid counts");
    if (st != GPF_OK) return st;
    g->prim_off_len = 2 * m + 3;
  }
  if (g->cell_start_cap < nc + 1) {  // the query set may have been re-binned into more cells
    dev_free(g->cell_start, g->cell_start_cap * sizeof(int));
    g->cell_start = nullptr;
    g->cell_start_cap = 0;
    gpf_status st = dev_alloc((void**)&g->cell_start, (size_t)(nc + 1) * sizeof(int), "cell starts");
    if (st != GPF_OK) return st;
    g->cell_start_cap = nc + 1;
  }
  Geom geo{qs->origin[0], qs->origin[1], qs->origin[2], qs->cell, qs->dims[0], qs->dims[1],
           qs->dims[2]};
  const int nb = (n + 255) / 256;
  const unsigned mb = (unsigned)((m + 255) / 256);
  // counts: prim_off[0 .. m] (entry m is 0); offsets: prim_off[m + 1 .. 2m + 1]
  // (the total last); degenerate counter at 2m + 2, next to the total, so
  // that one copy reads both back
  int* cnt = g->prim_off;
  int* off = g->prim_off + m + 1;
  int* bad = off + m + 1;
  GPF_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
  hipLaunchKernelGGL(frame_kernel, dim3(nb), dim3(256), 0, s, g->mu, g->quat, g->log_scale, g->rgb,
                     n, g->cutoff, g->ball, g->rec, g->ext, bad, cnt + m);
  hipLaunchKernelGGL(count_kernel, dim3(mb), dim3(256), 0, s, n, S, g->cutoff, g->ball, geo,
                     qs->occ_bits, qs->occ_of_dense, g->rec, g->ext, cnt);
  size_t scan_bytes = 0;
  GPF_HIP(rocprim::exclusive_scan(nullptr, scan_bytes, cnt, off, 0, (size_t)(m + 1),
                                  rocprim::plus<int>(), s));
  if (g->sort_tmp_bytes < scan_bytes) {
    dev_free(g->sort_tmp, g->sort_tmp_bytes);
    g->sort_tmp = nullptr;
    g->sort_tmp_bytes = 0;
    gpf_status st = dev_alloc(&g->sort_tmp, scan_bytes, "scan scratch");
    if (st != GPF_OK) return st;
    g->sort_tmp_bytes = scan_bytes;
  }
  if (!g->readback) {   // pinned, so that the copy below is one asynchronous transfer
    void* p = nullptr;
    const hipError_t e = hipHostMalloc(&p, 2 * sizeof(int), hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "hipHostMalloc(read-back)");
    g->readback = static_cast<int*>(p);
  }
  size_t tb = g->sort_tmp_bytes;
  GPF_HIP(rocprim::exclusive_scan(g->sort_tmp, tb, cnt, off, 0, (size_t)(m + 1),
                                  rocprim::plus<int>(), s));
  GPF_HIP(hipMemcpyAsync(g->readback, off + m, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  GPF_HIP(hipStreamSynchronize(s));
  const int host[2] = {g->readback[0], g->readback[1]};   // total entries, degenerate primitives
  if (host[1] > 0)
    return set_error(GPF_ERR_INVALID_ARGUMENT,
                     "field has a zero-norm quaternion or a non-finite parameter");
  const int64_t E = host[0];
  if (E < 0) return set_error(GPF_ERR_CAPACITY, "more than 2^31-1 cell-primitive entries");
  // the truncated query's survivor lists carry an entry index and a 2-bit tile mask
  if (!(g->ball > 0.f) && E >= ((int64_t)1 << 30))
    return set_error(GPF_ERR_CAPACITY, "more than 2^30-1 cell-primitive entries");
  if (g->cap < E) {
    int** bufs[4] = {&g->keys, &g->vals, &g->keys_sorted, &g->cell_prims};
    for (auto b : bufs) {
      dev_free(*b, g->cap * sizeof(int));
      *b = nullptr;
    }
    g->cap = 0;
    const int64_t want = E + E / 8 + 1024;
    for (auto b : bufs) {
      gpf_status st = dev_alloc((void**)b, (size_t)want * sizeof(int), "cell lists");
      if (st != GPF_OK) return st;
    }
    g->cap = want;
  }
  g->entries = E;
  hipLaunchKernelGGL(emit_kernel, dim3(mb), dim3(256), 0, s, n, S, g->cutoff, g->ball, geo,
                     qs->occ_bits, qs->occ_of_dense, g->rec, g->ext, off, g->keys, g->vals);
  // stable sort by cell slot: each cell's primitives end up in ascending order
  int bits_needed = 1;
  while ((1 << bits_needed) <= nc) ++bits_needed;
  size_t sort_bytes = 0;
  GPF_HIP(sort_pairs(nullptr, sort_bytes, g->keys, g->keys_sorted, g->vals, g->cell_prims,
                     (size_t)E, 0, bits_needed, s));
  if (g->sort_tmp_bytes < sort_bytes) {
    // sized for the lists' capacity, so that builds with more entries (up to
    // g->cap) reuse it: freeing device memory waits for the whole device
    size_t cap_bytes = 0;
    GPF_HIP(sort_pairs(nullptr, cap_bytes, g->keys, g->keys_sorted, g->vals, g->cell_prims,
                       (size_t)g->cap, 0, bits_needed, s));
    sort_bytes = std::max(sort_bytes, cap_bytes);
    dev_free(g->sort_tmp, g->sort_tmp_bytes);
    g->sort_tmp = nullptr;
    g->sort_tmp_bytes = 0;
    gpf_status st = dev_alloc(&g->sort_tmp, sort_bytes, "sort scratch");
    if (st != GPF_OK) return st;
    g->sort_tmp_bytes = sort_bytes;
  }
  sort_bytes = g->sort_tmp_bytes;
  GPF_HIP(sort_pairs(g->sort_tmp, sort_bytes, g->keys, g->keys_sorted, g->vals, g->cell_prims,
                     (size_t)E, 0, bits_needed, s));
  hipLaunchKernelGGL(cell_start_kernel, dim3((nc + 256) / 256), dim3(256), 0, s, g->keys_sorted,
                     (int)E, nc, g->cell_start);
  GPF_HIP(hipGetLastError());
  if (!(g->ball > 0.f)) {
    if (g->cell_recs_cap < E) {
      dev_free(g->cell_recs, g->cell_recs_cap * sizeof(PrimRec));
      g->cell_recs = nullptr;
      g->cell_recs_cap = 0;
      gpf_status st = dev_alloc((void**)&g->cell_recs, (size_t)g->cap * sizeof(PrimRec),
                                "cell-ordered records");
      if (st != GPF_OK) return st;
      g->cell_recs_cap = g->cap;
    }
    if (E > 0)
      hipLaunchKernelGGL(gather_recs_kernel, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, s,
                         g->cell_prims, g->rec, g->cell_recs, (int)E);
    GPF_HIP(hipGetLastError());
  }
  g->bytes = g->rec_cap * (sizeof(PrimRec) + sizeof(float4)) + g->prim_off_len * sizeof(int) +
             (size_t)g->cell_start_cap * sizeof(int) + 4 * g->cap * sizeof(int) + g->sort_tmp_bytes +
             g->cell_recs_cap * sizeof(PrimRec);
  if (g->ball > 0.f) {
    gpf_status st = build_centre_grid(g, s);
    if (st != GPF_OK) return st;
    g->bytes += g->cg_bytes;
  }
  return GPF_OK;
}

}  // namespace gpf
