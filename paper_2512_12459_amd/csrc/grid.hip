// Grid build: per-primitive frame (FP64 -> FP32 record), then registration of
// every primitive in the occupied query cells its cutoff ellipsoid may touch.
#include <cmath>

#include "common.h"
#include "scan.h"

namespace gpf {
namespace {

struct Geom {
  float ox, oy, oz, h;
  int dx, dy, dz;
};

// Frame of primitive i in FP64 (Sec. 4.1): qhat = q/|q|, R(qhat) with the local
// axes as columns, s = exp(log_scale), W = diag(1/s) R^T.  Writes the FP32
// record and returns the half-extents of the cutoff ellipsoid's box; returns
// false for a degenerate primitive (zero or non-finite quaternion/scale).
__device__ bool prim_frame(const float* __restrict__ mu, const float* __restrict__ quat,
                           const float* __restrict__ ls, const float* __restrict__ rgb, int i,
                           float cutoff, PrimRec* rec, float ext[3]) {
  double qw = quat[i * 4], qx = quat[i * 4 + 1], qy = quat[i * 4 + 2], qz = quat[i * 4 + 3];
  double nrm = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  double s[3] = {exp((double)ls[i * 3]), exp((double)ls[i * 3 + 1]), exp((double)ls[i * 3 + 2])};
  bool ok = nrm > 0.0 && isfinite(nrm) && isfinite(s[0]) && isfinite(s[1]) && isfinite(s[2]) &&
            s[0] > 0.0 && s[1] > 0.0 && s[2] > 0.0;
  if (!ok) {
    PrimRec z;
    z.r0 = make_float4(mu[i * 3], mu[i * 3 + 1], mu[i * 3 + 2], 0.f);
    z.r1 = z.r2 = z.r3 = make_float4(0.f, 0.f, 0.f, 0.f);
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
  r.r3 = make_float4(W[2][0], W[2][1], W[2][2], 0.f);
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

template <bool kEmit>
__global__ void __launch_bounds__(256) register_kernel(
    const float* __restrict__ mu, const float* __restrict__ quat, const float* __restrict__ ls,
    const float* __restrict__ rgb, int n, float cutoff, Geom g, const int* __restrict__ occ_of_dense,
    PrimRec* __restrict__ recs, float4* __restrict__ exts, int* __restrict__ cell_count,
    const int* __restrict__ cell_start, int* __restrict__ cell_prims, int* __restrict__ bad) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  PrimRec r;
  float ext[3];
  if (!kEmit) {
    bool ok = prim_frame(mu, quat, ls, rgb, i, cutoff, &r, ext);
    recs[i] = r;
    exts[i] = make_float4(ext[0], ext[1], ext[2], ok ? 1.f : 0.f);
    if (!ok) {
      atomicAdd(bad, 1);
      return;
    }
  } else {
    float4 e = exts[i];
    if (e.w == 0.f) return;
    r = recs[i];
    ext[0] = e.x;
    ext[1] = e.y;
    ext[2] = e.z;
  }
  const float c2 = (float)(kKappa2 * cutoff * cutoff);
  const float inv = 1.f / g.h;
  float m[3] = {r.r0.x, r.r0.y, r.r0.z};
  float o[3] = {g.ox, g.oy, g.oz};
  int d[3] = {g.dx, g.dy, g.dz};
  int lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float a0 = (m[a] - ext[a] - o[a]) * inv;
    float a1 = (m[a] + ext[a] - o[a]) * inv;
    if (a1 < -1e-3f || a0 > (float)d[a] + 1e-3f) return;  // box misses the grid
    lo[a] = max(0, (int)floorf(a0 - 1e-3f));
    hi[a] = min(d[a] - 1, (int)floorf(a1 + 1e-3f));
  }
  const float hh = 0.5f * g.h;
  for (int cz = lo[2]; cz <= hi[2]; ++cz)
    for (int cy = lo[1]; cy <= hi[1]; ++cy)
      for (int cx = lo[0]; cx <= hi[0]; ++cx) {
        int slot = occ_of_dense[(cz * g.dy + cy) * g.dx + cx];
        if (slot < 0) continue;
        float bx = o[0] + (cx + 0.5f) * g.h, by = o[1] + (cy + 0.5f) * g.h,
              bz = o[2] + (cz + 0.5f) * g.h;
        if (!box_may_touch(r, bx, by, bz, hh, c2)) continue;
        int pos = atomicAdd(&cell_count[slot], 1);
        // the emit pass repeats the counting pass's decisions on the same
        // stored record; the bound keeps every write inside the cell's range
        if (kEmit && pos < cell_start[slot + 1] - cell_start[slot])
          cell_prims[cell_start[slot] + pos] = i;
      }
}

}  // namespace

gpf_status launch_build_grid(gpf_grid* g, hipStream_t s) {
  const gpf_queries* qs = g->qs;
  const int n = (int)g->n;
  const int nc = (int)qs->ncells;
  if (g->rec_cap < n) {
    dev_free(g->rec, g->rec_cap * sizeof(PrimRec));
    dev_free(g->ext, g->rec_cap * sizeof(float4));
    g->rec = nullptr;
    g->ext = nullptr;
    g->rec_cap = 0;
    gpf_status st = dev_alloc((void**)&g->rec, (size_t)n * sizeof(PrimRec), "grid records");
    if (st != GPF_OK) return st;
    st = dev_alloc((void**)&g->ext, (size_t)n * sizeof(float4), "grid extents");
    if (st != GPF_OK) {
      dev_free(g->rec, (size_t)n * sizeof(PrimRec));
      g->rec = nullptr;
      return st;
    }
    g->rec_cap = n;
  }
  if (!g->cell_count) {
    gpf_status st = dev_alloc((void**)&g->cell_count, (size_t)(nc + 1) * sizeof(int), "cell counts");
    if (st != GPF_OK) return st;
    st = dev_alloc((void**)&g->cell_start, (size_t)(nc + 1) * sizeof(int), "cell starts");
    if (st != GPF_OK) return st;
  }
  Geom geo{qs->origin[0], qs->origin[1], qs->origin[2], qs->cell, qs->dims[0], qs->dims[1],
           qs->dims[2]};
  // cell_count[nc] doubles as the degenerate-primitive counter during counting
  GPF_HIP(hipMemsetAsync(g->cell_count, 0, (size_t)(nc + 1) * sizeof(int), s));
  int nb = (n + 255) / 256;
  hipLaunchKernelGGL(register_kernel<false>, dim3(nb), dim3(256), 0, s, g->mu, g->quat, g->log_scale,
                     g->rgb, n, g->cutoff, geo, qs->occ_of_dense, g->rec, g->ext, g->cell_count,
                     (const int*)nullptr, (int*)nullptr, g->cell_count + nc);
  int host[2] = {0, 0};
  GPF_HIP(hipMemcpyAsync(&host[1], g->cell_count + nc, sizeof(int), hipMemcpyDeviceToHost, s));
  GPF_HIP(hipMemsetAsync(g->cell_count + nc, 0, sizeof(int), s));
  hipLaunchKernelGGL(scan_exclusive_kernel, dim3(1), dim3(kScanThreads), 0, s, g->cell_count,
                     g->cell_start, nc);
  GPF_HIP(hipMemcpyAsync(&host[0], g->cell_start + nc, sizeof(int), hipMemcpyDeviceToHost, s));
  GPF_HIP(hipStreamSynchronize(s));
  if (host[1] > 0)
    return set_error(GPF_ERR_INVALID_ARGUMENT,
                     "field has a zero-norm quaternion or a non-finite parameter");
  int64_t E = host[0];
  if (E < 0) return set_error(GPF_ERR_CAPACITY, "more than 2^31-1 cell-primitive entries");
  if (g->cap < E) {
    dev_free(g->cell_prims, g->cap * sizeof(int));
    g->cell_prims = nullptr;
    g->cap = 0;
    int64_t want = E + E / 8 + 1024;
    gpf_status st = dev_alloc((void**)&g->cell_prims, (size_t)want * sizeof(int), "cell lists");
    if (st != GPF_OK) return st;
    g->cap = want;
  }
  g->entries = E;
  GPF_HIP(hipMemsetAsync(g->cell_count, 0, (size_t)nc * sizeof(int), s));
  hipLaunchKernelGGL(register_kernel<true>, dim3(nb), dim3(256), 0, s, g->mu, g->quat, g->log_scale,
                     g->rgb, n, g->cutoff, geo, qs->occ_of_dense, g->rec, g->ext, g->cell_count,
                     g->cell_start, g->cell_prims, (int*)nullptr);
  GPF_HIP(hipGetLastError());
  g->bytes = g->rec_cap * (sizeof(PrimRec) + sizeof(float4)) + 2 * (size_t)(nc + 1) * sizeof(int) + g->cap * sizeof(int);
  return GPF_OK;
}

}  // namespace gpf
