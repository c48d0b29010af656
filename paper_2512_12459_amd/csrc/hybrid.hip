// Hybrid radiance query (supplementary Alg. S3; Sec. 4.2 neighbourhood
// search, weight with distance falloff and normalised aggregation) and its
// gradient.
//
// Neighbourhood of a query point x: the Gaussians whose centre lies within r
// of x (ball); when the ball holds fewer than k_min centres, the k_min
// centres nearest to x (which contain the ball).  Both decisions use FP32
// squared distances in one fixed order, (dx*dx + dy*dy) + dz*dz with
// dx = x - mu and no fused multiply-add, against r2 = fl(r*r); ties in the
// nearest order go to the lower index.  Weight w = exp(-m^2/2) psi(|x - mu|)
// with no truncation, psi = 1 within r and exp(-3 t^2), t = (dist - r) /
// max(r, 1e-6), beyond; output L = sum w Phi / max(sum w, eps).
//
// Work decomposition:
//  - the grid lists, per occupied query cell, the Gaussians whose ball may
//    reach the cell.  The ball part runs like the truncated kernels: one wave
//    per group of two tiles, forward lane = point over survivors whose
//    records are staged in LDS and read back into vector registers,
//    backward lane = Gaussian over the group's points in LDS;
//    psi = 1 inside the ball, so only the Gaussian factor varies;
//  - points whose ball holds fewer than k_min centres are finished by a
//    thread-per-point pass that searches a uniform grid over the centres in
//    rings of cells for the k_min nearest, with the falloff and its gradient.
//    Beyond D = r + 7 max(r, 1e-6) the falloff is below 2^-212, so a
//    single-precision weight is exactly zero there whatever the Gaussian: the
//    search only looks within D (cells of edge just over D/2, two rings), and
//    nearest centres beyond D, which would add exact zeros, are left out.

#include "pointgrid.h"
#include "radiance_common.h"
#include "sort.h"

namespace gpf {
namespace {

constexpr int kHWaves = 4;         // waves (groups) per workgroup
constexpr int kHListCap = 128;     // survivor slots per stack and wave (backward)
constexpr int kHRowStride = 14;    // transpose row stride (12 sums, pad, row id)
constexpr int kHGroupQ = kTile * kGroupTiles;
constexpr int kTopUpMax = 8;       // largest k_min
constexpr int kCentreDim = 256;    // centre-grid cells per axis (max)
constexpr float kLog2e = 1.4426950408889634f;

// FP32 squared distance in the fixed order (no contraction into FMA).
__device__ __forceinline__ float sq_len(float dx, float dy, float dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}

// May a point of the (padded) box lie within the ball about m?
__device__ __forceinline__ bool ball_touch(float mx, float my, float mz, const TileCtx& c,
                                           float r2pad) {
  const float ex = fmaxf(fabsf(mx - c.cx) - c.hx, 0.f);
  const float ey = fmaxf(fabsf(my - c.cy) - c.hy, 0.f);
  const float ez = fmaxf(fabsf(mz - c.cz) - c.hz, 0.f);
  return ex * ex + ey * ey + ez * ez <= r2pad;
}

// u' = W' d (whitened, kappa-scaled): exp2(-|u'|^2) = exp(-m^2 / 2).
__device__ __forceinline__ void whiten(const PrimRec& r, float dx, float dy, float dz, float u[3]) {
  u[0] = fmaf(r.r1.z, dz, fmaf(r.r1.y, dy, r.r1.x * dx));
  u[1] = fmaf(r.r2.z, dz, fmaf(r.r2.y, dy, r.r2.x * dx));
  u[2] = fmaf(r.r3.z, dz, fmaf(r.r3.y, dy, r.r3.x * dx));
}

__device__ __forceinline__ bool nearer(float da, int ia, float db, int ib) {
  return da < db || (da == db && ia < ib);
}

// ---------------------------------------------------------------------------
// Ball part, forward: per point the sums over the ball (psi = 1), the ball
// count, and L = S / max(Z, eps).  Points with fewer than k_min ball centres
// are rewritten by the top-up pass.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kHWaves * 64) hybrid_fwd_kernel(
    const float4* __restrict__ xs, const int* __restrict__ perm,
    const GroupInfo* __restrict__ groups, int ngroups, const float4* __restrict__ tlo,
    const float4* __restrict__ thi, const int* __restrict__ cell_start,
    const int* __restrict__ cell_prims, const PrimRec* __restrict__ recs, float r2, float r2pad,
    float eps, float* __restrict__ L, float* __restrict__ Zout, int* __restrict__ count,
    int* __restrict__ keep, int* __restrict__ keep_count) {
  static_assert(kGroupTiles == 2, "the forward pairs the two tiles of a group");
  __shared__ float4 stage_all[kHWaves][64 * 4];   // staged survivor records, 64 per wave
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int g = xcd_remap(blockIdx.x) * kHWaves + wave;
  if (g >= ngroups) return;
  const GroupInfo gi = groups[g];
  const TileCtx ta = tile_ctx(tlo, thi, gi.first_tile);
  const bool has_b = gi.count > kTile;
  const TileCtx tb = has_b ? tile_ctx(tlo, thi, gi.first_tile + 1) : ta;
  float px[2], py[2], pz[2], acc[2][3], z[2];
  int cnt[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float4 p = xs[gi.start + min(lane + 64 * i, gi.count - 1)];
    px[i] = p.x;
    py[i] = p.y;
    pz[i] = p.z;
    acc[i][0] = acc[i][1] = acc[i][2] = 0.f;
    z[i] = 0.f;
    cnt[i] = 0;
  }
  const int cs = cell_start[gi.cell], ce = cell_start[gi.cell + 1];
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  float4* stage = stage_all[wave];
  int kept = 0;  // survivors so far (all of them, also past the list's capacity)
  int* kl = keep ? keep + (int64_t)g * kSurvPerGroup : nullptr;
  for (int base = cs; base < ce; base += 64) {
    const int j = base + lane;
    int mask = 0, pid = 0;
    if (j < ce) {
      pid = cell_prims[j];
      const float4 m = recs[pid].r0;
      mask = (ball_touch(m.x, m.y, m.z, ta, r2pad) ? 1 : 0) |
             ((has_b && ball_touch(m.x, m.y, m.z, tb, r2pad)) ? 2 : 0);
    }
    const uint64_t bal = __ballot(mask != 0);
    const int nb = __popcll(bal);   // wave-uniform
    if (nb == 0) continue;
    if (mask) {
      // the survivor's whole record, staged with the tile mask in place of
      // the primitive index
      const int slot = __popcll(bal & below);
      const PrimRec r = recs[pid];
      stage[slot * 4 + 0] = r.r0;
      stage[slot * 4 + 1] = r.r1;
      stage[slot * 4 + 2] = r.r2;
      stage[slot * 4 + 3] = make_float4(r.r3.x, r.r3.y, r.r3.z, __int_as_float(mask));
      // keep the survivors (cell-list order) for the backward
      if (kl && kept + slot < kSurvPerGroup) kl[kept + slot] = pid | (mask << 30);
    }
    wave_sync_lds();
    for (int s = 0; s < nb; ++s) {
      // broadcast LDS loads: the record in vector registers (an instruction
      // with a scalar-register operand issues at half rate on gfx950)
      const float4 R0 = stage[s * 4], R1 = stage[s * 4 + 1], R2 = stage[s * 4 + 2],
                   R3 = stage[s * 4 + 3];
      const int tiles = __builtin_amdgcn_readfirstlane(__float_as_int(R3.w));
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (!((tiles >> i) & 1)) continue;   // wave-uniform
        const float dx = px[i] - R0.x, dy = py[i] - R0.y, dz = pz[i] - R0.z;
        const bool in = sq_len(dx, dy, dz) <= r2;
        const float u0 = fmaf(R1.z, dz, fmaf(R1.y, dy, R1.x * dx));
        const float u1 = fmaf(R2.z, dz, fmaf(R2.y, dy, R2.x * dx));
        const float u2 = fmaf(R3.z, dz, fmaf(R3.y, dy, R3.x * dx));
        const float m2 = u0 * u0 + u1 * u1 + u2 * u2;
        const float w = in ? __builtin_amdgcn_exp2f(-m2) : 0.f;
        acc[i][0] += w * R0.w;
        acc[i][1] += w * R1.w;
        acc[i][2] += w * R2.w;
        z[i] += w;
        cnt[i] += in ? 1 : 0;
      }
    }
    kept += nb;
    wave_sync_lds();   // the next batch overwrites the stage
  }
  if (!kl) kept = 0;
  if (keep_count && lane == 0) keep_count[g] = kept;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int k = lane + 64 * i;
    if (k < gi.count) {
      const int o = perm[gi.start + k];
      const float zc = fmaxf(z[i], eps);
      L[(int64_t)o * 3 + 0] = acc[i][0] / zc;
      L[(int64_t)o * 3 + 1] = acc[i][1] / zc;
      L[(int64_t)o * 3 + 2] = acc[i][2] / zc;
      Zout[o] = z[i];
      count[o] = cnt[i];
    }
  }
}

// ---------------------------------------------------------------------------
// Nearest centres (top-up): rings of centre-grid cells around the point's
// cell until the k-th best squared distance is below the distance to every
// unvisited cell, or until every cell within the reach has been visited.
// bd/bi hold the k nearest within squared distance reach2 in (d2, index)
// order; unused slots keep index 0x7fffffff.
// near[c] = some cell within `rings` cells of c (per axis) holds a centre.
__global__ void centre_near_kernel(const int* __restrict__ cstart, int dx, int dy, int dz,
                                   int rings, unsigned char* __restrict__ near) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= (int64_t)dx * dy * dz) return;
  const int x = (int)(c % dx), y = (int)((c / dx) % dy), z = (int)(c / ((int64_t)dx * dy));
  bool any = false;
  for (int zc = max(z - rings, 0); zc <= min(z + rings, dz - 1) && !any; ++zc)
    for (int yc = max(y - rings, 0); yc <= min(y + rings, dy - 1) && !any; ++yc) {
      const int row = (zc * dy + yc) * dx;
      any = cstart[row + min(x + rings, dx - 1) + 1] > cstart[row + max(x - rings, 0)];
    }
  near[c] = any ? 1 : 0;
}

// ---------------------------------------------------------------------------
template <int K>
__device__ void nearest_centres(float px, float py, float pz, const PGrid& cg,
                                const int* __restrict__ cstart, const int* __restrict__ csorted,
                                const unsigned char* __restrict__ near,
                                const PrimRec* __restrict__ recs, int k, float reach2, int max_rings,
                                float bd[K], int bi[K]) {
#pragma unroll
  for (int a = 0; a < K; ++a) {
    bd[a] = INFINITY;
    bi[a] = 0x7fffffff;
  }
  const int3 c = pcell(cg, px, py, pz);
  // no centre in any cell the rings below would visit: nothing to find
  if (!near[(c.z * cg.dy + c.y) * cg.dx + c.x]) return;
  const int maxr = min(max_rings, max(cg.dx, max(cg.dy, cg.dz)));
  // one centre: the usual insertion into the (d2, index)-ordered list
  auto visit = [&](int s) {
    const int j = csorted[s];
    const float4 m = recs[j].r0;
    const float d = sq_len(px - m.x, py - m.y, pz - m.z);
    if (d > reach2 || !nearer(d, j, bd[K - 1], bi[K - 1])) return;
    bd[K - 1] = d;
    bi[K - 1] = j;
#pragma unroll
    for (int a = K - 1; a > 0; --a) {
      if (nearer(bd[a], bi[a], bd[a - 1], bi[a - 1])) {
        const float td = bd[a];
        bd[a] = bd[a - 1];
        bd[a - 1] = td;
        const int ti = bi[a];
        bi[a] = bi[a - 1];
        bi[a - 1] = ti;
      }
    }
  };
  for (int rr = 0; rr <= maxr; ++rr) {
    // the shell of Chebyshev radius rr around c: rows of the two z faces and
    // the two y faces are whole x runs (contiguous in the cell-sorted order);
    // every other row contributes its two end cells
    const int x0 = max(c.x - rr, 0), x1 = min(c.x + rr, cg.dx - 1);
    for (int zc = max(c.z - rr, 0); zc <= min(c.z + rr, cg.dz - 1); ++zc) {
      const bool zface = abs(zc - c.z) == rr;
      for (int yc = max(c.y - rr, 0); yc <= min(c.y + rr, cg.dy - 1); ++yc) {
        const int row = (zc * cg.dy + yc) * cg.dx;
        const bool whole = zface || abs(yc - c.y) == rr;
        // at most two cell runs of this row: [a0, a1] and [b0, b1] (empty if b0 > b1)
        const int a0 = whole ? x0 : (c.x - rr >= 0 ? c.x - rr : c.x + rr);
        const int a1 = whole ? x1 : a0;
        const int b0 = whole || c.x - rr < 0 ? 1 : c.x + rr, b1 = whole || c.x - rr < 0 ? 0 : b0;
#pragma unroll 1
        for (int run = 0; run < 2; ++run) {
          const int lo = run ? b0 : a0, hi = run ? b1 : a1;
          if (lo > hi || hi >= cg.dx) continue;
#pragma unroll 1
          for (int s = cstart[row + lo], e = cstart[row + hi + 1]; s < e; ++s) visit(s);
        }
      }
    }
    // every centre outside rings 0..rr is at least rr * h away
    float kth = bd[0];
#pragma unroll
    for (int a = 1; a < K; ++a)
      if (a == k - 1) kth = bd[a];
    const float reach = (float)rr * cg.h;
    if (kth < reach * reach * (1.f - 1e-5f)) break;
  }
}

// Weight of a top-up neighbour with the falloff; returns w and writes u', t
// and dist (dist from the FP32 squared distance).
__device__ __forceinline__ float topup_weight(const PrimRec& r, float px, float py, float pz,
                                              float d2, float rb, float u[3], float* t,
                                              float* dist) {
  whiten(r, px - r.r0.x, py - r.r0.y, pz - r.r0.z, u);
  const float m2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const float dd = sqrtf(d2);
  const float tt = dd > rb ? (dd - rb) / fmaxf(rb, 1e-6f) : 0.f;
  *t = tt;
  *dist = dd;
  return __builtin_amdgcn_exp2f(-m2) * __builtin_amdgcn_exp2f(-3.f * kLog2e * tt * tt);
}

// Top-up, forward: points whose ball holds fewer than k_min centres take the
// k_min nearest instead (the ball is among them).
template <int K>
__global__ void __launch_bounds__(256) hybrid_topup_fwd_kernel(
    const float* __restrict__ x, int64_t q, PGrid cg, const int* __restrict__ cstart,
    const int* __restrict__ csorted, const unsigned char* __restrict__ cnear,
    const PrimRec* __restrict__ recs, int k_min, float rb,
    float reach2, int max_rings, float eps, float* __restrict__ L, float* __restrict__ Zout,
    const int* __restrict__ count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= q || count[i] >= k_min) return;
  const float px = x[i * 3], py = x[i * 3 + 1], pz = x[i * 3 + 2];
  float bd[K];
  int bi[K];
  nearest_centres<K>(px, py, pz, cg, cstart, csorted, cnear, recs, k_min, reach2, max_rings, bd,
                     bi);
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, z = 0.f;
#pragma unroll
  for (int a = 0; a < K; ++a) {
    if (a >= k_min || bi[a] == 0x7fffffff) continue;
    const PrimRec r = recs[bi[a]];
    float u[3], t, dist;
    const float w = topup_weight(r, px, py, pz, bd[a], rb, u, &t, &dist);
    s0 += w * r.r0.w;
    s1 += w * r.r1.w;
    s2 += w * r.r2.w;
    z += w;
  }
  const float zc = fmaxf(z, eps);
  L[i * 3] = s0 / zc;
  L[i * 3 + 1] = s1 / zc;
  L[i * 3 + 2] = s2 / zc;
  Zout[i] = z;
}

// ---------------------------------------------------------------------------
// Ball part, backward.  With Zc = max(Z, eps), gp = g / Zc and
// gl = [Z >= eps] (g . L) / Zc per point, each pair contributes
//   dPhi += w gp,  and through w (psi = 1):  c = (gp . Phi - gl) w,
// gathered as GP = sum w gp, A' = sum c u', U' = sum c u' u'^T exactly as the
// truncated backward, and mapped to parameters by the same finalize pass.
// Top-up points get gp = gl = 0 here.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void hybrid_chunk(int id, bool valid, int qb, int qe,
                                             const PrimRec* __restrict__ recs, float r2,
                                             const float4* qx, const float4* qg, float* rw,
                                             float* __restrict__ grad_rows, int lane) {
  const PrimRec r = recs[id];
  float GP[3] = {0.f, 0.f, 0.f}, A[3] = {0.f, 0.f, 0.f};
  float U[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  bool any = false;
  for (int k = qb; k < qe; k += 2) {
    float4 xq[2], gq[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      xq[i] = qx[k + i];
      gq[i] = qg[k + i];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float dx = xq[i].x - r.r0.x, dy = xq[i].y - r.r0.y, dz = xq[i].z - r.r0.z;
      const bool in = sq_len(dx, dy, dz) <= r2;
      float u[3];
      whiten(r, dx, dy, dz, u);
      const float m2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
      const float w = in ? __builtin_amdgcn_exp2f(-m2) : 0.f;
      any |= in;
      const float a = gq[i].x * r.r0.w + gq[i].y * r.r1.w + gq[i].z * r.r2.w - gq[i].w;
      const float c = a * w;
      GP[0] += w * gq[i].x;
      GP[1] += w * gq[i].y;
      GP[2] += w * gq[i].z;
      const float cu0 = c * u[0], cu1 = c * u[1], cu2 = c * u[2];
      A[0] += cu0;
      A[1] += cu1;
      A[2] += cu2;
      U[0] += cu0 * u[0];
      U[1] += cu0 * u[1];
      U[2] += cu0 * u[2];
      U[3] += cu1 * u[1];
      U[4] += cu1 * u[2];
      U[5] += cu2 * u[2];
    }
  }
  const bool write = valid && any;
  const float sums[12] = {GP[0], GP[1], GP[2], A[0], A[1], A[2], U[0], U[1], U[2], U[3], U[4], U[5]};
  const int sub = lane >> 4, e = lane & 15;
#pragma unroll
  for (int h = 0; h < 4; ++h) {   // 16 rows at a time through a small transpose buffer
    if ((lane >> 4) == h) {
      const int rl = lane & 15;
#pragma unroll
      for (int k = 0; k < 12; ++k) rw[rl * kHRowStride + k] = write ? sums[k] : 0.f;
      rw[rl * kHRowStride + 13] = __int_as_float(write ? id : -1);
    }
    wave_sync_lds();
#pragma unroll 4
    for (int rr = 0; rr < 4; ++rr) {
      const int row = rr * 4 + sub;
      const int rid = __float_as_int(rw[row * kHRowStride + 13]);
      if (e < 12 && rid >= 0) unsafeAtomicAdd(grad_rows + (int64_t)rid * 16 + e, rw[row * kHRowStride + e]);
    }
    wave_sync_lds();
  }
}

// Six waves per SIMD (at most 80 VGPRs; LDS per wave: points and their
// upstream terms 4 KB, stacks 1.5 KB, transpose rows 0.9 KB).
__global__ void __launch_bounds__(kHWaves * 64) __attribute__((amdgpu_waves_per_eu(6, 6)))
hybrid_bwd_kernel(
    const float4* __restrict__ xs, const int* __restrict__ perm,
    const GroupInfo* __restrict__ groups, int ngroups, const float4* __restrict__ tlo,
    const float4* __restrict__ thi, const int* __restrict__ cell_start,
    const int* __restrict__ cell_prims, const PrimRec* __restrict__ recs, float r2, float r2pad,
    float eps, int k_min, const float* __restrict__ Lf, const float* __restrict__ Zf,
    const int* __restrict__ count, const float* __restrict__ dL, float* __restrict__ grad_rows,
    const int* __restrict__ keep, const int* __restrict__ keep_count) {
  static_assert(kGroupTiles == 2, "the backward splits survivors over the two tiles of a group");
  __shared__ int sv_all[kHWaves][3][kHListCap];
  __shared__ float4 qx_all[kHWaves][kHGroupQ];
  __shared__ float4 qg_all[kHWaves][kHGroupQ];
  __shared__ float rows_all[kHWaves][16 * kHRowStride];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int g = xcd_remap(blockIdx.x) * kHWaves + wave;
  if (g >= ngroups) return;
  const GroupInfo gi = groups[g];
  const TileCtx ta = tile_ctx(tlo, thi, gi.first_tile);
  const bool has_b = gi.count > kTile;
  const TileCtx tb = has_b ? tile_ctx(tlo, thi, gi.first_tile + 1) : ta;
  float4* qx = qx_all[wave];
  float4* qg = qg_all[wave];
  int* sv0 = sv_all[wave][0];
  int* sv1 = sv_all[wave][1];
  int* sv2 = sv_all[wave][2];
  float* rw = rows_all[wave];
  for (int k = lane; k < kHGroupQ; k += 64) {
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f), gg = make_float4(0.f, 0.f, 0.f, 0.f);
    if (k < gi.count) {
      const int o = perm[gi.start + k];
      p = xs[gi.start + k];
      if (count[o] >= k_min) {
        const float z = Zf[o];
        const float zc = fmaxf(z, eps);
        const float g0 = dL[(int64_t)o * 3] / zc, g1 = dL[(int64_t)o * 3 + 1] / zc,
                    g2 = dL[(int64_t)o * 3 + 2] / zc;
        const float gl = z >= eps ? g0 * Lf[(int64_t)o * 3] + g1 * Lf[(int64_t)o * 3 + 1] +
                                        g2 * Lf[(int64_t)o * 3 + 2]
                                  : 0.f;
        gg = make_float4(g0, g1, g2, gl);
      }
    }
    qx[k] = p;
    qg[k] = gg;
  }
  wave_sync_lds();
  const int qe_a = (min(gi.count, kTile) + 3) & ~3, qe_all = (gi.count + 3) & ~3;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int cs = cell_start[gi.cell], ce = cell_start[gi.cell + 1];
  int n0 = 0, n1 = 0, n2 = 0;
  // the forward's survivors of this group when it kept them all (the same
  // (centre, tile mask) pairs in the same order as the cull), else the cull
  const int nk = keep_count ? keep_count[g] : kSurvPerGroup + 1;
  const bool listed = nk <= kSurvPerGroup;
  const int* kl = listed ? keep + (int64_t)g * kSurvPerGroup : nullptr;
  const int lb = listed ? 0 : cs, le = listed ? nk : ce;
  for (int base = lb; base < le; base += 64) {
    const int j = base + lane;
    int mask = 0, pid = 0;
    if (j < le) {
      if (listed) {
        const int ent = kl[j];
        pid = ent & 0x3fffffff;
        mask = (ent >> 30) & 3;
      } else {
        pid = cell_prims[j];
        const float4 m = recs[pid].r0;
        mask = (ball_touch(m.x, m.y, m.z, ta, r2pad) ? 1 : 0) |
               ((has_b && ball_touch(m.x, m.y, m.z, tb, r2pad)) ? 2 : 0);
      }
    }
    const uint64_t m0 = __ballot(mask == 1), m1 = __ballot(mask == 2), m2 = __ballot(mask == 3);
    if (mask == 1) sv0[n0 + __popcll(m0 & below)] = pid;
    if (mask == 2) sv1[n1 + __popcll(m1 & below)] = pid;
    if (mask == 3) sv2[n2 + __popcll(m2 & below)] = pid;
    n0 += __popcll(m0);
    n1 += __popcll(m1);
    n2 += __popcll(m2);
    wave_sync_lds();
    if (n0 >= 64) {
      n0 -= 64;
      hybrid_chunk(sv0[n0 + lane], true, 0, qe_a, recs, r2, qx, qg, rw, grad_rows, lane);
    }
    if (n1 >= 64) {
      n1 -= 64;
      hybrid_chunk(sv1[n1 + lane], true, kTile, qe_all, recs, r2, qx, qg, rw, grad_rows, lane);
    }
    if (n2 >= 64) {
      n2 -= 64;
      hybrid_chunk(sv2[n2 + lane], true, 0, qe_all, recs, r2, qx, qg, rw, grad_rows, lane);
    }
  }
  const int total = n0 + n1 + n2;
  for (int chunk = 0; chunk < total; chunk += 64) {
    const int v = chunk + lane;
    int id = 0, cat = 0;
    if (v < n0) {
      id = sv0[v];
      cat = 1;
    } else if (v < n0 + n2) {
      id = sv2[v - n0];
      cat = 3;
    } else if (v < total) {
      id = sv1[v - n0 - n2];
      cat = 2;
    }
    const bool use_a = __ballot(cat & 1) != 0, use_b = __ballot(cat & 2) != 0;
    hybrid_chunk(id, cat != 0, use_a ? 0 : kTile, use_b ? qe_all : qe_a, recs, r2, qx, qg, rw,
                 grad_rows, lane);
  }
}

// Top-up, backward: per top-up point and neighbour, the same sums plus the
// falloff's direct centre term, c (6 t / max(r, 1e-6)) (x - mu) / dist, in row
// slots 12..14 (per-pair atomics: top-up points are the sparse exception).
template <int K>
__global__ void __launch_bounds__(256) hybrid_topup_bwd_kernel(
    const float* __restrict__ x, int64_t q, PGrid cg, const int* __restrict__ cstart,
    const int* __restrict__ csorted, const unsigned char* __restrict__ cnear,
    const PrimRec* __restrict__ recs, int k_min, float rb,
    float reach2, int max_rings, float eps, const float* __restrict__ Lf,
    const float* __restrict__ Zf, const int* __restrict__ count, const float* __restrict__ dL,
    float* __restrict__ grad_rows) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= q || count[i] >= k_min) return;
  const float px = x[i * 3], py = x[i * 3 + 1], pz = x[i * 3 + 2];
  const float z = Zf[i];
  const float zc = fmaxf(z, eps);
  const float g0 = dL[i * 3] / zc, g1 = dL[i * 3 + 1] / zc, g2 = dL[i * 3 + 2] / zc;
  const float gl = z >= eps ? g0 * Lf[i * 3] + g1 * Lf[i * 3 + 1] + g2 * Lf[i * 3 + 2] : 0.f;
  float bd[K];
  int bi[K];
  nearest_centres<K>(px, py, pz, cg, cstart, csorted, cnear, recs, k_min, reach2, max_rings, bd,
                     bi);
  const float slope = 6.f / fmaxf(rb, 1e-6f);
#pragma unroll
  for (int a = 0; a < K; ++a) {
    if (a >= k_min || bi[a] == 0x7fffffff) continue;
    const PrimRec r = recs[bi[a]];
    float u[3], t, dist;
    const float w = topup_weight(r, px, py, pz, bd[a], rb, u, &t, &dist);
    const float c = (g0 * r.r0.w + g1 * r.r1.w + g2 * r.r2.w - gl) * w;
    float* row = grad_rows + (int64_t)bi[a] * 16;
    unsafeAtomicAdd(row + 0, w * g0);
    unsafeAtomicAdd(row + 1, w * g1);
    unsafeAtomicAdd(row + 2, w * g2);
    unsafeAtomicAdd(row + 3, c * u[0]);
    unsafeAtomicAdd(row + 4, c * u[1]);
    unsafeAtomicAdd(row + 5, c * u[2]);
    unsafeAtomicAdd(row + 6, c * u[0] * u[0]);
    unsafeAtomicAdd(row + 7, c * u[0] * u[1]);
    unsafeAtomicAdd(row + 8, c * u[0] * u[2]);
    unsafeAtomicAdd(row + 9, c * u[1] * u[1]);
    unsafeAtomicAdd(row + 10, c * u[1] * u[2]);
    unsafeAtomicAdd(row + 11, c * u[2] * u[2]);
    if (t > 0.f) {
      const float f = c * slope * t / dist;
      unsafeAtomicAdd(row + 12, f * (px - r.r0.x));
      unsafeAtomicAdd(row + 13, f * (py - r.r0.y));
      unsafeAtomicAdd(row + 14, f * (pz - r.r0.z));
    }
  }
}

// Distance beyond which a single-precision weight is exactly zero (falloff
// below 2^-212), and the rings of centre-grid cells that cover it.
double topup_reach(float rb) { return (double)rb + 7.0 * std::fmax((double)rb, 1e-6); }
// Cells have edge at least (1 + 1e-4) D / 4, so a centre within D of a point
// lies at most ceil(D / h) cells away along each axis, with room for the
// single-precision rounding of cell indices.  (A quarter of the reach keeps
// the rings that a typical top-up point scans, those within a few ball radii,
// to a few dozen centres on surface-like fields.)
int topup_rings(const gpf_grid* g) {
  return (int)std::ceil(topup_reach(g->ball) / (double)g->cg_h);
}
float topup_reach2(float rb) {
  const double d = topup_reach(rb);
  return (float)(d * d * (1.0 + 1e-6));
}

PGrid centre_geom(const gpf_grid* g) {
  return PGrid{g->cg_origin[0], g->cg_origin[1], g->cg_origin[2], g->cg_h,
               g->cg_dims[0],   g->cg_dims[1],   g->cg_dims[2]};
}

}  // namespace

void free_centre_grid(gpf_grid* g) {
  dev_free(g->cg_start, (g->cg_cells_cap + 1) * sizeof(int));
  dev_free(g->cg_key, 2 * g->cg_n_cap * sizeof(unsigned));
  dev_free(g->cg_val, g->cg_n_cap * sizeof(int));
  dev_free(g->cg_sorted, g->cg_n_cap * sizeof(int));
  dev_free(g->cg_near, g->cg_cells_cap);
  dev_free(g->cg_box, kPointBoxBlocks * 6 * sizeof(float));
  dev_free(g->cg_tmp, g->cg_tmp_bytes);
  g->cg_start = g->cg_val = g->cg_sorted = nullptr;
  g->cg_key = nullptr;
  g->cg_near = nullptr;
  g->cg_box = nullptr;
  g->cg_tmp = nullptr;
  g->cg_cells_cap = g->cg_n_cap = 0;
  g->cg_tmp_bytes = 0;
  g->cg_bytes = 0;
}

gpf_status build_centre_grid(gpf_grid* g, hipStream_t s) {
  const int64_t n = g->n;
  if (!g->cg_box) {
    gpf_status st = dev_alloc((void**)&g->cg_box, kPointBoxBlocks * 6 * sizeof(float), "centre box");
    if (st != GPF_OK) return st;
  }
  hipLaunchKernelGGL(pbox_kernel, dim3(kPointBoxBlocks), dim3(256), 0, s, g->mu, n, g->cg_box);
  float hp[kPointBoxBlocks * 6];
  GPF_HIP(hipMemcpyAsync(hp, g->cg_box, sizeof(hp), hipMemcpyDeviceToHost, s));
  GPF_HIP(hipStreamSynchronize(s));
  PGrid pg;
  gpf_status st =
      point_grid_geometry(hp, n, kCentreDim, &pg, 0.25 * (1.0 + 1e-4) * topup_reach(g->ball));
  if (st != GPF_OK) return st;
  const int64_t cells = (int64_t)pg.dx * pg.dy * pg.dz;
  if (g->cg_cells_cap < cells || g->cg_n_cap < n) {
    free_centre_grid(g);
    if ((st = dev_alloc((void**)&g->cg_box, kPointBoxBlocks * 6 * sizeof(float), "centre box")) != GPF_OK ||
        (st = dev_alloc((void**)&g->cg_start, (cells + 1) * sizeof(int), "centre cells")) != GPF_OK ||
        (st = dev_alloc((void**)&g->cg_key, 2 * n * sizeof(unsigned), "centre keys")) != GPF_OK ||
        (st = dev_alloc((void**)&g->cg_val, n * sizeof(int), "centre order")) != GPF_OK ||
        (st = dev_alloc((void**)&g->cg_sorted, n * sizeof(int), "centre order")) != GPF_OK ||
        (st = dev_alloc((void**)&g->cg_near, cells, "centre reach")) != GPF_OK)
      return st;
    g->cg_cells_cap = cells;
    g->cg_n_cap = n;
  }
  // the sort's scratch depends on n and the key width: grown when needed
  const int bits = cell_key_bits(cells);
  size_t tb = 0;
  GPF_HIP(sort_pairs(nullptr, tb, g->cg_key, g->cg_key + n, g->cg_val, g->cg_sorted, (size_t)n, 0,
                     bits, s));
  if (g->cg_tmp_bytes < tb) {
    dev_free(g->cg_tmp, g->cg_tmp_bytes);
    g->cg_tmp = nullptr;
    g->cg_tmp_bytes = 0;
    if ((st = dev_alloc(&g->cg_tmp, tb, "centre sort")) != GPF_OK) return st;
    g->cg_tmp_bytes = tb;
  }
  g->cg_origin[0] = pg.ox;
  g->cg_origin[1] = pg.oy;
  g->cg_origin[2] = pg.oz;
  g->cg_h = pg.h;
  g->cg_dims[0] = pg.dx;
  g->cg_dims[1] = pg.dy;
  g->cg_dims[2] = pg.dz;
  // centres by cell: a stable radix sort of (cell, index), then the cell
  // starts by binary search (no atomics, so crowded cells cost nothing extra)
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(point_key_kernel, dim3(blocks), dim3(256), 0, s, g->mu, n, pg, g->cg_key,
                     g->cg_val);
  tb = g->cg_tmp_bytes;
  GPF_HIP(sort_pairs(g->cg_tmp, tb, g->cg_key, g->cg_key + n, g->cg_val, g->cg_sorted, (size_t)n, 0,
                     bits, s));
  hipLaunchKernelGGL(sorted_cell_starts_kernel, dim3((unsigned)((cells + 256) / 256)), dim3(256), 0,
                     s, g->cg_key + n, n, cells, g->cg_start);
  hipLaunchKernelGGL(centre_near_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s,
                     g->cg_start, pg.dx, pg.dy, pg.dz, topup_rings(g), g->cg_near);
  GPF_HIP(hipGetLastError());
  g->cg_bytes = ((g->cg_cells_cap + 1) + 4 * g->cg_n_cap + kPointBoxBlocks * 6) * sizeof(int) +
                g->cg_cells_cap + g->cg_tmp_bytes;
  return GPF_OK;
}

gpf_status launch_hybrid_fwd(const gpf_grid* gc, float eps, float* L, float* Z, int* count,
                             hipStream_t s) {
  gpf_grid* g = const_cast<gpf_grid*>(gc);  // the survivor lists live in the handle
  const gpf_queries* qs = g->qs;
  ensure_survivor_lists(g);
  const float r2 = g->ball * g->ball;
  const float r2pad = r2 * 1.001f + 1e-10f;
  hipLaunchKernelGGL(hybrid_fwd_kernel, dim3(xcd_grid((qs->ngroups + kHWaves - 1) / kHWaves)),
                     dim3(kHWaves * 64), 0, s, qs->xs, qs->perm, qs->groups, (int)qs->ngroups,
                     qs->tile_lo, qs->tile_hi, g->cell_start, g->cell_prims, g->rec, r2, r2pad,
                     eps, L, Z, count, g->surv, g->surv ? g->surv_count : nullptr);
  const unsigned blocks = (unsigned)((qs->q + 255) / 256);
  // the nearest-centre list only needs k_min slots: 4 covers k_min <= 4
  auto topup = g->k_min <= 4 ? hybrid_topup_fwd_kernel<4> : hybrid_topup_fwd_kernel<kTopUpMax>;
  hipLaunchKernelGGL(topup, dim3(blocks), dim3(256), 0, s, qs->x_user, qs->q, centre_geom(g),
                     g->cg_start, g->cg_sorted, g->cg_near, g->rec, g->k_min, g->ball,
                     topup_reach2(g->ball), topup_rings(g), eps, L, Z, count);
  GPF_HIP(hipGetLastError());
  g->surv_ready = g->surv != nullptr;
  return GPF_OK;
}

gpf_status launch_hybrid_bwd(const gpf_grid* gc, float eps, const float* L, const float* Z,
                             const int* count, const float* dL, gpf_field_grad* grad,
                             hipStream_t s) {
  gpf_grid* g = const_cast<gpf_grid*>(gc);  // scratch rows live in the handle
  const gpf_queries* qs = g->qs;
  gpf_status st = ensure_grad_rows(g, s);
  if (st != GPF_OK) return st;
  const float r2 = g->ball * g->ball;
  const float r2pad = r2 * 1.001f + 1e-10f;
  hipLaunchKernelGGL(hybrid_bwd_kernel, dim3(xcd_grid((qs->ngroups + kHWaves - 1) / kHWaves)),
                     dim3(kHWaves * 64), 0, s, qs->xs, qs->perm, qs->groups, (int)qs->ngroups,
                     qs->tile_lo, qs->tile_hi, g->cell_start, g->cell_prims, g->rec, r2, r2pad,
                     eps, g->k_min, L, Z, count, dL, (float*)g->grad_rows,
                     g->surv_ready ? g->surv : nullptr, g->surv_ready ? g->surv_count : nullptr);
  const unsigned blocks = (unsigned)((qs->q + 255) / 256);
  auto topup = g->k_min <= 4 ? hybrid_topup_bwd_kernel<4> : hybrid_topup_bwd_kernel<kTopUpMax>;
  hipLaunchKernelGGL(topup, dim3(blocks), dim3(256), 0, s, qs->x_user, qs->q, centre_geom(g),
                     g->cg_start, g->cg_sorted, g->cg_near, g->rec, g->k_min, g->ball,
                     topup_reach2(g->ball), topup_rings(g), eps, L, Z, count, dL,
                     (float*)g->grad_rows);
  GPF_HIP(hipGetLastError());
  return launch_grad_finalize(g, g->grad_rows, grad, s);
}

}  // namespace gpf
