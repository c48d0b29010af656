// Radiance query (forward), its gradient (backward) and the exact pair count.
//
// Work decomposition: one wave64 per query tile (<= 64 sorted points in one
// occupied grid cell).  The wave first culls its cell's primitive list
// against the tile's tight box with the whitened-frame separating test and
// compacts the survivors into a per-wave LDS list; then
//  - forward:  lane = query, loop over survivors (their records are read with
//              wave-uniform scalar loads), accumulate L in registers;
//  - backward: lane = survivor, loop over the tile's queries (broadcast from
//              LDS), accumulate the 18 per-primitive sums in registers, map
//              them to parameter gradients and add them with atomics.
// Weights are recomputed in the backward; nothing per pair is stored.
#include "common.h"

namespace gpf {
namespace {

constexpr int kWaves = 4;        // waves (tiles) per workgroup
constexpr int kSurvCap = 512;    // survivor slots per wave

struct TileCtx {
  float cx, cy, cz;   // tile box centre
  float hx, hy, hz;   // tile box half-extent (padded)
};

__device__ __forceinline__ TileCtx tile_ctx(const float4* __restrict__ tlo,
                                            const float4* __restrict__ thi, int t) {
  float4 lo = tlo[t], hi = thi[t];
  TileCtx c;
  c.cx = 0.5f * (lo.x + hi.x);
  c.cy = 0.5f * (lo.y + hi.y);
  c.cz = 0.5f * (lo.z + hi.z);
  c.hx = 0.5f * (hi.x - lo.x) * 1.0001f + 1e-7f;
  c.hy = 0.5f * (hi.y - lo.y) * 1.0001f + 1e-7f;
  c.hz = 0.5f * (hi.z - lo.z) * 1.0001f + 1e-7f;
  return c;
}

// May the primitive's cutoff ellipsoid reach any point of the tile box?
// Lower bound of |u'_k| over the box is |u'_k(centre)| - sum_j |W'_kj| h_j.
__device__ __forceinline__ bool tile_may_touch(const PrimRec& r, const TileCtx& c, float c2) {
  float dx = c.cx - r.r0.x, dy = c.cy - r.r0.y, dz = c.cz - r.r0.z;
  float4 w[3] = {r.r1, r.r2, r.r3};
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float u = w[k].x * dx + w[k].y * dy + w[k].z * dz;
    float rad = fabsf(w[k].x) * c.hx + fabsf(w[k].y) * c.hy + fabsf(w[k].z) * c.hz;
    float lb = fmaxf(fabsf(u) - rad * 1.0001f - 1e-5f, 0.f);
    acc += lb * lb;
  }
  return acc <= c2 * 1.0001f;
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Appends this lane's candidate (if it survives) to the wave's LDS list.
__device__ __forceinline__ int append_survivor(int* sv, int ns, bool pass, int pid, int lane) {
  uint64_t b = __ballot(pass);
  if (pass) {
    uint64_t below = b & ((lane == 0) ? 0ull : (~0ull >> (64 - lane)));
    sv[ns + __popcll(below)] = pid;
  }
  return ns + __popcll(b);
}

// ---------------------------------------------------------------------------
// Forward
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kWaves * 64) eval_fwd_kernel(
    const float4* __restrict__ xs, const int* __restrict__ perm, const TileInfo* __restrict__ tiles,
    const float4* __restrict__ tlo, const float4* __restrict__ thi, int ntiles,
    const int* __restrict__ cell_start, const int* __restrict__ cell_prims,
    const PrimRec* __restrict__ recs, float c2, float* __restrict__ L) {
  __shared__ int surv[kWaves][kSurvCap];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = xcd_remap(blockIdx.x, gridDim.x) * kWaves + wave;
  if (t >= ntiles) return;
  const TileInfo ti = tiles[t];
  const TileCtx tc = tile_ctx(tlo, thi, t);
  const float4 p = xs[ti.start + min(lane, ti.count - 1)];
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;
  const int cs = cell_start[ti.cell], ce = cell_start[ti.cell + 1];
  int* sv = surv[wave];
  int ns = 0;
  for (int base = cs; base < ce; base += 64) {
    const int j = base + lane;
    bool pass = false;
    int pid = 0;
    if (j < ce) {
      pid = cell_prims[j];
      pass = tile_may_touch(recs[pid], tc, c2);
    }
    ns = append_survivor(sv, ns, pass, pid, lane);
    if (ns > kSurvCap - 64 || base + 64 >= ce) {
      wave_sync_lds();
      for (int s = 0; s < ns; ++s) {
        const int id = __builtin_amdgcn_readfirstlane(sv[s]);
        const PrimRec r = recs[id];
        const float dx = p.x - r.r0.x, dy = p.y - r.r0.y, dz = p.z - r.r0.z;
        const float u0 = r.r1.x * dx + r.r1.y * dy + r.r1.z * dz;
        const float u1 = r.r2.x * dx + r.r2.y * dy + r.r2.z * dz;
        const float u2 = r.r3.x * dx + r.r3.y * dy + r.r3.z * dz;
        const float m2 = u0 * u0 + u1 * u1 + u2 * u2;
        const float w = (m2 <= c2) ? __builtin_amdgcn_exp2f(-m2) : 0.f;
        a0 += w * r.r0.w;
        a1 += w * r.r1.w;
        a2 += w * r.r2.w;
      }
      ns = 0;
      wave_sync_lds();
    }
  }
  if (lane < ti.count) {
    const int o = perm[ti.start + lane];
    L[(int64_t)o * 3 + 0] = a0;
    L[(int64_t)o * 3 + 1] = a1;
    L[(int64_t)o * 3 + 2] = a2;
  }
}

// ---------------------------------------------------------------------------
// Exact pair count (same traversal as the forward)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kWaves * 64) count_pairs_kernel(
    const float4* __restrict__ xs, const TileInfo* __restrict__ tiles,
    const float4* __restrict__ tlo, const float4* __restrict__ thi, int ntiles,
    const int* __restrict__ cell_start, const int* __restrict__ cell_prims,
    const PrimRec* __restrict__ recs, float c2, unsigned long long* __restrict__ out) {
  __shared__ int surv[kWaves][kSurvCap];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = blockIdx.x * kWaves + wave;
  if (t >= ntiles) return;
  const TileInfo ti = tiles[t];
  const TileCtx tc = tile_ctx(tlo, thi, t);
  const float4 p = xs[ti.start + min(lane, ti.count - 1)];
  const bool active = lane < ti.count;
  unsigned cnt = 0;
  const int cs = cell_start[ti.cell], ce = cell_start[ti.cell + 1];
  int* sv = surv[wave];
  int ns = 0;
  for (int base = cs; base < ce; base += 64) {
    const int j = base + lane;
    bool pass = false;
    int pid = 0;
    if (j < ce) {
      pid = cell_prims[j];
      pass = tile_may_touch(recs[pid], tc, c2);
    }
    ns = append_survivor(sv, ns, pass, pid, lane);
    if (ns > kSurvCap - 64 || base + 64 >= ce) {
      wave_sync_lds();
      for (int s = 0; s < ns; ++s) {
        const int id = __builtin_amdgcn_readfirstlane(sv[s]);
        const PrimRec r = recs[id];
        const float dx = p.x - r.r0.x, dy = p.y - r.r0.y, dz = p.z - r.r0.z;
        const float u0 = r.r1.x * dx + r.r1.y * dy + r.r1.z * dz;
        const float u1 = r.r2.x * dx + r.r2.y * dy + r.r2.z * dz;
        const float u2 = r.r3.x * dx + r.r3.y * dy + r.r3.z * dz;
        const float m2 = u0 * u0 + u1 * u1 + u2 * u2;
        cnt += (active && m2 <= c2) ? 1u : 0u;
      }
      ns = 0;
      wave_sync_lds();
    }
  }
  // wave total, one atomic per wave
  unsigned long long tot = cnt;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off, 64);
  if (lane == 0) atomicAdd(out, tot);
}

// ---------------------------------------------------------------------------
// Backward
// ---------------------------------------------------------------------------
struct GradOut {
  float *mu, *quat, *ls, *rgb;
};

// Maps the per-primitive sums (in the kappa-scaled whitened frame) to
// parameter gradients and adds them.  With u' = kappa u, W' = kappa W:
//   dmu = W^T A = W'^T A' / kappa^2,   dsigma_k = S'_k / kappa^2,
//   dR[j][k] = -M[k][j] / s_k = -M'[k][j] / (kappa s_k),
//   dq = (I - qhat qhat^T) dqhat / |q|,  dqhat = sum_jk dR[j][k] dR[j][k]/dqhat.
__device__ __forceinline__ void grad_epilogue(const PrimRec& r, const float* __restrict__ quat,
                                              const float* __restrict__ ls, int pid,
                                              const float GP[3], const float A[3], const float S[3],
                                              const float M[3][3], GradOut go) {
  const float ik2 = (float)(1.0 / kKappa2);
  const float ik = (float)(1.0 / 0.84932180028801904272);  // 1 / sqrt(kKappa2)
  const float4 wr[3] = {r.r1, r.r2, r.r3};
  float dmu[3];
  dmu[0] = (wr[0].x * A[0] + wr[1].x * A[1] + wr[2].x * A[2]) * ik2;
  dmu[1] = (wr[0].y * A[0] + wr[1].y * A[1] + wr[2].y * A[2]) * ik2;
  dmu[2] = (wr[0].z * A[0] + wr[1].z * A[1] + wr[2].z * A[2]) * ik2;
  float qw = quat[pid * 4], qx = quat[pid * 4 + 1], qy = quat[pid * 4 + 2], qz = quat[pid * 4 + 3];
  const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  const float iq = 1.f / qn;
  qw *= iq; qx *= iq; qy *= iq; qz *= iq;
  float G[3][3];  // G[j][k] = d loss / d R[j][k]
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float inv_s = __expf(-ls[pid * 3 + k]) * ik;
#pragma unroll
    for (int j = 0; j < 3; ++j) G[j][k] = -M[k][j] * inv_s;
  }
  float gw = 2.f * (qz * (G[1][0] - G[0][1]) + qy * (G[0][2] - G[2][0]) + qx * (G[2][1] - G[1][2]));
  float gx = 2.f * (qy * (G[0][1] + G[1][0]) + qz * (G[0][2] + G[2][0]) + qw * (G[2][1] - G[1][2]) -
                    2.f * qx * (G[1][1] + G[2][2]));
  float gy = 2.f * (qx * (G[0][1] + G[1][0]) + qz * (G[1][2] + G[2][1]) + qw * (G[0][2] - G[2][0]) -
                    2.f * qy * (G[0][0] + G[2][2]));
  float gz = 2.f * (qx * (G[0][2] + G[2][0]) + qy * (G[1][2] + G[2][1]) + qw * (G[1][0] - G[0][1]) -
                    2.f * qz * (G[0][0] + G[1][1]));
  const float dot = qw * gw + qx * gx + qy * gy + qz * gz;
  gw = (gw - dot * qw) * iq;
  gx = (gx - dot * qx) * iq;
  gy = (gy - dot * qy) * iq;
  gz = (gz - dot * qz) * iq;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    unsafeAtomicAdd(go.mu + pid * 3 + a, dmu[a]);
    unsafeAtomicAdd(go.ls + pid * 3 + a, S[a] * ik2);
    unsafeAtomicAdd(go.rgb + pid * 3 + a, GP[a]);
  }
  unsafeAtomicAdd(go.quat + pid * 4 + 0, gw);
  unsafeAtomicAdd(go.quat + pid * 4 + 1, gx);
  unsafeAtomicAdd(go.quat + pid * 4 + 2, gy);
  unsafeAtomicAdd(go.quat + pid * 4 + 3, gz);
}

__global__ void __launch_bounds__(kWaves * 64) eval_bwd_kernel(
    const float4* __restrict__ xs, const int* __restrict__ perm, const TileInfo* __restrict__ tiles,
    const float4* __restrict__ tlo, const float4* __restrict__ thi, int ntiles,
    const int* __restrict__ cell_start, const int* __restrict__ cell_prims,
    const PrimRec* __restrict__ recs, const float* __restrict__ quat, const float* __restrict__ ls,
    float c2, const float* __restrict__ dL, GradOut go) {
  __shared__ int surv[kWaves][kSurvCap];
  __shared__ float4 qx_s[kWaves][kTile];
  __shared__ float4 qg_s[kWaves][kTile];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = xcd_remap(blockIdx.x, gridDim.x) * kWaves + wave;
  if (t >= ntiles) return;
  const TileInfo ti = tiles[t];
  const TileCtx tc = tile_ctx(tlo, thi, t);
  {
    const int k = ti.start + min(lane, ti.count - 1);
    const float4 p = xs[k];
    const int o = perm[k];
    qx_s[wave][lane] = p;
    qg_s[wave][lane] = lane < ti.count
                           ? make_float4(dL[(int64_t)o * 3], dL[(int64_t)o * 3 + 1],
                                         dL[(int64_t)o * 3 + 2], 0.f)
                           : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  const int nq = ti.count;
  const int cs = cell_start[ti.cell], ce = cell_start[ti.cell + 1];
  int* sv = surv[wave];
  int ns = 0;
  for (int base = cs; base < ce; base += 64) {
    const int j = base + lane;
    bool pass = false;
    int pid = 0;
    if (j < ce) {
      pid = cell_prims[j];
      pass = tile_may_touch(recs[pid], tc, c2);
    }
    ns = append_survivor(sv, ns, pass, pid, lane);
    const bool last = base + 64 >= ce;
    if (ns >= 64 || (last && ns > 0)) {
      wave_sync_lds();
      // consume survivors 64 at a time: lane = primitive
      int done = 0;
      while (ns - done >= 64 || (last && done < ns)) {
        const bool valid = done + lane < ns;
        const int id = valid ? sv[done + lane] : 0;
        const PrimRec r = recs[id];
        float GP[3] = {0.f, 0.f, 0.f}, A[3] = {0.f, 0.f, 0.f}, S[3] = {0.f, 0.f, 0.f};
        float M[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
        bool any = false;
        for (int k = 0; k < nq; ++k) {
          const float4 x = qx_s[wave][k];
          const float dx = x.x - r.r0.x, dy = x.y - r.r0.y, dz = x.z - r.r0.z;
          const float u0 = r.r1.x * dx + r.r1.y * dy + r.r1.z * dz;
          const float u1 = r.r2.x * dx + r.r2.y * dy + r.r2.z * dz;
          const float u2 = r.r3.x * dx + r.r3.y * dy + r.r3.z * dz;
          const float m2 = u0 * u0 + u1 * u1 + u2 * u2;
          if (m2 <= c2) {
            const float4 g = qg_s[wave][k];
            const float w = __builtin_amdgcn_exp2f(-m2);
            const float a = g.x * r.r0.w + g.y * r.r1.w + g.z * r.r2.w;
            const float c = a * w;
            GP[0] += w * g.x;
            GP[1] += w * g.y;
            GP[2] += w * g.z;
            const float cu[3] = {c * u0, c * u1, c * u2};
            const float uu[3] = {u0, u1, u2};
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              A[q] += cu[q];
              S[q] += cu[q] * uu[q];
              M[q][0] += cu[q] * dx;
              M[q][1] += cu[q] * dy;
              M[q][2] += cu[q] * dz;
            }
            any = true;
          }
        }
        if (valid && any) grad_epilogue(r, quat, ls, id, GP, A, S, M, go);
        done += 64;
      }
      // keep the unconsumed tail at the front of the list
      const int rem = ns - done;
      if (rem > 0) {
        const int v = lane < rem ? sv[done + lane] : 0;
        wave_sync_lds();
        if (lane < rem) sv[lane] = v;
        ns = rem;
      } else {
        ns = 0;
      }
      wave_sync_lds();
    }
  }
}

}  // namespace

static int fwd_blocks(int64_t ntiles) { return (int)((ntiles + kWaves - 1) / kWaves); }

gpf_status launch_eval_fwd(const gpf_grid* g, float* L, hipStream_t s) {
  const gpf_queries* qs = g->qs;
  const float c2 = (float)(kKappa2 * g->cutoff * g->cutoff);
  hipLaunchKernelGGL(eval_fwd_kernel, dim3(fwd_blocks(qs->ntiles)), dim3(kWaves * 64), 0, s,
                     qs->xs, qs->perm, qs->tiles, qs->tile_lo, qs->tile_hi, (int)qs->ntiles,
                     g->cell_start, g->cell_prims, g->rec, c2, L);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

gpf_status launch_eval_bwd(const gpf_grid* g, const float* dL, gpf_field_grad* grad,
                           hipStream_t s) {
  const gpf_queries* qs = g->qs;
  const float c2 = (float)(kKappa2 * g->cutoff * g->cutoff);
  GradOut go{grad->mu, grad->quat, grad->log_scale, grad->rgb};
  hipLaunchKernelGGL(eval_bwd_kernel, dim3(fwd_blocks(qs->ntiles)), dim3(kWaves * 64), 0, s,
                     qs->xs, qs->perm, qs->tiles, qs->tile_lo, qs->tile_hi, (int)qs->ntiles,
                     g->cell_start, g->cell_prims, g->rec, g->quat, g->log_scale, c2, dL, go);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

gpf_status launch_count_pairs(const gpf_grid* g, unsigned long long* d_count, hipStream_t s) {
  const gpf_queries* qs = g->qs;
  const float c2 = (float)(kKappa2 * g->cutoff * g->cutoff);
  GPF_HIP(hipMemsetAsync(d_count, 0, sizeof(unsigned long long), s));
  hipLaunchKernelGGL(count_pairs_kernel, dim3(fwd_blocks(qs->ntiles)), dim3(kWaves * 64), 0, s,
                     qs->xs, qs->tiles, qs->tile_lo, qs->tile_hi, (int)qs->ntiles, g->cell_start,
                     g->cell_prims, g->rec, c2, d_count);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

}  // namespace gpf
