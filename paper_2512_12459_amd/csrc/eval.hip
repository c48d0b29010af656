// Radiance query (forward), its gradient (backward) and the exact pair count,
// for the 3-sigma truncated, un-normalised sum.
//
// Work decomposition: query points are sorted by cell and cut into tiles of
// 64; two consecutive tiles of one cell form a group.
//  - forward:  one wave per group, lane = query point (one per tile); the
//              cell's candidates are culled against both tile boxes into an
//              LDS list, then each survivor is read with wave-uniform loads
//              (scalar in the fitting pass, broadcast LDS loads of staged
//              records in the standalone forward) and evaluated on the tiles
//              it may touch;
//  - backward: one wave per group, lane = survivor (64 at a time), looping
//              over the group's points broadcast from LDS; the 12 sums per
//              primitive are added to padded rows with row-coalesced atomics
//              and mapped to parameter gradients once per primitive;
//  - fitting pass: one wave per group runs the forward, the squared error
//              against the targets and the backward with the resulting
//              upstream gradient, over the survivors it has just kept.
// Weights are recomputed in the backward; nothing per pair is stored.
#include <mutex>

#include "radiance_common.h"

namespace gpf {

// Gradient rows of the allocation-free backward: one 64-byte row per
// primitive for up to kNoAllocMaxPrims primitives (16 MiB on every device the
// library runs on, held until the process ends).  Host code never uses this
// name as an address: the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) float4 scratch[kNoAllocMaxPrims * 4];

namespace {

constexpr int kWaves = 4;        // waves (tiles) per workgroup
constexpr int kSurvCap = 512;    // survivor slots per wave

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
constexpr int kFwdSurvCap = 256;   // staged survivors per wave

// Forward of one group of two consecutive tiles of one cell, run by one wave:
// lane l owns point l of the first tile and point l of the second (px, py,
// pz; acc receives their radiance).  Lane = candidate culls the cell's
// records [cs, ce) (one contiguous block of 64 at a time) against both tile
// boxes; a survivor is staged in sv (kFwdSurvCap ints of LDS) as
// entry | tile mask << 30.  Every lane then evaluates each survivor for the
// tiles it may touch (a wave-uniform branch per tile), reading mu, W' and the
// flux with wave-uniform scalar loads: d = x - mu, u' = W' d (the local frame
// of Alg. S3), w = 2^-|u'|^2 inside the cut.  With kl non-null the survivors
// are also stored there in cell-list order (at most kSurvPerGroup of them).
// Returns the number of survivors, also past the list's capacity.
__device__ __forceinline__ int fwd_group(const TileCtx& ta, const TileCtx& tb, bool has_b,
                                         const float (&px)[2], const float (&py)[2],
                                         const float (&pz)[2], float (&acc)[2][3], int cs, int ce,
                                         const PrimRec* __restrict__ cell_recs, float c2, int* sv,
                                         int* __restrict__ kl, int lane) {
  int ns = 0, kept = 0;
  for (int base = cs; base < ce; base += 64) {
    const int j = base + lane;
    int mask = 0;
    if (j < ce) {
      const PrimRec r = cell_recs[j];
      mask = (tile_may_touch(r, ta, c2) ? 1 : 0) | ((has_b && tile_may_touch(r, tb, c2)) ? 2 : 0);
    }
    const uint64_t bal = __ballot(mask != 0);
    if (mask) {
      const uint64_t below = bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane)));
      sv[ns + __popcll(below)] = j | (mask << 30);
    }
    ns += __popcll(bal);
    if (ns > kFwdSurvCap - 64 || base + 64 >= ce) {
      wave_sync_lds();
      const int nsu = __builtin_amdgcn_readfirstlane(ns);  // wave-uniform trip count
      if (kl)
        for (int s = lane; s < nsu && kept + s < kSurvPerGroup; s += 64) kl[kept + s] = sv[s];
      kept += nsu;
      for (int s = 0; s < nsu; ++s) {
        const int head = __builtin_amdgcn_readfirstlane(sv[s]);
        const PrimRec r = cell_recs[head & 0x3fffffff];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          if (!((head >> (30 + i)) & 1)) continue;   // wave-uniform
          const float dx = px[i] - r.r0.x, dy = py[i] - r.r0.y, dz = pz[i] - r.r0.z;
          const float u0 = fmaf(r.r1.z, dz, fmaf(r.r1.y, dy, r.r1.x * dx));
          const float u1 = fmaf(r.r2.z, dz, fmaf(r.r2.y, dy, r.r2.x * dx));
          const float u2 = fmaf(r.r3.z, dz, fmaf(r.r3.y, dy, r.r3.x * dx));
          const float m2 = fmaf(u2, u2, fmaf(u1, u1, u0 * u0));
          const float w = (m2 <= c2) ? __builtin_amdgcn_exp2f(-m2) : 0.f;
          acc[i][0] = fmaf(w, r.r0.w, acc[i][0]);
          acc[i][1] = fmaf(w, r.r1.w, acc[i][1]);
          acc[i][2] = fmaf(w, r.r2.w, acc[i][2]);
        }
      }
      ns = 0;
      wave_sync_lds();
    }
  }
  return kept;
}

// The standalone forward kernel's variant of fwd_group.  On gfx950 a VALU
// instruction that reads or writes a scalar register issues at half the rate
// of one whose operands are all vector registers (measured with FP32 FMA
// streams), so this variant stages the survivors' records in LDS, reads each
// back with broadcast loads into vector registers and keeps the tile boxes and
// the cutoff in vector registers too.  The broadcast loads cost LDS bandwidth
// that the fitting pass's backward half needs for its own point reads, so the
// fitting pass keeps fwd_group (measured: the standalone forward 11% faster,
// the fitting pass 2% slower with this variant).  Both evaluate the same
// pairs in the same order with the same arithmetic and give identical sums.
constexpr int kStage = 64;   // staged survivor records per wave (64 bytes each)

// x must be wave-uniform: the scalar-register operand of the copy takes one
// lane's value (the compiler reads the first lane of a vector register).
__device__ __forceinline__ float in_vgpr(float x) {
  float v;
  asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
  return v;
}

__device__ __forceinline__ TileCtx ctx_in_vgprs(const TileCtx& c) {
  TileCtx v;
  v.cx = in_vgpr(c.cx);
  v.cy = in_vgpr(c.cy);
  v.cz = in_vgpr(c.cz);
  v.hx = in_vgpr(c.hx);
  v.hy = in_vgpr(c.hy);
  v.hz = in_vgpr(c.hz);
  return v;
}

// Weight inside the cut, zero beyond it: w = 2^-m2 if m2 <= c2.  The test is
// the sign of c2 - m2 (exact: the difference of two floats is negative exactly
// when m2 > c2), applied as a bit mask with v_bfi_b32 (the compiler would
// otherwise turn the mask back into a compare that writes a scalar mask).
__device__ __forceinline__ float cut_weight(float m2, float c2v) {
  const float e = __builtin_amdgcn_exp2f(-m2);
  const int beyond = __float_as_int(c2v - m2) >> 31;   // all ones beyond the cut
  float w;
  asm("v_bfi_b32 %0, %1, 0, %2" : "=v"(w) : "v"(beyond), "v"(e));   // beyond ? 0 : e
  return w;
}

// One staged survivor (record R in vector registers; tile mask in bits 0..1
// of the wave-uniform `tiles`) on the tiles it may touch, as fwd_group.
__device__ __forceinline__ void eval_staged(const float4 (&R)[4], int tiles, const float (&px)[2],
                                            const float (&py)[2], const float (&pz)[2],
                                            float (&acc)[2][3], float c2v) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (!((tiles >> i) & 1)) continue;   // wave-uniform
    const float dx = px[i] - R[0].x, dy = py[i] - R[0].y, dz = pz[i] - R[0].z;
    const float u0 = fmaf(R[1].z, dz, fmaf(R[1].y, dy, R[1].x * dx));
    const float u1 = fmaf(R[2].z, dz, fmaf(R[2].y, dy, R[2].x * dx));
    const float u2 = fmaf(R[3].z, dz, fmaf(R[3].y, dy, R[3].x * dx));
    const float m2 = fmaf(u2, u2, fmaf(u1, u1, u0 * u0));
    const float w = cut_weight(m2, c2v);
    acc[i][0] = fmaf(w, R[0].w, acc[i][0]);
    acc[i][1] = fmaf(w, R[1].w, acc[i][1]);
    acc[i][2] = fmaf(w, R[2].w, acc[i][2]);
  }
}

// fwd_group with the survivors' records (already in the culling lanes'
// registers) staged in LDS (stage: kStage x 64 bytes, the tile mask in place
// of the primitive index), a batch of up to 64 at a time, and read back with
// broadcast loads; kl receives the survivors as in fwd_group.
__device__ __forceinline__ int fwd_group_staged(const TileCtx& ta_s, const TileCtx& tb_s,
                                                bool has_b, const float (&px)[2],
                                                const float (&py)[2], const float (&pz)[2],
                                                float (&acc)[2][3], int cs, int ce,
                                                const PrimRec* __restrict__ cell_recs, float c2,
                                                float4* stage, int* __restrict__ kl, int lane) {
  const TileCtx ta = ctx_in_vgprs(ta_s), tb = ctx_in_vgprs(tb_s);
  const float c2v = in_vgpr(c2);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int kept = 0;
  for (int base = cs; base < ce; base += 64) {
    const int j = base + lane;
    // past the cell's end a lane re-reads the last record and keeps nothing
    const PrimRec r = cell_recs[min(j, ce - 1)];
    int mask = 0;
    if (j < ce)
      mask = (tile_may_touch(r, ta, c2v) ? 1 : 0) | ((has_b && tile_may_touch(r, tb, c2v)) ? 2 : 0);
    const uint64_t bal = __ballot(mask != 0);
    const int nb = __popcll(bal);   // wave-uniform
    if (nb == 0) continue;
    if (mask) {
      const int slot = __popcll(bal & below);
      stage[slot * 4 + 0] = r.r0;
      stage[slot * 4 + 1] = r.r1;
      stage[slot * 4 + 2] = r.r2;
      stage[slot * 4 + 3] = make_float4(r.r3.x, r.r3.y, r.r3.z, __int_as_float(mask));
      if (kl && kept + slot < kSurvPerGroup) kl[kept + slot] = j | (mask << 30);
    }
    wave_sync_lds();
    for (int s = 0; s < nb; ++s) {
      float4 R[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) R[k] = stage[s * 4 + k];
      eval_staged(R, __builtin_amdgcn_readfirstlane(__float_as_int(R[3].w)), px, py, pz, acc, c2v);
    }
    kept += nb;
    wave_sync_lds();   // the next batch overwrites the stage
  }
  return kept;
}

// The points of a group as fwd_group takes them (lanes past the group's
// count repeat its last point).
__device__ __forceinline__ void load_group_points(const float4* __restrict__ xs,
                                                  const GroupInfo& gi, float (&px)[2],
                                                  float (&py)[2], float (&pz)[2],
                                                  float (&acc)[2][3], int lane) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float4 p = xs[gi.start + min(lane + 64 * i, gi.count - 1)];
    px[i] = p.x;
    py[i] = p.y;
    pz[i] = p.z;
    acc[i][0] = acc[i][1] = acc[i][2] = 0.f;
  }
}

// One wave per group, held to 64 VGPRs (8 waves per SIMD).
__global__ void __launch_bounds__(kWaves * 64) __attribute__((amdgpu_waves_per_eu(8, 8)))
eval_fwd_kernel(
    const float4* __restrict__ xs, const int* __restrict__ perm,
    const GroupInfo* __restrict__ groups, int ngroups, const float4* __restrict__ tlo,
    const float4* __restrict__ thi, const int* __restrict__ cell_start,
    const PrimRec* __restrict__ cell_recs, float c2,
    float* __restrict__ L, int* __restrict__ keep, int* __restrict__ keep_count) {
  static_assert(kGroupTiles == 2, "the forward pairs the two tiles of a group");
  __shared__ float4 stage_all[kWaves][kStage * 4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = xcd_remap(blockIdx.x) * kWaves + wave;
  if (g >= ngroups) return;
  const GroupInfo gi = groups[g];
  const TileCtx ta = tile_ctx(tlo, thi, gi.first_tile);
  const bool has_b = gi.count > kTile;
  const TileCtx tb = has_b ? tile_ctx(tlo, thi, gi.first_tile + 1) : ta;
  float px[2], py[2], pz[2], acc[2][3];
  load_group_points(xs, gi, px, py, pz, acc, lane);
  const int cs = cell_start[gi.cell], ce = cell_start[gi.cell + 1];
  int* kl = keep ? keep + (int64_t)g * kSurvPerGroup : nullptr;
  const int kept = fwd_group_staged(ta, tb, has_b, px, py, pz, acc, cs, ce, cell_recs, c2,
                                    stage_all[wave], kl, lane);
  if (keep_count && lane == 0) keep_count[g] = kept;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int k = lane + 64 * i;
    if (k < gi.count) {
      const int o = perm[gi.start + k];
      L[(int64_t)o * 3 + 0] = acc[i][0];
      L[(int64_t)o * 3 + 1] = acc[i][1];
      L[(int64_t)o * 3 + 2] = acc[i][2];
    }
  }
}
// ---------------------------------------------------------------------------
// Exact pair count (same traversal as the forward)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kWaves * 64) count_pairs_kernel(
    const float4* __restrict__ xs, const TileInfo* __restrict__ tiles,
    const float4* __restrict__ tlo, const float4* __restrict__ thi, int ntiles,
    const int* __restrict__ cell_start, const PrimRec* __restrict__ cell_recs, float c2,
    unsigned long long* __restrict__ out) {
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
    const bool pass = j < ce && tile_may_touch(cell_recs[j], tc, c2);
    ns = append_survivor(sv, ns, pass, j, lane);
    if (ns > kSurvCap - 64 || base + 64 >= ce) {
      wave_sync_lds();
      for (int s = 0; s < ns; ++s) {
        const int id = __builtin_amdgcn_readfirstlane(sv[s]);
        const PrimRec r = cell_recs[id];
        const float dx = p.x - r.r0.x, dy = p.y - r.r0.y, dz = p.z - r.r0.z;
        const float u0 = fmaf(r.r1.z, dz, fmaf(r.r1.y, dy, r.r1.x * dx));
        const float u1 = fmaf(r.r2.z, dz, fmaf(r.r2.y, dy, r.r2.x * dx));
        const float u2 = fmaf(r.r3.z, dz, fmaf(r.r3.y, dy, r.r3.x * dx));
        const float m2 = fmaf(u2, u2, fmaf(u1, u1, u0 * u0));
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
constexpr int kBwdWaves = 4;                  // independent waves per workgroup
constexpr int kBwdThreads = kBwdWaves * 64;
constexpr int kGroupQ = kTile * kGroupTiles;  // points per group (max, a multiple of 4)
constexpr int kListCap = 128;                 // survivor slots per list and wave
constexpr int kRowStride = 14;                // transpose row stride (12 sums, pad, row id)

// 64 survivors (lane = primitive, cell entry ent) against the points [qb, qe) of the wave's
// group, held in LDS (points past the group's count carry a zero upstream
// gradient).  The 12 per-primitive sums are added to the padded per-primitive
// buffer with row-coalesced atomics: after an LDS transpose (16 rows at a
// time, so that the buffer stays small), 16 lanes update one 64-byte row per
// instruction.
__device__ __forceinline__ void bwd_chunk(int ent, bool valid, int qb, int qe,
                                          const PrimRec* __restrict__ cell_recs, float c2,
                                          const float2* qp, float* rw,
                                          float* __restrict__ grad_rows, int lane) {
  const PrimRec r = cell_recs[ent];
  const int id = __float_as_int(r.r3.w);
  float GP[3] = {0.f, 0.f, 0.f}, A[3] = {0.f, 0.f, 0.f};
  float U[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  bool any = false;
  for (int k = qb; k < qe; k += 2) {
    float4 xq[2], gq[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {   // point k: (x, y), (z, gx), (gy, gz)
      const float2 a = qp[3 * (k + i)], b = qp[3 * (k + i) + 1], c = qp[3 * (k + i) + 2];
      xq[i] = make_float4(a.x, a.y, b.x, 0.f);
      gq[i] = make_float4(b.y, c.x, c.y, 0.f);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float dx = xq[i].x - r.r0.x, dy = xq[i].y - r.r0.y, dz = xq[i].z - r.r0.z;
      const float u0 = fmaf(r.r1.z, dz, fmaf(r.r1.y, dy, r.r1.x * dx));
      const float u1 = fmaf(r.r2.z, dz, fmaf(r.r2.y, dy, r.r2.x * dx));
      const float u2 = fmaf(r.r3.z, dz, fmaf(r.r3.y, dy, r.r3.x * dx));
      const float m2 = fmaf(u2, u2, fmaf(u1, u1, u0 * u0));
      const bool in = m2 <= c2;
      const float w = in ? __builtin_amdgcn_exp2f(-m2) : 0.f;
      any |= in;
      const float a = fmaf(gq[i].z, r.r2.w, fmaf(gq[i].y, r.r1.w, gq[i].x * r.r0.w));
      const float c = a * w;
      GP[0] = fmaf(w, gq[i].x, GP[0]);
      GP[1] = fmaf(w, gq[i].y, GP[1]);
      GP[2] = fmaf(w, gq[i].z, GP[2]);
      const float cu0 = c * u0, cu1 = c * u1, cu2 = c * u2;
      A[0] += cu0;
      A[1] += cu1;
      A[2] += cu2;
      U[0] = fmaf(cu0, u0, U[0]);
      U[1] = fmaf(cu0, u1, U[1]);
      U[2] = fmaf(cu0, u2, U[2]);
      U[3] = fmaf(cu1, u1, U[3]);
      U[4] = fmaf(cu1, u2, U[4]);
      U[5] = fmaf(cu2, u2, U[5]);
    }
  }
  // the sums are added over groups as they are and mapped to parameter
  // gradients once per primitive by the finalize pass
  const bool write = valid && any;
  const float sums[12] = {GP[0], GP[1], GP[2], A[0], A[1], A[2], U[0], U[1], U[2], U[3], U[4], U[5]};
  const int sub = lane >> 4, e = lane & 15;
#pragma unroll
  for (int h = 0; h < 4; ++h) {   // 16 rows at a time
    if ((lane >> 4) == h) {
      const int rl = lane & 15;
#pragma unroll
      for (int k = 0; k < 12; ++k) rw[rl * kRowStride + k] = write ? sums[k] : 0.f;
      rw[rl * kRowStride + 13] = __int_as_float(write ? id : -1);
    }
    wave_sync_lds();
#pragma unroll 4
    for (int rr = 0; rr < 4; ++rr) {
      const int row = rr * 4 + sub;
      const int rid = __float_as_int(rw[row * kRowStride + 13]);
      if (e < 12 && rid >= 0) unsafeAtomicAdd(grad_rows + (int64_t)rid * 16 + e, rw[row * kRowStride + e]);
    }
    wave_sync_lds();
  }
}

// Backward of one group of two consecutive tiles of one cell, run by one wave
// with no workgroup-wide synchronisation; the group's points and their
// upstream gradients are in qp.  The survivors are sorted onto three LDS
// stacks by tile mask (first tile only, second tile only, both).  A stack
// that holds 64 entries is drained at once as a pure chunk over the points of
// its tiles; the remainders (under 64 each) are taken at the end in the order
// first-tile-only, both, second-tile-only, so a chunk loops over the second
// tile only if one of its survivors may touch it, and over the first likewise.
// The survivors come from the forward's list kl when it holds all nk of them
// (nk <= kSurvPerGroup): the same (primitive, tile mask) pairs, in the same
// order, as the cull would find, so the same (primitive, point) slots are
// evaluated without testing any candidate again (stacks drain at other
// moments, which only regroups the sums).  Otherwise lane = candidate culls
// the cell's records [cs, ce) against both tile boxes.
__device__ __forceinline__ void bwd_group(const GroupInfo& gi, const TileCtx& ta,
                                          const TileCtx& tb, bool has_b, int cs, int ce,
                                          const PrimRec* __restrict__ cell_recs, float c2,
                                          const float2* qp, int* sv0, int* sv1, int* sv2,
                                          float* rw, float* __restrict__ grad_rows,
                                          const int* __restrict__ kl, int nk, int lane) {
  const int qe_a = (min(gi.count, kTile) + 3) & ~3, qe_all = (gi.count + 3) & ~3;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int n0 = 0, n1 = 0, n2 = 0;  // stack heights, each below 64 between batches
  if (kl && nk <= kSurvPerGroup) {
    for (int base = 0; base < nk; base += 64) {
      const int ent = (base + lane < nk) ? kl[base + lane] : 0;
      const int mask = (base + lane < nk) ? ((ent >> 30) & 3) : 0;
      const int pid = ent & 0x3fffffff;   // cell entry
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
        bwd_chunk(sv0[n0 + lane], true, 0, qe_a, cell_recs, c2, qp, rw, grad_rows, lane);
      }
      if (n1 >= 64) {
        n1 -= 64;
        bwd_chunk(sv1[n1 + lane], true, kTile, qe_all, cell_recs, c2, qp, rw, grad_rows, lane);
      }
      if (n2 >= 64) {
        n2 -= 64;
        bwd_chunk(sv2[n2 + lane], true, 0, qe_all, cell_recs, c2, qp, rw, grad_rows, lane);
      }
    }
  } else {
    // The candidates in batches of 64.  Entries past the end repeat the
    // cell's last one, keeping every load unconditional and in bounds.  (No
    // prefetch of the next batch: its 16 registers would set the whole
    // kernel's register count, and this path only runs where a group's list
    // overflowed or no forward kept one.)
    for (int base = cs; base < ce; base += 64) {
      const PrimRec rec_c = cell_recs[min(base + lane, ce - 1)];
      const int pid = base + lane;   // cell entry
      int mask = 0;
      if (base + lane < ce)
        mask = (tile_may_touch(rec_c, ta, c2) ? 1 : 0) |
               ((has_b && tile_may_touch(rec_c, tb, c2)) ? 2 : 0);
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
        bwd_chunk(sv0[n0 + lane], true, 0, qe_a, cell_recs, c2, qp, rw, grad_rows, lane);
      }
      if (n1 >= 64) {
        n1 -= 64;
        bwd_chunk(sv1[n1 + lane], true, kTile, qe_all, cell_recs, c2, qp, rw, grad_rows, lane);
      }
      if (n2 >= 64) {
        n2 -= 64;
        bwd_chunk(sv2[n2 + lane], true, 0, qe_all, cell_recs, c2, qp, rw, grad_rows, lane);
      }
    }
  }
  const int total = n0 + n1 + n2;
  for (int chunk = 0; chunk < total; chunk += 64) {
    const int v = chunk + lane;
    int id = cs, cat = 0;   // padded lanes read a valid entry and add nothing
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
    bwd_chunk(id, cat != 0, use_a ? 0 : kTile, use_b ? qe_all : qe_a, cell_recs, c2, qp,
              rw, grad_rows, lane);
  }
}

// Point k of a group in the backward's LDS layout: (x, y), (z, gx), (gy, gz).
// Points past the group's count sit at the first tile's centre (any finite
// point would do) with a zero upstream gradient.
__device__ __forceinline__ void put_point(float2* qp, int k, float x, float y, float z, float gx,
                                          float gy, float gz) {
  qp[3 * k] = make_float2(x, y);
  qp[3 * k + 1] = make_float2(z, gx);
  qp[3 * k + 2] = make_float2(gy, gz);
}

// One wave per group; dL[q][3] in the points' original order.  Six waves per
// SIMD: at most 80 VGPRs, and 5.5 KB of LDS per wave (points 3 KB, stacks
// 1.5 KB, transpose rows 0.9 KB).
__global__ void __launch_bounds__(kBwdThreads) __attribute__((amdgpu_waves_per_eu(6, 6)))
eval_bwd_kernel(
    const float4* __restrict__ xs, const int* __restrict__ perm,
    const GroupInfo* __restrict__ groups, int ngroups, const float4* __restrict__ tlo,
    const float4* __restrict__ thi, const int* __restrict__ cell_start,
    const PrimRec* __restrict__ cell_recs, float c2,
    const float* __restrict__ dL, float* __restrict__ grad_rows, const int* __restrict__ keep,
    const int* __restrict__ keep_count) {
  static_assert(kGroupTiles == 2, "the backward splits survivors over the two tiles of a group");
  __shared__ int sv_all[kBwdWaves][3 * kListCap];
  __shared__ float2 qp_all[kBwdWaves][3 * kGroupQ];
  __shared__ float rows_all[kBwdWaves][16 * kRowStride];
  // wave-uniform (the compiler cannot see it): the group and everything
  // derived from it live in scalar registers and the loops stay uniform
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int g = xcd_remap(blockIdx.x) * kBwdWaves + wave;
  if (g >= ngroups) return;  // per wave: no workgroup barrier follows
  const GroupInfo gi = groups[g];
  const TileCtx ta = tile_ctx(tlo, thi, gi.first_tile);
  const bool has_b = gi.count > kTile;
  const TileCtx tb = has_b ? tile_ctx(tlo, thi, gi.first_tile + 1) : ta;
  float2* qp = qp_all[wave];
  for (int k = lane; k < kGroupQ; k += 64) {
    if (k < gi.count) {
      const int o = perm[gi.start + k];
      const float4 p = xs[gi.start + k];
      put_point(qp, k, p.x, p.y, p.z, dL[(int64_t)o * 3], dL[(int64_t)o * 3 + 1],
                dL[(int64_t)o * 3 + 2]);
    } else {
      put_point(qp, k, ta.cx, ta.cy, ta.cz, 0.f, 0.f, 0.f);
    }
  }
  wave_sync_lds();
  const int cs = cell_start[gi.cell], ce = cell_start[gi.cell + 1];
  const int* kl = keep_count ? keep + (int64_t)g * kSurvPerGroup : nullptr;
  const int nk = keep_count ? keep_count[g] : 0;
  bwd_group(gi, ta, tb, has_b, cs, ce, cell_recs, c2, qp, sv_all[wave], sv_all[wave] + kListCap,
            sv_all[wave] + 2 * kListCap, rows_all[wave], grad_rows, kl, nk, lane);
}

// One fitting pass per group (Sec. 4.3), one wave each: the forward of the
// group's points, their squared error against the targets T (original
// order) and upstream gradient dL = scale (L - T), then the backward of the
// same group with that dL, over the survivors the forward has just kept (and
// stored with their count, as the forward kernel does).
// L is written in the original order; loss[0] += sum (L - T)^2 in FP64, one
// atomic per group.  The forward's staging list shares LDS with the
// backward's stacks; occupancy as for the backward kernel.
__global__ void __launch_bounds__(kBwdThreads) __attribute__((amdgpu_waves_per_eu(6, 6)))
fit_pass_kernel(
    const float4* __restrict__ xs, const int* __restrict__ perm,
    const GroupInfo* __restrict__ groups, int ngroups, const float4* __restrict__ tlo,
    const float4* __restrict__ thi, const int* __restrict__ cell_start,
    const PrimRec* __restrict__ cell_recs, float c2, const float* __restrict__ T, float scale,
    float* __restrict__ L, double* __restrict__ loss, int* __restrict__ keep,
    int* __restrict__ keep_count, float* __restrict__ grad_rows) {
  static_assert(kGroupTiles == 2, "the pass pairs the two tiles of a group");
  static_assert(kFwdSurvCap <= 3 * kListCap, "the forward staging fits in the backward stacks");
  __shared__ int sv_all[kBwdWaves][3 * kListCap];
  __shared__ float2 qp_all[kBwdWaves][3 * kGroupQ];
  __shared__ float rows_all[kBwdWaves][16 * kRowStride];
  // wave-uniform (the compiler cannot see it): the group and everything
  // derived from it live in scalar registers and the loops stay uniform
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int g = xcd_remap(blockIdx.x) * kBwdWaves + wave;
  if (g >= ngroups) return;  // per wave: no workgroup barrier follows
  const GroupInfo gi = groups[g];
  const TileCtx ta = tile_ctx(tlo, thi, gi.first_tile);
  const bool has_b = gi.count > kTile;
  const TileCtx tb = has_b ? tile_ctx(tlo, thi, gi.first_tile + 1) : ta;
  float px[2], py[2], pz[2], acc[2][3];
  load_group_points(xs, gi, px, py, pz, acc, lane);
  const int cs = cell_start[gi.cell], ce = cell_start[gi.cell + 1];
  int* kl = keep ? keep + (int64_t)g * kSurvPerGroup : nullptr;
  const int nk = fwd_group(ta, tb, has_b, px, py, pz, acc, cs, ce, cell_recs, c2,
                           sv_all[wave], kl, lane);
  if (keep_count && lane == 0) keep_count[g] = nk;   // the lists stay valid for a later backward
  // other lanes of this wave read the list back below
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  float2* qp = qp_all[wave];
  double part = 0.0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int k = lane + 64 * i;
    if (k < gi.count) {
      const int o = perm[gi.start + k];
      float d[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        d[c] = acc[i][c] - T[(int64_t)o * 3 + c];
        L[(int64_t)o * 3 + c] = acc[i][c];
        part += (double)d[c] * (double)d[c];
      }
      put_point(qp, k, px[i], py[i], pz[i], scale * d[0], scale * d[1], scale * d[2]);
    } else {
      put_point(qp, k, ta.cx, ta.cy, ta.cz, 0.f, 0.f, 0.f);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
  if (lane == 0) unsafeAtomicAdd(loss, part);
  wave_sync_lds();
  bwd_group(gi, ta, tb, has_b, cs, ce, cell_recs, c2, qp, sv_all[wave], sv_all[wave] + kListCap,
            sv_all[wave] + 2 * kListCap, rows_all[wave], grad_rows, kl, nk, lane);
}


__global__ void __launch_bounds__(256) zero_float4_kernel(float4* __restrict__ p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

}  // namespace

static int fwd_blocks(int64_t ntiles) { return (int)((ntiles + kWaves - 1) / kWaves); }

// The forward's survivor lists (kept for the backward of the same build);
// allocated on first use and grown with the number of groups.  Without them
// (allocation refused) the forward keeps nothing and the backward culls.
void ensure_survivor_lists(gpf_grid* g) {
  const int64_t ng = g->qs->ngroups;
  if (g->surv_groups >= ng) return;
  dev_free(g->surv, (size_t)g->surv_groups * kSurvPerGroup * sizeof(int));
  dev_free(g->surv_count, (size_t)g->surv_groups * sizeof(int));
  g->surv = g->surv_count = nullptr;
  g->surv_groups = 0;
  if (dev_alloc((void**)&g->surv, (size_t)ng * kSurvPerGroup * sizeof(int), "survivor lists") !=
          GPF_OK ||
      dev_alloc((void**)&g->surv_count, (size_t)ng * sizeof(int), "survivor counts") != GPF_OK) {
    dev_free(g->surv, (size_t)ng * kSurvPerGroup * sizeof(int));
    g->surv = nullptr;
    return;
  }
  g->surv_groups = ng;
}

gpf_status launch_eval_fwd(const gpf_grid* gc, float* L, hipStream_t s) {
  gpf_grid* g = const_cast<gpf_grid*>(gc);  // the survivor lists live in the handle
  const gpf_queries* qs = g->qs;
  const float c2 = (float)(kKappa2 * g->cutoff * g->cutoff);
  ensure_survivor_lists(g);
  hipLaunchKernelGGL(eval_fwd_kernel, dim3(xcd_grid(fwd_blocks(qs->ngroups))), dim3(kWaves * 64), 0, s,
                     qs->xs, qs->perm, qs->groups, (int)qs->ngroups,
                     qs->tile_lo, qs->tile_hi, g->cell_start, g->cell_recs, c2, L, g->surv,
                     g->surv ? g->surv_count : nullptr);
  GPF_HIP(hipGetLastError());
  g->surv_ready = g->surv != nullptr;
  return GPF_OK;
}

// The padded per-primitive rows the backward passes gather into (allocated
// and cleared once per handle; the finalize pass leaves them zeroed).
gpf_status ensure_grad_rows(gpf_grid* g, hipStream_t s) {
  if (g->grad_cap < g->n) {
    dev_free(g->grad_rows, g->grad_cap * sizeof(float4) * 4);
    g->grad_rows = nullptr;
    g->grad_cap = 0;
    gpf_status st = dev_alloc((void**)&g->grad_rows, (size_t)g->n * sizeof(float4) * 4,
                              "gradient rows");
    if (st != GPF_OK) return st;
    GPF_HIP(hipMemsetAsync(g->grad_rows, 0, (size_t)g->n * sizeof(float4) * 4, s));
    g->grad_cap = g->n;
    g->bytes += (size_t)g->n * sizeof(float4) * 4;
  }
  return GPF_OK;
}

gpf_status launch_grad_finalize(gpf_grid* g, float4* rows, gpf_field_grad* grad, hipStream_t s) {
  hipLaunchKernelGGL(grad_finalize_kernel, dim3((unsigned)((g->n + 255) / 256)), dim3(256), 0, s,
                     rows, (int)g->n, g->rec, g->quat, g->log_scale, grad->mu,
                     grad->quat, grad->log_scale, grad->rgb);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

// The backward into gradient rows `rows` ([n][4] float4, zero on entry; the
// finalize pass leaves them zero again).
static gpf_status launch_eval_bwd_rows(gpf_grid* g, const float* dL, gpf_field_grad* grad,
                                       float4* rows, hipStream_t s) {
  const gpf_queries* qs = g->qs;
  const float c2 = (float)(kKappa2 * g->cutoff * g->cutoff);
  hipLaunchKernelGGL(eval_bwd_kernel, dim3(xcd_grid((qs->ngroups + kBwdWaves - 1) / kBwdWaves)),
                     dim3(kBwdThreads), 0, s, qs->xs,
                     qs->perm, qs->groups, (int)qs->ngroups,
                     qs->tile_lo, qs->tile_hi, g->cell_start, g->cell_recs, c2, dL,
                     (float*)rows, g->surv_ready ? g->surv : nullptr,
                     g->surv_ready ? g->surv_count : nullptr);
  GPF_HIP(hipGetLastError());
  return launch_grad_finalize(g, rows, grad, s);
}

gpf_status launch_eval_bwd(const gpf_grid* gc, const float* dL, gpf_field_grad* grad,
                           hipStream_t s) {
  gpf_grid* g = const_cast<gpf_grid*>(gc);  // scratch rows live in the handle
  gpf_status st = ensure_grad_rows(g, s);
  if (st != GPF_OK) return st;
  return launch_eval_bwd_rows(g, dL, grad, g->grad_rows, s);
}

// One fitting pass into the handle's gradient rows, then the finalize pass.
gpf_status launch_fit_pass(const gpf_grid* gc, const float* T, float* L, double* loss,
                           gpf_field_grad* grad, hipStream_t s) {
  gpf_grid* g = const_cast<gpf_grid*>(gc);  // survivor lists and rows live in the handle
  const gpf_queries* qs = g->qs;
  const float c2 = (float)(kKappa2 * g->cutoff * g->cutoff);
  const float scale = (float)(2.0 / (double)qs->q);   // as gpf_mse_loss
  ensure_survivor_lists(g);
  gpf_status st = ensure_grad_rows(g, s);
  if (st != GPF_OK) return st;
  hipLaunchKernelGGL(fit_pass_kernel, dim3(xcd_grid((qs->ngroups + kBwdWaves - 1) / kBwdWaves)),
                     dim3(kBwdThreads), 0, s, qs->xs, qs->perm, qs->groups, (int)qs->ngroups,
                     qs->tile_lo, qs->tile_hi, g->cell_start, g->cell_recs, c2, T, scale, L, loss,
                     g->surv, g->surv ? g->surv_count : nullptr, (float*)g->grad_rows);
  GPF_HIP(hipGetLastError());
  g->surv_ready = g->surv != nullptr;
  return launch_grad_finalize(g, g->grad_rows, grad, s);
}

// Device address of `scratch`, looked up once per device (with that device
// current) and kept; hipGetSymbolAddress allocates nothing.
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_addr[kMaxDevices] = {};

static gpf_status scratch_rows(float4** rows) {
  int dev = 0;
  GPF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(GPF_ERR_CAPACITY, "device ordinal beyond the library's per-device table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return set_error(GPF_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_addr[dev] = p;
  }
  *rows = static_cast<float4*>(g_scratch_addr[dev]);
  return GPF_OK;
}

gpf_status launch_eval_bwd_noalloc(const gpf_grid* gc, const float* dL, gpf_field_grad* grad,
                                   hipStream_t s) {
  gpf_grid* g = const_cast<gpf_grid*>(gc);
  if (g->n > kNoAllocMaxPrims)
    return set_error(GPF_ERR_CAPACITY, "the allocation-free backward takes at most " +
                                           std::to_string(kNoAllocMaxPrims) + " primitives, got " +
                                           std::to_string(g->n));
  float4* rows = nullptr;
  gpf_status st = scratch_rows(&rows);
  if (st != GPF_OK) return st;
  // the array keeps whatever the last call on this device left: clear the
  // rows this call gathers into (a fill kernel, no memset node)
  const int64_t n4 = g->n * 4;
  hipLaunchKernelGGL(zero_float4_kernel, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s, rows,
                     n4);
  GPF_HIP(hipGetLastError());
  return launch_eval_bwd_rows(g, dL, grad, rows, s);
}

gpf_status launch_count_pairs(const gpf_grid* g, unsigned long long* d_count, hipStream_t s) {
  const gpf_queries* qs = g->qs;
  const float c2 = (float)(kKappa2 * g->cutoff * g->cutoff);
  GPF_HIP(hipMemsetAsync(d_count, 0, sizeof(unsigned long long), s));
  hipLaunchKernelGGL(count_pairs_kernel, dim3(fwd_blocks(qs->ntiles)), dim3(kWaves * 64), 0, s,
                     qs->xs, qs->tiles, qs->tile_lo, qs->tile_hi, (int)qs->ntiles, g->cell_start,
                     g->cell_recs, c2, d_count);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

}  // namespace gpf
