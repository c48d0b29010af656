// Device helpers shared by the truncated radiance kernels (eval.hip) and the
// hybrid-query kernels (hybrid.hip): tile boxes, wave-level LDS ordering, the
// map from per-primitive sums to parameter gradients and the pass that adds
// the gathered rows to the caller's gradient arrays.
#pragma once

#include "common.h"

namespace gpf {
namespace {

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

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Maps the per-primitive sums (kappa-scaled whitened frame, u' = kappa u,
// W' = kappa W) to the 13 parameter gradients:
//   GP = sum w g,  A' = sum c u',  U' = sum c u' u'^T   (c = w g.Phi).
// Since d = W^-1 u = R diag(s) u' / kappa, the sums M[k][j] = sum c u_k d_j
// follow from U': M[k][j] = sum_l U'[k][l] R[j][l] s_l / kappa^2.  Then
//   dmu = W^T A = W'^T A' / kappa^2,   dsigma_k = U'[k][k] / kappa^2,
//   dR[j][k] = -M[k][j] / s_k,
//   dq = (I - qhat qhat^T) dqhat / |q|,  dqhat = sum_jk dR[j][k] dR[j][k]/dqhat,
//   dPhi = GP.
// out: [0..2] mu, [3..6] quat, [7..9] log_scale, [10..12] rgb.
__device__ __forceinline__ void grad_epilogue(const PrimRec& r, const float* __restrict__ quat,
                                              const float* __restrict__ ls, int pid,
                                              const float GP[3], const float A[3],
                                              const float U[6], float out[13]) {
  const float ik2 = (float)(1.0 / kKappa2);
  const float4 wr[3] = {r.r1, r.r2, r.r3};
  out[0] = (wr[0].x * A[0] + wr[1].x * A[1] + wr[2].x * A[2]) * ik2;
  out[1] = (wr[0].y * A[0] + wr[1].y * A[1] + wr[2].y * A[2]) * ik2;
  out[2] = (wr[0].z * A[0] + wr[1].z * A[1] + wr[2].z * A[2]) * ik2;
  float qw = quat[pid * 4], qx = quat[pid * 4 + 1], qy = quat[pid * 4 + 2], qz = quat[pid * 4 + 3];
  const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  const float iq = 1.f / qn;
  qw *= iq; qx *= iq; qy *= iq; qz *= iq;
  float R[3][3];
  R[0][0] = 1.f - 2.f * (qy * qy + qz * qz);
  R[0][1] = 2.f * (qx * qy - qw * qz);
  R[0][2] = 2.f * (qx * qz + qw * qy);
  R[1][0] = 2.f * (qx * qy + qw * qz);
  R[1][1] = 1.f - 2.f * (qx * qx + qz * qz);
  R[1][2] = 2.f * (qy * qz - qw * qx);
  R[2][0] = 2.f * (qx * qz - qw * qy);
  R[2][1] = 2.f * (qy * qz + qw * qx);
  R[2][2] = 1.f - 2.f * (qx * qx + qy * qy);
  const float sc[3] = {__expf(ls[pid * 3]), __expf(ls[pid * 3 + 1]), __expf(ls[pid * 3 + 2])};
  const float Uf[3][3] = {{U[0], U[1], U[2]}, {U[1], U[3], U[4]}, {U[2], U[4], U[5]}};
  float G[3][3];  // G[j][k] = d loss / d R[j][k] = -M[k][j] / s_k
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float f = -ik2 / sc[k];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      G[j][k] = f * (Uf[k][0] * R[j][0] * sc[0] + Uf[k][1] * R[j][1] * sc[1] +
                     Uf[k][2] * R[j][2] * sc[2]);
  }
  float gw = 2.f * (qz * (G[1][0] - G[0][1]) + qy * (G[0][2] - G[2][0]) + qx * (G[2][1] - G[1][2]));
  float gx = 2.f * (qy * (G[0][1] + G[1][0]) + qz * (G[0][2] + G[2][0]) + qw * (G[2][1] - G[1][2]) -
                    2.f * qx * (G[1][1] + G[2][2]));
  float gy = 2.f * (qx * (G[0][1] + G[1][0]) + qz * (G[1][2] + G[2][1]) + qw * (G[0][2] - G[2][0]) -
                    2.f * qy * (G[0][0] + G[2][2]));
  float gz = 2.f * (qx * (G[0][2] + G[2][0]) + qy * (G[1][2] + G[2][1]) + qw * (G[1][0] - G[0][1]) -
                    2.f * qz * (G[0][0] + G[1][1]));
  const float dot = qw * gw + qx * gx + qy * gy + qz * gz;
  out[3] = (gw - dot * qw) * iq;
  out[4] = (gx - dot * qx) * iq;
  out[5] = (gy - dot * qy) * iq;
  out[6] = (gz - dot * qz) * iq;
  out[7] = U[0] * ik2;
  out[8] = U[3] * ik2;
  out[9] = U[5] * ik2;
  out[10] = GP[0];
  out[11] = GP[1];
  out[12] = GP[2];
}

// Per primitive: the sums (GP, A', U') gathered over every group become the
// 13 parameter gradients, plus any direct centre gradient gathered in slots
// 12..14 (terms that do not pass through the whitened frame); they are added
// to the caller's arrays and the rows are cleared for the next call.
__global__ void __launch_bounds__(256) grad_finalize_kernel(float4* __restrict__ rows, int n,
                                                            const PrimRec* __restrict__ recs,
                                                            const float* __restrict__ quat,
                                                            const float* __restrict__ ls,
                                                            float* __restrict__ gmu,
                                                            float* __restrict__ gq,
                                                            float* __restrict__ gls,
                                                            float* __restrict__ grgb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 a = rows[i * 4], b = rows[i * 4 + 1], c = rows[i * 4 + 2], d = rows[i * 4 + 3];
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  rows[i * 4] = z;
  rows[i * 4 + 1] = z;
  rows[i * 4 + 2] = z;
  rows[i * 4 + 3] = z;
  const float GP[3] = {a.x, a.y, a.z}, A[3] = {a.w, b.x, b.y};
  const float U[6] = {b.z, b.w, c.x, c.y, c.z, c.w};
  float out[13];
  grad_epilogue(recs[i], quat, ls, i, GP, A, U, out);
  gmu[i * 3] += out[0] + d.x;
  gmu[i * 3 + 1] += out[1] + d.y;
  gmu[i * 3 + 2] += out[2] + d.z;
  gq[i * 4] += out[3];
  gq[i * 4 + 1] += out[4];
  gq[i * 4 + 2] += out[5];
  gq[i * 4 + 3] += out[6];
  gls[i * 3] += out[7];
  gls[i * 3 + 1] += out[8];
  gls[i * 3 + 2] += out[9];
  grgb[i * 3] += out[10];
  grgb[i * 3 + 1] += out[11];
  grgb[i * 3 + 2] += out[12];
}

}  // namespace
}  // namespace gpf
