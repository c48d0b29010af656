// The box + glass/mirror sphere scene shared by the photon tracer and the
// camera integrator: Philox4x64-10 uniforms, box and sphere crossings, and
// the sphere's specular interactions.
//
// Box [0,1]^3 with diffuse faces floor y=0 (0), ceiling y=1 (1), x=0 (2),
// x=1 (3), back z=0 (4); the side z=1 (5) is open.  Sphere of radius 0.2 at
// (0.5, 0.5, 0.5): glass of index 1.5 (sphere == 1) or a mirror of
// reflectance (0.95, 0.64, 0.54) (sphere == 2).
#pragma once

#include "common.h"

namespace gpf {
namespace {

constexpr float kTEps = 1e-4f;
constexpr float kIor = 1.5f;
constexpr float kSphR = 0.2f;
constexpr float kPi = 3.14159265358979323846f;
constexpr int kSphereGlass = 1, kSphereMirror = 2;

__constant__ float kAlbedo[5][3] = {{0.73f, 0.73f, 0.73f}, {0.73f, 0.73f, 0.73f},
                                     {0.63f, 0.06f, 0.05f}, {0.14f, 0.45f, 0.09f},
                                     {0.73f, 0.73f, 0.73f}};
__constant__ float kMirrorRho[3] = {0.95f, 0.64f, 0.54f};
__constant__ float kNormal[5][3] = {{0, 1, 0}, {0, -1, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 0, 1}};
__constant__ float kTangT[5][3] = {{0, 0, 1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 0, 0}};
__constant__ float kTangB[5][3] = {{1, 0, 0}, {0, 0, 1}, {0, 0, 1}, {0, 1, 0}, {0, 1, 0}};

// Philox4x64-10 (Salmon et al., SC'11).
__device__ __forceinline__ void philox(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B97F4A7C15ull;
      k1 += 0xBB67AE8584CAA73Bull;
    }
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Four uniforms (w >> 40) * 2^-24 of counter (a, b, c2, 0), key (seed, 0).
__device__ __forceinline__ void uniforms(uint64_t a, uint64_t b, uint64_t c2, uint64_t seed,
                                         float u[4]) {
  uint64_t c[4] = {a, b, c2, 0ull};
  philox(c, seed, 0ull);
#pragma unroll
  for (int i = 0; i < 4; ++i) u[i] = (float)(c[i] >> 40) * (1.0f / 16777216.0f);
}

__device__ __forceinline__ float dot3(const float a[3], const float b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Nearest box face crossed ahead of o along d: its distance and the face
// (5 = the open side, -1 = none).  Only faces the direction leaves through
// count (the face a path sits on, which it leaves inwards, never does), and a
// point on or past such a face meets it at once (distance 0), so a path that
// starts on an edge cannot slip out through the neighbouring face.  Ties go
// to the lower face index.
__device__ __forceinline__ float box_crossing(const float o[3], const float d[3], int& face) {
  float tb = INFINITY;
  face = -1;
  const float tf[6] = {d[1] < 0.f ? fmaxf((0.f - o[1]) / d[1], 0.f) : INFINITY,
                       d[1] > 0.f ? fmaxf((1.f - o[1]) / d[1], 0.f) : INFINITY,
                       d[0] < 0.f ? fmaxf((0.f - o[0]) / d[0], 0.f) : INFINITY,
                       d[0] > 0.f ? fmaxf((1.f - o[0]) / d[0], 0.f) : INFINITY,
                       d[2] < 0.f ? fmaxf((0.f - o[2]) / d[2], 0.f) : INFINITY,
                       d[2] > 0.f ? fmaxf((1.f - o[2]) / d[2], 0.f) : INFINITY};
#pragma unroll
  for (int k = 0; k < 6; ++k)
    if (tf[k] < tb) {
      tb = tf[k];
      face = k;
    }
  return tb;
}

// Nearest sphere crossing ahead of o along d (beyond kTEps), or INFINITY.
__device__ __forceinline__ float sphere_crossing(const float o[3], const float d[3]) {
  const float oc[3] = {o[0] - 0.5f, o[1] - 0.5f, o[2] - 0.5f};
  const float b = dot3(oc, d);
  const float cc = dot3(oc, oc) - kSphR * kSphR;
  const float disc = b * b - cc;
  float ts = INFINITY;
  if (disc > 0.f) {
    const float sq = sqrtf(disc);
    const float t0 = -b - sq, t1 = -b + sq;
    ts = t0 > kTEps ? t0 : (t1 > kTEps ? t1 : INFINITY);
  }
  return ts;
}

// Specular interaction at sphere point x for direction d (updated in place,
// unit length): glass reflects when u0 < F (exact unpolarised Fresnel, total
// internal reflection F = 1) and refracts otherwise, the mirror reflects.
// Returns the radiance throughput factor of the chosen branch for a camera
// path: 1 for a Fresnel-sampled reflection, (eta_i / eta_t)^2 for a
// refraction, the mirror's reflectance (channel c) for the mirror.
__device__ __forceinline__ void sphere_scatter(float d[3], const float x[3], float u0, int sphere,
                                               float fac[3]) {
  float ns[3] = {(x[0] - 0.5f) / kSphR, (x[1] - 0.5f) / kSphR, (x[2] - 0.5f) / kSphR};
  const float cos_o = -dot3(d, ns);
  const bool inside = cos_o < 0.f;
  if (inside) ns[0] = -ns[0], ns[1] = -ns[1], ns[2] = -ns[2];
  const float cos_i = fabsf(cos_o);
  float nd[3];
  fac[0] = fac[1] = fac[2] = 1.f;
  bool reflect = true;
  float eta = 1.f, cos_t = 0.f;
  if (sphere == kSphereMirror) {
#pragma unroll
    for (int a = 0; a < 3; ++a) fac[a] = kMirrorRho[a];
  } else {
    const float ei = inside ? kIor : 1.f, et = inside ? 1.f : kIor;
    eta = ei / et;
    const float sin2_t = eta * eta * fmaxf(0.f, 1.f - cos_i * cos_i);
    float F = 1.f;
    if (sin2_t < 1.f) {
      cos_t = sqrtf(fmaxf(0.f, 1.f - sin2_t));
      const float rs = (ei * cos_i - et * cos_t) / (ei * cos_i + et * cos_t);
      const float rp = (ei * cos_t - et * cos_i) / (ei * cos_t + et * cos_i);
      F = 0.5f * (rs * rs + rp * rp);
    }
    reflect = u0 < F;
    if (!reflect) fac[0] = fac[1] = fac[2] = eta * eta;
  }
  if (reflect) {
#pragma unroll
    for (int a = 0; a < 3; ++a) nd[a] = d[a] + 2.f * cos_i * ns[a];
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) nd[a] = eta * d[a] + (eta * cos_i - cos_t) * ns[a];
  }
  const float inv = 1.f / sqrtf(dot3(nd, nd));
#pragma unroll
  for (int a = 0; a < 3; ++a) d[a] = nd[a] * inv;
}

}  // namespace
}  // namespace gpf
