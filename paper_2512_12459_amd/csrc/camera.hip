// Hybrid camera integrator (Sec. 4.2 rendering with the field; supplementary
// Alg. S2): camera paths follow the sphere's specular interactions with a
// throughput beta and end at the first diffuse surface, where the field's
// radiance is taken and weighted by beta, or on the light when the path so far
// was specular.  Then the pixel composition and its gradient.
//
// One thread per (pixel, sample) path k = pixel * samples + s.  The primary
// ray passes through the pixel centre (row 0 at the top); the glass sphere's
// branch at depth j is decided by u0 of the uniforms for counter (k, j, 1, 0)
// (Philox4x64-10, key (seed, 0)), so camera decisions never share a counter
// with photon paths (third word 0).
#include "common.h"
#include "scene.h"

namespace gpf {
namespace {

struct CamBasis {
  float eye[3], fwd[3], right[3], up[3];
  float tan_half, aspect;
  int width, height;
};

__global__ void __launch_bounds__(256) camera_kernel(CamBasis cb, int samples, int64_t n,
                                                     uint64_t seed, int max_depth, float lo,
                                                     float hi, int sphere, float3 le,
                                                     float* __restrict__ xo,
                                                     float* __restrict__ bo,
                                                     int* __restrict__ fo,
                                                     float* __restrict__ leo) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t pix = k / samples;
  const int row = (int)(pix / cb.width), col = (int)(pix - (int64_t)row * cb.width);
  const float sx = (2.f * ((float)col + 0.5f) / (float)cb.width - 1.f) * cb.tan_half * cb.aspect;
  const float sy = (1.f - 2.f * ((float)row + 0.5f) / (float)cb.height) * cb.tan_half;
  float d[3], o[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    d[a] = cb.fwd[a] + sx * cb.right[a] + sy * cb.up[a];
    o[a] = cb.eye[a];
  }
  {
    const float inv = 1.f / sqrtf(dot3(d, d));
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] *= inv;
  }
  float beta[3] = {1.f, 1.f, 1.f};
  float x_rec[3] = {0.f, 0.f, 0.f}, b_rec[3] = {0.f, 0.f, 0.f}, l_rec[3] = {0.f, 0.f, 0.f};
  int f_rec = -1;
  for (int j = 1; j <= max_depth; ++j) {
    int face;
    const float tb = box_crossing(o, d, face);
    const float ts = sphere ? sphere_crossing(o, d) : INFINITY;
    const bool hit_s = ts < tb;
    if (!hit_s && (face < 0 || face == 5)) break;  // leaves through the open side
    const float t = hit_s ? ts : tb;
    const float x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
    if (!hit_s) {
      const bool lit = face == 1 && x[0] >= lo && x[0] <= hi && x[2] >= lo && x[2] <= hi;
      if (lit) {
        l_rec[0] = le.x * beta[0];
        l_rec[1] = le.y * beta[1];
        l_rec[2] = le.z * beta[2];
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          x_rec[a] = x[a];
          b_rec[a] = beta[a];
        }
        f_rec = face;
      }
      break;
    }
    float u[4];
    uniforms((uint64_t)k, (uint64_t)j, 1ull, seed, u);
    float fac[3];
    sphere_scatter(d, x, u[0], sphere, fac);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      beta[a] *= fac[a];
      o[a] = x[a];
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    xo[k * 3 + a] = x_rec[a];
    bo[k * 3 + a] = b_rec[a];
    leo[k * 3 + a] = l_rec[a];
  }
  fo[k] = f_rec;
}

// First index of the ascending slot[0..m) that is >= v.
__device__ __forceinline__ int64_t lower_bound(const int64_t* slot, int64_t m, int64_t v) {
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (slot[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// L_pix[p] = (1/S) sum_s Le[p S + s] + (1/S) sum over the diffuse hits k of
// pixel p (slot[k] in [p S, p S + S)) of beta_c[k] * Lq[k], in slot order.
__global__ void __launch_bounds__(256) compose_kernel(const float* __restrict__ Le, int64_t n_pix,
                                                      int S, const int64_t* __restrict__ slot,
                                                      const float* __restrict__ beta_c,
                                                      const float* __restrict__ Lq, int64_t m,
                                                      float* __restrict__ L) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n_pix) return;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;
  for (int s = 0; s < S; ++s) {
    const int64_t k = p * S + s;
    a0 += Le[k * 3];
    a1 += Le[k * 3 + 1];
    a2 += Le[k * 3 + 2];
  }
  for (int64_t k = m > 0 ? lower_bound(slot, m, p * S) : 0; k < m && slot[k] < (p + 1) * S; ++k) {
    a0 += beta_c[k * 3] * Lq[k * 3];
    a1 += beta_c[k * 3 + 1] * Lq[k * 3 + 1];
    a2 += beta_c[k * 3 + 2] * Lq[k * 3 + 2];
  }
  const float inv = 1.f / (float)S;
  L[p * 3] = a0 * inv;
  L[p * 3 + 1] = a1 * inv;
  L[p * 3 + 2] = a2 * inv;
}

__global__ void __launch_bounds__(256) compose_bwd_kernel(const float* __restrict__ dL,
                                                          int64_t n_pix, int S,
                                                          const int64_t* __restrict__ slot,
                                                          const float* __restrict__ beta_c,
                                                          int64_t m, float* __restrict__ dLq) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int64_t sk = slot[k];
  const int64_t p = sk >= 0 ? sk / S : n_pix;   // a slot outside the image gets no gradient
  const float inv = 1.f / (float)S;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    dLq[k * 3 + a] = p < n_pix ? beta_c[k * 3 + a] * (dL[p * 3 + a] * inv) : 0.f;
}

}  // namespace

gpf_status launch_camera_trace(const gpf_camera* cam, int samples, uint64_t seed, int max_depth,
                               float lo, float hi, int sphere, float* x, float* beta, int* face,
                               float* Le, hipStream_t s) {
  // camera frame in FP64, rounded once
  double e[3], f[3], up[3];
  for (int a = 0; a < 3; ++a) {
    e[a] = cam->eye[a];
    f[a] = (double)cam->target[a] - cam->eye[a];
    up[a] = cam->up[a];
  }
  auto norm = [](double v[3]) {
    const double l = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int a = 0; a < 3; ++a) v[a] /= l;
  };
  norm(f);
  double r[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
  norm(r);
  const double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
  CamBasis cb;
  for (int a = 0; a < 3; ++a) {
    cb.eye[a] = (float)e[a];
    cb.fwd[a] = (float)f[a];
    cb.right[a] = (float)r[a];
    cb.up[a] = (float)u[a];
  }
  cb.tan_half = (float)std::tan(cam->vfov_deg * M_PI / 360.0);
  cb.aspect = (float)((double)cam->width / (double)cam->height);
  cb.width = cam->width;
  cb.height = cam->height;
  const double area = (double)(hi - lo) * (double)(hi - lo);
  const float3 le = area > 0 ? make_float3((float)(12.0 / (M_PI * area)), (float)(10.0 / (M_PI * area)),
                                           (float)(8.0 / (M_PI * area)))
                             : make_float3(0.f, 0.f, 0.f);
  const int64_t n = (int64_t)cam->width * cam->height * samples;
  hipLaunchKernelGGL(camera_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cb, samples,
                     n, seed, max_depth, lo, hi, sphere, le, x, beta, face, Le);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

gpf_status launch_camera_compose(const float* Le, int64_t n_pix, int S, const int64_t* slot,
                                 const float* beta_c, const float* Lq, int64_t m, float* L,
                                 hipStream_t s) {
  hipLaunchKernelGGL(compose_kernel, dim3((unsigned)((n_pix + 255) / 256)), dim3(256), 0, s, Le,
                     n_pix, S, slot, beta_c, Lq, m, L);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

gpf_status launch_camera_compose_backward(const float* dL, int64_t n_pix, int S,
                                          const int64_t* slot, const float* beta_c, int64_t m,
                                          float* dLq, hipStream_t s) {
  if (m == 0) return GPF_OK;
  hipLaunchKernelGGL(compose_bwd_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, dL,
                     n_pix, S, slot, beta_c, m, dLq);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

}  // namespace gpf
