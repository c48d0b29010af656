// Learned initialiser network on MFMA: 96 -> 128 (GELU) -> 128 (GELU) -> 10,
// bfloat16 operands with FP32 accumulation (v_mfma_f32_16x16x32_bf16), FP32
// master weights updated by Adam.
//
// MFMA fragment layout (16x16x32, wave64; l = lane, r = l & 15, g = l >> 4):
//   A[16 x 32]: lane l holds A[r][8g .. 8g+7]
//   B[32 x 16]: lane l holds B[8g .. 8g+7][r]
//   D[16 x 16]: lane l holds D[4g + i][r], i = 0..3
// Weights are kept in bfloat16 copies laid out so that every fragment is one
// 16-byte load: W^T (output-major) for the forward products, W (input-major)
// for the backward products.
#include "common.h"
#include "mlp.h"

namespace gpf {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int kLd = 136;   // row stride (bf16) of row-major LDS tiles
constexpr int kTs = 72;    // row stride (bf16) of feature-major LDS tiles (64 samples)

__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest, ties to even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.f + erff(z * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) +
         z * __expf(-0.5f * z * z) * 0.39894228040143268f;
}

// masters (FP32, W[in][out]) -> bfloat16 copies
__global__ void __launch_bounds__(256) mlp_convert_kernel(const float* __restrict__ p,
                                                          MlpWeights w) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  // w1t[n][k] = W1[k][n]
  if (t < kH * kIn) {
    const int n = t / kIn, k = t % kIn;
    w.w1t[t] = f2bf(p[kOffW1 + k * kH + n]);
  }
  if (t < kH * kH) {
    const int n = t / kH, k = t % kH;
    w.w2t[t] = f2bf(p[kOffW2 + k * kH + n]);   // w2t[n][k] = W2[k][n]
    w.w2[t] = f2bf(p[kOffW2 + t]);             // w2[i][o]  = W2[i][o]
  }
  if (t < 16 * kH) {
    const int n = t / kH, k = t % kH;            // w3t[n][k] = W3[k][n], n < 10
    w.w3t[t] = n < kOut ? f2bf(p[kOffW3 + k * kOut + n]) : (uint16_t)0;
  }
  if (t < kH * 32) {
    const int n = t / 32, k = t % 32;            // w3p[i][o] = W3[i][o], o < 10
    w.w3p[t] = k < kOut ? f2bf(p[kOffW3 + n * kOut + k]) : (uint16_t)0;
  }
}

// ---------------------------------------------------------------------------
// Inference: one wave per 16 samples.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) mlp_forward_kernel(const uint16_t* __restrict__ X,
                                                          int64_t B, MlpWeights w,
                                                          const float* __restrict__ p,
                                                          float* __restrict__ Y) {
  __shared__ __attribute__((aligned(16))) uint16_t hs[4][16 * kLd];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (row0 >= B) return;
  const int64_t xrow = min(row0 + r, B - 1);
  uint16_t* h = hs[wave];
  // layer 1
#pragma unroll
  for (int nb = 0; nb < kH / 16; ++nb) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < kIn / 32; ++kc)
      acc = mfma(ld8(X + xrow * kIn + 32 * kc + 8 * g), ld8(w.w1t + (16 * nb + r) * kIn + 32 * kc + 8 * g), acc);
    const float bias = p[kOffB1 + 16 * nb + r];
#pragma unroll
    for (int i = 0; i < 4; ++i) h[(4 * g + i) * kLd + 16 * nb + r] = f2bf(gelu(acc[i] + bias));
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // layer 2 (all products first, then overwrite the tile)
  f32x4 z2[kH / 16];
#pragma unroll
  for (int nb = 0; nb < kH / 16; ++nb) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < kH / 32; ++kc)
      acc = mfma(ld8(h + r * kLd + 32 * kc + 8 * g), ld8(w.w2t + (16 * nb + r) * kH + 32 * kc + 8 * g), acc);
    z2[nb] = acc;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int nb = 0; nb < kH / 16; ++nb) {
    const float bias = p[kOffB2 + 16 * nb + r];
#pragma unroll
    for (int i = 0; i < 4; ++i) h[(4 * g + i) * kLd + 16 * nb + r] = f2bf(gelu(z2[nb][i] + bias));
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // layer 3
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kc = 0; kc < kH / 32; ++kc)
    acc = mfma(ld8(h + r * kLd + 32 * kc + 8 * g), ld8(w.w3t + r * kH + 32 * kc + 8 * g), acc);
  if (r < kOut) {
    const float bias = p[kOffB3 + r];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = row0 + 4 * g + i;
      if (row < B) Y[row * kOut + r] = acc[i] + bias;
    }
  }
}

// ---------------------------------------------------------------------------
// Training: forward, MSE, backward for 64 samples per workgroup (16 per wave);
// weight gradients are products over the workgroup's samples and are added to
// the FP32 gradient buffer with atomics.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float col_sum16(float v) {
  // sum over the four lane groups that hold the same column
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// dW[in][out] (+)= sum_s ActT[in][s] DltT[out][s] over the 64 samples.
template <int NM, int NN>
__device__ __forceinline__ void weight_grad(const uint16_t* act_t, const uint16_t* dlt_t,
                                            float* __restrict__ gW, int out_dim, int wave,
                                            int r, int g) {
  for (int blk = wave; blk < NM * NN; blk += 4) {
    const int mb = blk / NN, nb = blk % NN;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < 2; ++kc)
      acc = mfma(ld8(act_t + (16 * mb + r) * kTs + 32 * kc + 8 * g),
                 ld8(dlt_t + (16 * nb + r) * kTs + 32 * kc + 8 * g), acc);
    const int col = 16 * nb + r;
    if (col < out_dim) {
#pragma unroll
      for (int i = 0; i < 4; ++i) unsafeAtomicAdd(gW + (16 * mb + 4 * g + i) * out_dim + col, acc[i]);
    }
  }
}

__global__ void __launch_bounds__(256) mlp_train_kernel(const uint16_t* __restrict__ X,
                                                        const float* __restrict__ T, int64_t B,
                                                        MlpWeights w,
                                                        const float* __restrict__ p,
                                                        float* __restrict__ grad,
                                                        double* __restrict__ loss_sum) {
  __shared__ __attribute__((aligned(16))) uint16_t xt[kIn * kTs];
  __shared__ __attribute__((aligned(16))) uint16_t h1t[kH * kTs];
  __shared__ __attribute__((aligned(16))) uint16_t h2t[kH * kTs];
  __shared__ __attribute__((aligned(16))) uint16_t dt[kH * kTs];
  __shared__ __attribute__((aligned(16))) uint16_t dyt[16 * kTs];
  __shared__ __attribute__((aligned(16))) uint16_t scr[4][16 * kLd];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int r = lane & 15, g = lane >> 4;
  const int64_t base = (int64_t)blockIdx.x * 64;
  const int64_t row0 = base + 16 * wave;
  const int s0 = 16 * wave;  // this wave's first sample within the workgroup
  const float dscale = 2.f / (float)(B * kOut);

  // X^T of the workgroup's samples (rows beyond B repeat the last row; their
  // upstream gradient is zero, so they contribute nothing)
  for (int e = tid; e < 64 * kIn; e += 256) {
    const int s = e / kIn, k = e % kIn;
    const int64_t row = min(base + s, B - 1);
    xt[k * kTs + s] = X[row * kIn + k];
  }
  const int64_t xrow = min(row0 + r, B - 1);
  uint16_t* h = scr[wave];

  // ---- forward
  f32x4 z1[kH / 16], z2[kH / 16];
#pragma unroll
  for (int nb = 0; nb < kH / 16; ++nb) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < kIn / 32; ++kc)
      acc = mfma(ld8(X + xrow * kIn + 32 * kc + 8 * g), ld8(w.w1t + (16 * nb + r) * kIn + 32 * kc + 8 * g), acc);
    const float bias = p[kOffB1 + 16 * nb + r];
    uint16_t hv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      z1[nb][i] = acc[i] + bias;
      hv[i] = f2bf(gelu(z1[nb][i]));
      h[(4 * g + i) * kLd + 16 * nb + r] = hv[i];
    }
    *reinterpret_cast<uint2*>(h1t + (16 * nb + r) * kTs + s0 + 4 * g) =
        make_uint2(hv[0] | ((uint32_t)hv[1] << 16), hv[2] | ((uint32_t)hv[3] << 16));
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int nb = 0; nb < kH / 16; ++nb) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < kH / 32; ++kc)
      acc = mfma(ld8(h + r * kLd + 32 * kc + 8 * g), ld8(w.w2t + (16 * nb + r) * kH + 32 * kc + 8 * g), acc);
    z2[nb] = acc;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int nb = 0; nb < kH / 16; ++nb) {
    const float bias = p[kOffB2 + 16 * nb + r];
    uint16_t hv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      z2[nb][i] += bias;
      hv[i] = f2bf(gelu(z2[nb][i]));
      h[(4 * g + i) * kLd + 16 * nb + r] = hv[i];
    }
    *reinterpret_cast<uint2*>(h2t + (16 * nb + r) * kTs + s0 + 4 * g) =
        make_uint2(hv[0] | ((uint32_t)hv[1] << 16), hv[2] | ((uint32_t)hv[3] << 16));
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  f32x4 y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kc = 0; kc < kH / 32; ++kc)
    y = mfma(ld8(h + r * kLd + 32 * kc + 8 * g), ld8(w.w3t + r * kH + 32 * kc + 8 * g), y);

  // ---- loss and dY (rows beyond B and padded columns get zero)
  float dy[4];
  double lsum = 0.0;
  {
    const float bias = r < kOut ? p[kOffB3 + r] : 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = row0 + 4 * g + i;
      const bool ok = r < kOut && row < B;
      const float d = ok ? (y[i] + bias) - T[row * kOut + r] : 0.f;
      lsum += (double)d * (double)d;
      dy[i] = dscale * d;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // dY row-major [16][32] (columns >= 10 zero) in the scratch tile, and dY^T
  {
    uint16_t dv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dv[i] = f2bf(dy[i]);
      h[(4 * g + i) * kLd + r] = dv[i];
      h[(4 * g + i) * kLd + 16 + r] = 0;
    }
    *reinterpret_cast<uint2*>(dyt + r * kTs + s0 + 4 * g) =
        make_uint2(dv[0] | ((uint32_t)dv[1] << 16), dv[2] | ((uint32_t)dv[3] << 16));
    float cs = col_sum16(dy[0] + dy[1] + dy[2] + dy[3]);
    if (g == 0 && r < kOut) unsafeAtomicAdd(grad + kOffB3 + r, cs);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
  if (lane == 0 && loss_sum) atomicAdd(loss_sum, lsum);
  __syncthreads();  // xt, h1t, h2t, dyt complete

  // ---- dW3 = H2^T dY
  weight_grad<kH / 16, 1>(h2t, dyt, grad + kOffW3, kOut, wave, r, g);

  // ---- dZ2 = (dY W3^T) * gelu'(Z2)
  f32x4 dz[kH / 16];
#pragma unroll
  for (int nb = 0; nb < kH / 16; ++nb) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma(ld8(h + r * kLd + 8 * g), ld8(w.w3p + (16 * nb + r) * 32 + 8 * g), acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) dz[nb][i] = acc[i] * gelu_grad(z2[nb][i]);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int nb = 0; nb < kH / 16; ++nb) {
    uint16_t dv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dv[i] = f2bf(dz[nb][i]);
      h[(4 * g + i) * kLd + 16 * nb + r] = dv[i];
    }
    *reinterpret_cast<uint2*>(dt + (16 * nb + r) * kTs + s0 + 4 * g) =
        make_uint2(dv[0] | ((uint32_t)dv[1] << 16), dv[2] | ((uint32_t)dv[3] << 16));
    const float cs = col_sum16(dz[nb][0] + dz[nb][1] + dz[nb][2] + dz[nb][3]);
    if (g == 0) unsafeAtomicAdd(grad + kOffB2 + 16 * nb + r, cs);
  }
  __syncthreads();  // dZ2^T complete

  // ---- dW2 = H1^T dZ2
  weight_grad<kH / 16, kH / 16>(h1t, dt, grad + kOffW2, kH, wave, r, g);

  // ---- dZ1 = (dZ2 W2^T) * gelu'(Z1)
#pragma unroll
  for (int nb = 0; nb < kH / 16; ++nb) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < kH / 32; ++kc)
      acc = mfma(ld8(h + r * kLd + 32 * kc + 8 * g), ld8(w.w2 + (16 * nb + r) * kH + 32 * kc + 8 * g), acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) dz[nb][i] = acc[i] * gelu_grad(z1[nb][i]);
  }
  __syncthreads();  // every wave is done reading dZ2^T
#pragma unroll
  for (int nb = 0; nb < kH / 16; ++nb) {
    uint16_t dv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) dv[i] = f2bf(dz[nb][i]);
    *reinterpret_cast<uint2*>(dt + (16 * nb + r) * kTs + s0 + 4 * g) =
        make_uint2(dv[0] | ((uint32_t)dv[1] << 16), dv[2] | ((uint32_t)dv[3] << 16));
    const float cs = col_sum16(dz[nb][0] + dz[nb][1] + dz[nb][2] + dz[nb][3]);
    if (g == 0) unsafeAtomicAdd(grad + kOffB1 + 16 * nb + r, cs);
  }
  __syncthreads();  // dZ1^T complete

  // ---- dW1 = X^T dZ1
  weight_grad<kIn / 16, kH / 16>(xt, dt, grad + kOffW1, kH, wave, r, g);
}

__global__ void zero_kernel(float* __restrict__ a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.f;
}

}  // namespace

gpf_status mlp_convert(const float* params, MlpWeights w, hipStream_t s) {
  hipLaunchKernelGGL(mlp_convert_kernel, dim3((kH * kH + 255) / 256), dim3(256), 0, s, params, w);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

gpf_status mlp_forward(const uint16_t* X, int64_t B, MlpWeights w, const float* params, float* Y,
                       hipStream_t s) {
  const int64_t blocks = (B + 63) / 64;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, B, w, params,
                     Y);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

gpf_status mlp_grad(const uint16_t* X, const float* T, int64_t B, MlpWeights w,
                    const float* params, float* grad, double* loss_sum, hipStream_t s) {
  hipLaunchKernelGGL(zero_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, grad, kParams);
  const int64_t blocks = (B + 63) / 64;
  hipLaunchKernelGGL(mlp_train_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, T, B, w, params,
                     grad, loss_sum);
  GPF_HIP(hipGetLastError());
  return GPF_OK;
}

}  // namespace gpf
