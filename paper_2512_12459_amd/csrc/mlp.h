// Learned initialiser network: sizes, parameter layout and launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gpf.h"

namespace gpf {

constexpr int kIn = 96;    // 16 neighbours x (offset 3 + log power ratio 3)
constexpr int kH = 128;    // hidden width
constexpr int kOut = 10;   // quaternion delta 4, log-scale delta 3, log-flux delta 3
// FP32 master parameters, W[in][out] row-major: W1 b1 W2 b2 W3 b3
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kIn * kH;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kH * kOut;
constexpr int kParams = kOffB3 + kOut;  // 30218

// bfloat16 weight copies laid out for 16-byte MFMA fragment loads.
struct MlpWeights {
  uint16_t* w1t;  // [128][96]  W1^T
  uint16_t* w2t;  // [128][128] W2^T
  uint16_t* w2;   // [128][128] W2
  uint16_t* w3t;  // [16][128]  W3^T, rows >= 10 zero
  uint16_t* w3p;  // [128][32]  W3, columns >= 10 zero
};
constexpr int kW16Elems = kH * kIn + 2 * kH * kH + 16 * kH + kH * 32;

gpf_status mlp_convert(const float* params, MlpWeights w, hipStream_t s);
gpf_status mlp_forward(const uint16_t* X, int64_t B, MlpWeights w, const float* params, float* Y,
                       hipStream_t s);
gpf_status mlp_grad(const uint16_t* X, const float* T, int64_t B, MlpWeights w,
                    const float* params, float* grad, double* loss_sum, hipStream_t s);

}  // namespace gpf

struct gpf_mlp {
  int device = 0;
  float* params = nullptr;  // [kParams] FP32 masters
  float* m = nullptr;       // Adam moments
  float* v = nullptr;
  float* grad = nullptr;    // [kParams] gradient scratch
  uint16_t* w16 = nullptr;  // bfloat16 copies (one allocation)
  gpf::MlpWeights w{};
  int64_t step = 0;
};
