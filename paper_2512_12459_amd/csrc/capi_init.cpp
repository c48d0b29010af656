// C ABI of the initialisation path: photon kNN and features, the learned
// initialiser network (create, parameters, forward, gradient, training step)
// and gpf_init_from_photons.
#include <cstring>
#include <string>

#include "common.h"
#include "mlp.h"

namespace gpf {
gpf_status photon_knn(const float* pos, int64_t n, int k, int* idx, float* d2, hipStream_t s);
gpf_status photon_features(const float* pos, const float* power, int64_t n, const int* idx,
                           const float* d2, uint16_t* X, hipStream_t s);
gpf_status photon_params(const float* pos, const float* power, int64_t n, const float* d2, int k,
                         const float* Y, gpf_field_out out, hipStream_t s);
gpf_status photon_targets(const float* power, int64_t n, const float* d2, int k, const float* quat,
                          const float* ls, const float* rgb, float* T, hipStream_t s);
}  // namespace gpf

using namespace gpf;

namespace {
constexpr int64_t kMaxPhotons = (int64_t)1 << 28;

gpf_status check_photons(const float* pos, int64_t p, int k) {
  if (!pos) return set_error(GPF_ERR_INVALID_ARGUMENT, "photon positions are NULL");
  if (k < 3 || k > 32) return set_error(GPF_ERR_INVALID_ARGUMENT, "k must lie in [3, 32]");
  if (p < k + 1) return set_error(GPF_ERR_INVALID_ARGUMENT, "need at least k + 1 photons");
  if (p > kMaxPhotons) return set_error(GPF_ERR_CAPACITY, "more than 2^28 photons");
  return GPF_OK;
}
}  // namespace

extern "C" {

int64_t gpf_mlp_num_params(void) { return kParams; }

gpf_status gpf_mlp_create(gpf_mlp** out) {
  if (!out) return set_error(GPF_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  gpf_mlp* m = new gpf_mlp();
  GPF_HIP(hipGetDevice(&m->device));
  gpf_status st;
  if ((st = dev_alloc((void**)&m->params, kParams * 4, "mlp params")) != GPF_OK ||
      (st = dev_alloc((void**)&m->m, kParams * 4, "mlp adam m")) != GPF_OK ||
      (st = dev_alloc((void**)&m->v, kParams * 4, "mlp adam v")) != GPF_OK ||
      (st = dev_alloc((void**)&m->grad, kParams * 4, "mlp grad")) != GPF_OK ||
      (st = dev_alloc((void**)&m->w16, (size_t)kW16Elems * 2, "mlp bf16 weights")) != GPF_OK) {
    gpf_mlp_destroy(m);
    return st;
  }
  m->w.w1t = m->w16;
  m->w.w2t = m->w.w1t + kH * kIn;
  m->w.w2 = m->w.w2t + kH * kH;
  m->w.w3t = m->w.w2 + kH * kH;
  m->w.w3p = m->w.w3t + 16 * kH;
  hipError_t e = hipMemset(m->params, 0, kParams * 4);
  if (e == hipSuccess) e = hipMemset(m->m, 0, kParams * 4);
  if (e == hipSuccess) e = hipMemset(m->v, 0, kParams * 4);
  if (e == hipSuccess) e = hipMemset(m->w16, 0, (size_t)kW16Elems * 2);
  if (e != hipSuccess) {
    gpf_mlp_destroy(m);
    return hip_fail(e, "mlp init");
  }
  *out = m;
  return GPF_OK;
}

void gpf_mlp_destroy(gpf_mlp* m) {
  if (!m) return;
  dev_free(m->params, kParams * 4);
  dev_free(m->m, kParams * 4);
  dev_free(m->v, kParams * 4);
  dev_free(m->grad, kParams * 4);
  dev_free(m->w16, (size_t)kW16Elems * 2);
  delete m;
}

gpf_status gpf_mlp_set_params(gpf_mlp* m, const float* params) {
  if (!m || !params) return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  GPF_HIP(hipMemcpy(m->params, params, kParams * 4, hipMemcpyHostToDevice));
  GPF_HIP(hipMemset(m->m, 0, kParams * 4));
  GPF_HIP(hipMemset(m->v, 0, kParams * 4));
  m->step = 0;
  gpf_status st = mlp_convert(m->params, m->w, nullptr);
  if (st != GPF_OK) return st;
  GPF_HIP(hipDeviceSynchronize());
  return GPF_OK;
}

gpf_status gpf_mlp_get_params(const gpf_mlp* m, float* params) {
  if (!m || !params) return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  GPF_HIP(hipDeviceSynchronize());
  GPF_HIP(hipMemcpy(params, m->params, kParams * 4, hipMemcpyDeviceToHost));
  return GPF_OK;
}

gpf_status gpf_mlp_forward(const gpf_mlp* m, const uint16_t* X, int64_t b, float* Y, void* stream) {
  if (!m || !X || !Y) return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  if (b < 1 || b > ((int64_t)1 << 31) - 64) return set_error(GPF_ERR_INVALID_ARGUMENT, "bad batch size");
  return mlp_forward(X, b, m->w, m->params, Y, (hipStream_t)stream);
}

gpf_status gpf_mlp_gradient(gpf_mlp* m, const uint16_t* X, const float* T, int64_t b, float* grad,
                            double* loss_sum, void* stream) {
  if (!m || !X || !T || !grad) return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  if (b < 1 || b > ((int64_t)1 << 31) - 64) return set_error(GPF_ERR_INVALID_ARGUMENT, "bad batch size");
  hipStream_t s = (hipStream_t)stream;
  gpf_status st = mlp_grad(X, T, b, m->w, m->params, m->grad, loss_sum, s);
  if (st != GPF_OK) return st;
  GPF_HIP(hipMemcpyAsync(grad, m->grad, kParams * 4, hipMemcpyDeviceToDevice, s));
  return GPF_OK;
}

gpf_status gpf_mlp_train_step(gpf_mlp* m, const uint16_t* X, const float* T, int64_t b, float lr,
                              double* loss_sum, void* stream) {
  if (!m || !X || !T) return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  if (b < 1 || b > ((int64_t)1 << 31) - 64) return set_error(GPF_ERR_INVALID_ARGUMENT, "bad batch size");
  if (!(lr >= 0.f)) return set_error(GPF_ERR_INVALID_ARGUMENT, "bad learning rate");
  hipStream_t s = (hipStream_t)stream;
  gpf_status st = mlp_grad(X, T, b, m->w, m->params, m->grad, loss_sum, s);
  if (st != GPF_OK) return st;
  m->step += 1;
  st = launch_adam(m->params, m->grad, m->m, m->v, kParams, lr, 0.9f, 0.999f, 1e-8f, m->step,
                   nullptr, s);
  if (st != GPF_OK) return st;
  return mlp_convert(m->params, m->w, s);
}

gpf_status gpf_photon_knn(const float* pos, int64_t p, int k, int32_t* idx, float* d2, void* stream) {
  gpf_status st = check_photons(pos, p, k);
  if (st != GPF_OK) return st;
  if (!idx || !d2) return set_error(GPF_ERR_INVALID_ARGUMENT, "output is NULL");
  return photon_knn(pos, p, k, idx, d2, (hipStream_t)stream);
}

gpf_status gpf_photon_features(const float* pos, const float* power, int64_t p, const int32_t* idx,
                               const float* d2, uint16_t* X, void* stream) {
  if (!pos || !power || !idx || !d2 || !X) return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  if (p < 1 || p > kMaxPhotons) return set_error(GPF_ERR_INVALID_ARGUMENT, "bad photon count");
  return photon_features(pos, power, p, idx, d2, X, (hipStream_t)stream);
}

gpf_status gpf_mlp_targets(const float* power, int64_t p, const float* d2, int k,
                           const gpf_field* fitted, float* T, void* stream) {
  if (!power || !d2 || !fitted || !T || !fitted->quat || !fitted->log_scale || !fitted->rgb)
    return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  if (k < 3 || k > 32) return set_error(GPF_ERR_INVALID_ARGUMENT, "k must lie in [3, 32]");
  if (fitted->n != p || p < 1) return set_error(GPF_ERR_INVALID_ARGUMENT, "field size differs from p");
  return photon_targets(power, p, d2, k, fitted->quat, fitted->log_scale, fitted->rgb, T,
                        (hipStream_t)stream);
}

gpf_status gpf_init_from_photons(const float* pos, const float* power, int64_t p, int k,
                                 const gpf_mlp* mlp, gpf_field_out* out, void* stream) {
  gpf_status st = check_photons(pos, p, k);
  if (st != GPF_OK) return st;
  if (!power) return set_error(GPF_ERR_INVALID_ARGUMENT, "photon power is NULL");
  if (!out || !out->mu || !out->quat || !out->log_scale || !out->rgb)
    return set_error(GPF_ERR_INVALID_ARGUMENT, "output field has a NULL array");
  if (mlp && k != 16) return set_error(GPF_ERR_INVALID_ARGUMENT, "the learned initialiser needs k = 16");
  hipStream_t s = (hipStream_t)stream;
  int* idx = nullptr;
  float* d2 = nullptr;
  uint16_t* X = nullptr;
  float* Y = nullptr;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    dev_free(idx, p * k * 4);
    dev_free(d2, p * k * 4);
    dev_free(X, p * kIn * 2);
    dev_free(Y, p * kOut * 4);
  };
  if ((st = dev_alloc((void**)&idx, p * k * 4, "knn index")) != GPF_OK ||
      (st = dev_alloc((void**)&d2, p * k * 4, "knn distance")) != GPF_OK) {
    cleanup();
    return st;
  }
  st = photon_knn(pos, p, k, idx, d2, s);
  if (st == GPF_OK && mlp) {
    if ((st = dev_alloc((void**)&X, p * kIn * 2, "features")) == GPF_OK &&
        (st = dev_alloc((void**)&Y, p * kOut * 4, "network outputs")) == GPF_OK &&
        (st = photon_features(pos, power, p, idx, d2, X, s)) == GPF_OK)
      st = mlp_forward(X, p, mlp->w, mlp->params, Y, s);
  }
  if (st == GPF_OK) st = photon_params(pos, power, p, d2, k, Y, *out, s);
  cleanup();
  return st;
}

}  // extern "C"
