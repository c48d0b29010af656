// C ABI entry points: argument validation, handle lifetime, error reporting.
// Every compute step runs in the HIP kernels of the sibling .hip files.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "common.h"

namespace gpf {

static thread_local std::string g_last_error;

gpf_status set_error(gpf_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

gpf_status hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    return set_error(GPF_ERR_OUT_OF_MEMORY, std::string(what) + ": " + hipGetErrorString(e));
  }
  return set_error(GPF_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Optional cap on the bytes this library holds on the device at once, read
// from GPF_DEVICE_BYTES_LIMIT; lets tests force the out-of-memory path.
static std::mutex g_mem_mu;
static size_t g_mem_used = 0;

static size_t byte_limit() {
  const char* s = std::getenv("GPF_DEVICE_BYTES_LIMIT");
  if (!s || !*s) return SIZE_MAX;
  return (size_t)std::strtoull(s, nullptr, 10);
}

gpf_status dev_alloc(void** p, size_t bytes, const char* what) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    if (g_mem_used + bytes > byte_limit())
      return set_error(GPF_ERR_OUT_OF_MEMORY,
                       std::string(what) + ": device byte budget exceeded");
    g_mem_used += bytes;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    g_mem_used -= bytes;
    *p = nullptr;
    return hip_fail(e, what);
  }
  return GPF_OK;
}

void dev_free(void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  if (bytes == 0) bytes = 16;
  std::lock_guard<std::mutex> lk(g_mem_mu);
  g_mem_used -= bytes;
}

static bool field_ok(const gpf_field* f, std::string* why) {
  if (!f) { *why = "field is NULL"; return false; }
  if (f->n < 1 || f->n > ((int64_t)1 << 30) - 1) { *why = "field n out of range [1, 2^30-1]"; return false; }
  if (!f->mu || !f->quat || !f->log_scale || !f->rgb) { *why = "field has a NULL array"; return false; }
  return true;
}

static gpf_status check_grid_use(const gpf_grid* g, const gpf_field* f, const float* x, int64_t q,
                                 bool hybrid = false) {
  if (!g) return set_error(GPF_ERR_INVALID_ARGUMENT, "grid is NULL");
  if ((g->ball > 0.f) != hybrid)
    return set_error(GPF_ERR_INVALID_ARGUMENT, hybrid ? "grid was built for the truncated query"
                                                      : "grid was built for the hybrid query");
  std::string why;
  if (!field_ok(f, &why)) return set_error(GPF_ERR_INVALID_ARGUMENT, why);
  if (!x) return set_error(GPF_ERR_INVALID_ARGUMENT, "x is NULL");
  if (g->mu != f->mu || g->quat != f->quat || g->log_scale != f->log_scale ||
      g->rgb != f->rgb || g->n != f->n)
    return set_error(GPF_ERR_STALE, "field differs from the one the grid was built from");
  if (g->qs_gen != g->qs->gen)
    return set_error(GPF_ERR_STALE, "query set was re-binned after the grid was built");
  if (x != g->qs->x_user || q != g->qs->q)
    return set_error(GPF_ERR_STALE, "query points differ from the binned query set");
  return GPF_OK;
}

}  // namespace gpf

using namespace gpf;

extern "C" {

const char* gpf_last_error(void) { return g_last_error.c_str(); }
const char* gpf_version(void) { return "gpf 0.1 gfx950"; }

gpf_status gpf_bin_queries(const float* x, int64_t q, float cell_size, void* stream,
                           gpf_queries** out) {
  if (!out) return set_error(GPF_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (!x) return set_error(GPF_ERR_INVALID_ARGUMENT, "x is NULL");
  if (q < 1 || q > (int64_t)INT32_MAX - 64)
    return set_error(GPF_ERR_INVALID_ARGUMENT, "q out of range [1, 2^31-65]");
  if (!(cell_size > 0.f) || !(cell_size < 1e30f))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "cell_size must be positive and finite");
  gpf_queries* qs = new gpf_queries();
  GPF_HIP(hipGetDevice(&qs->device));
  gpf_status st = launch_bin_queries(x, q, cell_size, false, (hipStream_t)stream, qs);
  if (st != GPF_OK) {
    gpf_queries_destroy(qs);
    return st;
  }
  *out = qs;
  return GPF_OK;
}

gpf_status gpf_rebin_queries(gpf_queries* qs, const float* x, int64_t q, float cell_size,
                             void* stream) {
  if (!qs) return set_error(GPF_ERR_INVALID_ARGUMENT, "query set is NULL");
  if (!x) return set_error(GPF_ERR_INVALID_ARGUMENT, "x is NULL");
  if (q < 1 || q > (int64_t)INT32_MAX - 64)
    return set_error(GPF_ERR_INVALID_ARGUMENT, "q out of range [1, 2^31-65]");
  if (!(cell_size > 0.f) || !(cell_size < 1e30f))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "cell_size must be positive and finite");
  int dev = 0;
  GPF_HIP(hipGetDevice(&dev));
  if (dev != qs->device)
    return set_error(GPF_ERR_INVALID_ARGUMENT, "query set belongs to another device");
  return launch_bin_queries(x, q, cell_size, true, (hipStream_t)stream, qs);
}

void gpf_queries_destroy(gpf_queries* qs) {
  if (!qs) return;
  release_bin_outputs(qs);
  release_bin_scratch(qs);
  delete qs;
}

gpf_status gpf_queries_info(const gpf_queries* qs, int64_t* q, int64_t* cells, int64_t* tiles,
                            size_t* device_bytes) {
  if (!qs) return set_error(GPF_ERR_INVALID_ARGUMENT, "query set is NULL");
  if (q) *q = qs->q;
  if (cells) *cells = qs->ncells;
  if (tiles) *tiles = qs->ntiles;
  if (device_bytes) *device_bytes = qs->bytes;
  return GPF_OK;
}

gpf_status gpf_build_grid(const gpf_field* f, float cutoff, const gpf_queries* qs, void* stream,
                          gpf_grid** grid) {
  if (!grid) return set_error(GPF_ERR_INVALID_ARGUMENT, "grid out-pointer is NULL");
  std::string why;
  if (!field_ok(f, &why)) return set_error(GPF_ERR_INVALID_ARGUMENT, why);
  if (!qs) return set_error(GPF_ERR_INVALID_ARGUMENT, "query set is NULL");
  if (!(cutoff > 0.f) || !(cutoff <= 16.f))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "cutoff must lie in (0, 16]");
  if (qs->q < 1) return set_error(GPF_ERR_INVALID_ARGUMENT, "query set holds no binning");
  gpf_grid* g = *grid;
  bool fresh = (g == nullptr);
  if (!fresh && g->qs != qs)
    return set_error(GPF_ERR_STALE, "grid was built for a different query set");
  if (!fresh && g->ball > 0.f)
    return set_error(GPF_ERR_INVALID_ARGUMENT, "grid was built for the hybrid query");
  if (fresh) g = new gpf_grid();
  g->qs = qs;
  g->mu = f->mu;
  g->quat = f->quat;
  g->log_scale = f->log_scale;
  g->rgb = f->rgb;
  g->n = f->n;
  g->cutoff = cutoff;
  gpf_status st = launch_build_grid(g, (hipStream_t)stream);
  if (st != GPF_OK) {
    if (fresh) gpf_grid_destroy(g);
    else g->n = -1;  // poison: the handle no longer matches any field
    return st;
  }
  g->qs_gen = qs->gen;
  *grid = g;
  return GPF_OK;
}

void gpf_grid_destroy(gpf_grid* g) {
  if (!g) return;
  dev_free(g->rec, g->rec_cap * sizeof(PrimRec));
  dev_free(g->ext, g->rec_cap * sizeof(float4));
  dev_free(g->prim_off, (size_t)g->prim_off_len * sizeof(int));
  dev_free(g->cell_start, g->cell_start_cap * sizeof(int));
  dev_free(g->keys, g->cap * sizeof(int));
  dev_free(g->vals, g->cap * sizeof(int));
  dev_free(g->keys_sorted, g->cap * sizeof(int));
  dev_free(g->cell_prims, g->cap * sizeof(int));
  dev_free(g->cell_recs, g->cell_recs_cap * sizeof(PrimRec));
  dev_free(g->sort_tmp, g->sort_tmp_bytes);
  dev_free(g->grad_rows, g->grad_cap * sizeof(float4) * 4);
  dev_free(g->surv, (size_t)g->surv_groups * kSurvPerGroup * sizeof(int));
  dev_free(g->surv_count, (size_t)g->surv_groups * sizeof(int));
  free_centre_grid(g);
  if (g->readback) (void)hipHostFree(g->readback);
  delete g;
}

gpf_status gpf_grid_info(const gpf_grid* g, int64_t* entries, size_t* device_bytes) {
  if (!g) return set_error(GPF_ERR_INVALID_ARGUMENT, "grid is NULL");
  if (entries) *entries = g->entries;
  if (device_bytes)
    *device_bytes = g->bytes + (size_t)g->grad_cap * 4 * sizeof(float4) +
                    (size_t)g->surv_groups * (kSurvPerGroup + 1) * sizeof(int);
  return GPF_OK;
}

gpf_status gpf_eval_radiance(const gpf_grid* g, const gpf_field* f, const float* x, int64_t q,
                             float* L, void* stream) {
  gpf_status st = check_grid_use(g, f, x, q);
  if (st != GPF_OK) return st;
  if (!L) return set_error(GPF_ERR_INVALID_ARGUMENT, "L is NULL");
  return launch_eval_fwd(g, L, (hipStream_t)stream);
}

gpf_status gpf_eval_radiance_backward(const gpf_grid* g, const gpf_field* f, const float* x,
                                      int64_t q, const float* dL, gpf_field_grad* grad,
                                      void* stream) {
  gpf_status st = check_grid_use(g, f, x, q);
  if (st != GPF_OK) return st;
  if (!dL) return set_error(GPF_ERR_INVALID_ARGUMENT, "dL is NULL");
  if (!grad || !grad->mu || !grad->quat || !grad->log_scale || !grad->rgb)
    return set_error(GPF_ERR_INVALID_ARGUMENT, "gradient buffers must be non-NULL");
  const void* fp[4] = {f->mu, f->quat, f->log_scale, f->rgb};
  const void* gp[4] = {grad->mu, grad->quat, grad->log_scale, grad->rgb};
  for (auto a : fp)
    for (auto b : gp)
      if (a == b) return set_error(GPF_ERR_INVALID_ARGUMENT, "gradient buffer aliases the field");
  return launch_eval_bwd(g, dL, grad, (hipStream_t)stream);
}

gpf_status gpf_eval_radiance_backward_noalloc(const gpf_grid* g, const gpf_field* f,
                                              const float* x, int64_t q, const float* dL,
                                              gpf_field_grad* grad, void* stream) {
  gpf_status st = check_grid_use(g, f, x, q);
  if (st != GPF_OK) return st;
  if (!dL) return set_error(GPF_ERR_INVALID_ARGUMENT, "dL is NULL");
  if (!grad || !grad->mu || !grad->quat || !grad->log_scale || !grad->rgb)
    return set_error(GPF_ERR_INVALID_ARGUMENT, "gradient buffers must be non-NULL");
  const void* fp[4] = {f->mu, f->quat, f->log_scale, f->rgb};
  const void* gp[4] = {grad->mu, grad->quat, grad->log_scale, grad->rgb};
  for (auto a : fp)
    for (auto b : gp)
      if (a == b) return set_error(GPF_ERR_INVALID_ARGUMENT, "gradient buffer aliases the field");
  return launch_eval_bwd_noalloc(g, dL, grad, (hipStream_t)stream);
}

gpf_status gpf_fit_pass(const gpf_grid* g, const gpf_field* f, const float* x, int64_t q,
                        const float* T, float* L, double* loss_sum, gpf_field_grad* grad,
                        void* stream) {
  gpf_status st = check_grid_use(g, f, x, q);
  if (st != GPF_OK) return st;
  if (!T || !L || !loss_sum)
    return set_error(GPF_ERR_INVALID_ARGUMENT, "T, L and loss_sum must be non-NULL");
  if (T == L) return set_error(GPF_ERR_INVALID_ARGUMENT, "L aliases T");
  if (!grad || !grad->mu || !grad->quat || !grad->log_scale || !grad->rgb)
    return set_error(GPF_ERR_INVALID_ARGUMENT, "gradient buffers must be non-NULL");
  const void* fp[4] = {f->mu, f->quat, f->log_scale, f->rgb};
  const void* gp[4] = {grad->mu, grad->quat, grad->log_scale, grad->rgb};
  for (auto a : fp)
    for (auto b : gp)
      if (a == b) return set_error(GPF_ERR_INVALID_ARGUMENT, "gradient buffer aliases the field");
  return launch_fit_pass(g, T, L, loss_sum, grad, (hipStream_t)stream);
}

gpf_status gpf_build_grid_hybrid(const gpf_field* f, float r, int k_min, const gpf_queries* qs,
                                 void* stream, gpf_grid** grid) {
  if (!grid) return set_error(GPF_ERR_INVALID_ARGUMENT, "grid out-pointer is NULL");
  std::string why;
  if (!field_ok(f, &why)) return set_error(GPF_ERR_INVALID_ARGUMENT, why);
  if (!qs) return set_error(GPF_ERR_INVALID_ARGUMENT, "query set is NULL");
  if (!(r > 0.f) || !std::isfinite(r)) return set_error(GPF_ERR_INVALID_ARGUMENT, "r must be positive and finite");
  if (k_min < 1 || k_min > 8) return set_error(GPF_ERR_INVALID_ARGUMENT, "k_min must lie in [1, 8]");
  if (qs->q < 1) return set_error(GPF_ERR_INVALID_ARGUMENT, "query set holds no binning");
  gpf_grid* g = *grid;
  bool fresh = (g == nullptr);
  if (!fresh && g->qs != qs)
    return set_error(GPF_ERR_STALE, "grid was built for a different query set");
  if (!fresh && !(g->ball > 0.f))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "grid was built for the truncated query");
  if (fresh) g = new gpf_grid();
  g->qs = qs;
  g->mu = f->mu;
  g->quat = f->quat;
  g->log_scale = f->log_scale;
  g->rgb = f->rgb;
  g->n = f->n;
  g->cutoff = 3.f;
  g->ball = r;
  g->k_min = k_min;
  gpf_status st = launch_build_grid(g, (hipStream_t)stream);
  if (st != GPF_OK) {
    if (fresh) gpf_grid_destroy(g);
    else g->n = -1;  // poison: the handle no longer matches any field
    return st;
  }
  g->qs_gen = qs->gen;
  *grid = g;
  return GPF_OK;
}

gpf_status gpf_eval_hybrid(const gpf_grid* g, const gpf_field* f, const float* x, int64_t q,
                           float eps, float* L, float* Z, int* count, void* stream) {
  gpf_status st = check_grid_use(g, f, x, q, true);
  if (st != GPF_OK) return st;
  if (!L || !Z || !count) return set_error(GPF_ERR_INVALID_ARGUMENT, "L, Z and count must be non-NULL");
  if (!(eps > 0.f) || !std::isfinite(eps)) return set_error(GPF_ERR_INVALID_ARGUMENT, "eps must be positive and finite");
  return launch_hybrid_fwd(g, eps, L, Z, count, (hipStream_t)stream);
}

gpf_status gpf_eval_hybrid_backward(const gpf_grid* g, const gpf_field* f, const float* x,
                                    int64_t q, float eps, const float* L, const float* Z,
                                    const int* count, const float* dL, gpf_field_grad* grad,
                                    void* stream) {
  gpf_status st = check_grid_use(g, f, x, q, true);
  if (st != GPF_OK) return st;
  if (!L || !Z || !count || !dL) return set_error(GPF_ERR_INVALID_ARGUMENT, "L, Z, count and dL must be non-NULL");
  if (!(eps > 0.f) || !std::isfinite(eps)) return set_error(GPF_ERR_INVALID_ARGUMENT, "eps must be positive and finite");
  if (!grad || !grad->mu || !grad->quat || !grad->log_scale || !grad->rgb)
    return set_error(GPF_ERR_INVALID_ARGUMENT, "gradient buffers must be non-NULL");
  const void* fp[4] = {f->mu, f->quat, f->log_scale, f->rgb};
  const void* gp[4] = {grad->mu, grad->quat, grad->log_scale, grad->rgb};
  for (auto a : fp)
    for (auto b : gp)
      if (a == b) return set_error(GPF_ERR_INVALID_ARGUMENT, "gradient buffer aliases the field");
  return launch_hybrid_bwd(g, eps, L, Z, count, dL, grad, (hipStream_t)stream);
}

gpf_status gpf_count_pairs(const gpf_grid* g, const gpf_field* f, int64_t* pairs, void* stream) {
  if (!g) return set_error(GPF_ERR_INVALID_ARGUMENT, "grid is NULL");
  if (!pairs) return set_error(GPF_ERR_INVALID_ARGUMENT, "pairs is NULL");
  gpf_status st = check_grid_use(g, f, g->qs->x_user, g->qs->q);
  if (st != GPF_OK) return st;
  unsigned long long* d = nullptr;
  st = dev_alloc((void**)&d, sizeof(*d), "count_pairs");
  if (st != GPF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  unsigned long long h = 0;
  st = launch_count_pairs(g, d, s);
  if (st == GPF_OK) {
    hipError_t e = hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "count_pairs readback");
  }
  dev_free(d, sizeof(*d));
  if (st == GPF_OK) *pairs = (int64_t)h;
  return st;
}

gpf_status gpf_trace_photons(int64_t n_paths, uint64_t seed, int max_events, float light_lo,
                             float light_hi, int sphere, float* pos, float* power, int* surface,
                             void* stream) {
  if (n_paths < 1 || n_paths >= ((int64_t)1 << 31))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "n_paths must lie in [1, 2^31 - 1]");
  if (max_events < 1 || max_events > 16)
    return set_error(GPF_ERR_INVALID_ARGUMENT, "max_events must lie in [1, 16]");
  if (!(light_lo >= 0.f) || !(light_hi <= 1.f) || !(light_lo <= light_hi))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "light square must satisfy 0 <= lo <= hi <= 1");
  if (!pos || !power || !surface) return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL output");
  if (sphere < 0 || sphere > 2) return set_error(GPF_ERR_INVALID_ARGUMENT, "sphere must be 0, 1 or 2");
  return launch_trace_photons(n_paths, seed, max_events, light_lo, light_hi, sphere, pos,
                              power, surface, (hipStream_t)stream);
}

gpf_status gpf_compact_photons(const float* pos, const float* power, const int* surface, int64_t m,
                               float* out_pos, float* out_power, int* out_surface, int64_t* out_slot,
                               int64_t capacity, int64_t* count, void* stream) {
  if (!pos || !power || !surface || !out_pos || !out_power || !out_surface || !count)
    return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  if (m < 1 || m >= ((int64_t)1 << 31) - 1)
    return set_error(GPF_ERR_INVALID_ARGUMENT, "m must lie in [1, 2^31 - 2]");
  if (capacity < 0) return set_error(GPF_ERR_INVALID_ARGUMENT, "capacity must be >= 0");
  return compact_photons(pos, power, surface, m, out_pos, out_power, out_surface, out_slot,
                         capacity, count, (hipStream_t)stream);
}

gpf_status gpf_photon_map_build(const float* ppos, const float* ppower, const int* psurface,
                                int64_t np, float r, void* stream, gpf_photon_map** map) {
  if (!ppos || !ppower || !psurface || !map) return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  *map = nullptr;
  if (np < 1 || np >= ((int64_t)1 << 31))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "np must lie in [1, 2^31 - 1]");
  if (!(r > 0.f) || !std::isfinite(r)) return set_error(GPF_ERR_INVALID_ARGUMENT, "r must be positive and finite");
  return photon_map_build(ppos, ppower, psurface, np, r, map, (hipStream_t)stream);
}

gpf_status gpf_photon_map_rebuild(gpf_photon_map* map, const float* ppos, const float* ppower,
                                  const int* psurface, int64_t np, float r, void* stream) {
  if (!map || !ppos || !ppower || !psurface) return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  if (np < 1 || np >= ((int64_t)1 << 31))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "np must lie in [1, 2^31 - 1]");
  if (!(r > 0.f) || !std::isfinite(r)) return set_error(GPF_ERR_INVALID_ARGUMENT, "r must be positive and finite");
  return photon_map_fill(map, ppos, ppower, psurface, np, r, (hipStream_t)stream);
}

void gpf_photon_map_destroy(gpf_photon_map* map) { photon_map_free(map); }

gpf_status gpf_photon_map_gather(const gpf_photon_map* map, const float* x, const int* x_surface,
                                 int64_t q, float weight, int accumulate, float* L, int* count,
                                 void* stream) {
  if (!map || !x || !x_surface || !L) return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  if (q < 1 || q >= ((int64_t)1 << 31))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "q must lie in [1, 2^31 - 1]");
  if (!std::isfinite(weight)) return set_error(GPF_ERR_INVALID_ARGUMENT, "weight must be finite");
  return photon_map_gather(map, x, x_surface, q, weight, accumulate != 0, L, count,
                           (hipStream_t)stream);
}

gpf_status gpf_photon_map_gather_binned(const gpf_photon_map* map, const gpf_queries* queries,
                                        const int* x_surface, float weight, int accumulate,
                                        float* L, int* count, void* stream) {
  if (!map || !queries || !x_surface || !L) return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  if (!std::isfinite(weight)) return set_error(GPF_ERR_INVALID_ARGUMENT, "weight must be finite");
  if (queries->q < 1) return set_error(GPF_ERR_INVALID_ARGUMENT, "query set holds no binning");
  return photon_map_gather_binned(map, queries, x_surface, weight, accumulate != 0, L, count,
                                  (hipStream_t)stream);
}

gpf_status gpf_photon_density(const float* x, const int* x_surface, int64_t q, const float* ppos,
                              const float* ppower, const int* psurface, int64_t np, float r,
                              float weight, int accumulate, float* L, int* count, void* stream) {
  if (!x || !x_surface || !L) return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  if (q < 1 || q >= ((int64_t)1 << 31))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "q must lie in [1, 2^31 - 1]");
  if (!std::isfinite(weight)) return set_error(GPF_ERR_INVALID_ARGUMENT, "weight must be finite");
  gpf_photon_map* m = nullptr;
  gpf_status st = gpf_photon_map_build(ppos, ppower, psurface, np, r, stream, &m);
  if (st != GPF_OK) return st;
  st = photon_map_gather(m, x, x_surface, q, weight, accumulate != 0, L, count, (hipStream_t)stream);
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  photon_map_free(m);
  if (st == GPF_OK && e != hipSuccess) st = hip_fail(e, "density estimate");
  return st;
}

gpf_status gpf_camera_trace(const gpf_camera* cam, int samples, uint64_t seed, int max_depth,
                            float light_lo, float light_hi, int sphere, float* x, float* beta,
                            int* face, float* Le, void* stream) {
  if (!cam || !x || !beta || !face || !Le) return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  if (cam->width < 1 || cam->height < 1) return set_error(GPF_ERR_INVALID_ARGUMENT, "empty image");
  if (samples < 1 || samples > 1024) return set_error(GPF_ERR_INVALID_ARGUMENT, "samples must lie in [1, 1024]");
  if ((int64_t)cam->width * cam->height * samples >= ((int64_t)1 << 31))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "width * height * samples must stay below 2^31");
  if (max_depth < 1 || max_depth > 64) return set_error(GPF_ERR_INVALID_ARGUMENT, "max_depth must lie in [1, 64]");
  if (sphere < 0 || sphere > 2) return set_error(GPF_ERR_INVALID_ARGUMENT, "sphere must be 0, 1 or 2");
  if (!(light_lo >= 0.f) || !(light_hi <= 1.f) || !(light_lo <= light_hi))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "light square must satisfy 0 <= lo <= hi <= 1");
  if (!(cam->vfov_deg > 0.f && cam->vfov_deg < 180.f))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "vfov_deg must lie in (0, 180)");
  double f[3], c[3];
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(cam->eye[a]) || !std::isfinite(cam->target[a]) || !std::isfinite(cam->up[a]))
      return set_error(GPF_ERR_INVALID_ARGUMENT, "camera vectors must be finite");
    f[a] = (double)cam->target[a] - cam->eye[a];
  }
  c[0] = f[1] * cam->up[2] - f[2] * cam->up[1];
  c[1] = f[2] * cam->up[0] - f[0] * cam->up[2];
  c[2] = f[0] * cam->up[1] - f[1] * cam->up[0];
  const double lf = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  const double lu = std::sqrt((double)cam->up[0] * cam->up[0] + (double)cam->up[1] * cam->up[1] +
                              (double)cam->up[2] * cam->up[2]);
  if (!(lf > 0) || !(std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]) > 1e-9 * lf * lu))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "eye equals target or up is parallel to the view");
  return launch_camera_trace(cam, samples, seed, max_depth, light_lo, light_hi, sphere, x, beta, face,
                             Le, (hipStream_t)stream);
}

gpf_status gpf_camera_compose(const float* Le, int64_t n_pix, int samples, const int64_t* slot,
                              const float* beta_c, const float* Lq, int64_t m, float* L_pix,
                              void* stream) {
  if (!Le || !L_pix || (m > 0 && (!slot || !beta_c || !Lq)))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  if (n_pix < 1 || samples < 1 || m < 0 || n_pix * (int64_t)samples >= ((int64_t)1 << 31))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "bad sizes");
  return launch_camera_compose(Le, n_pix, samples, slot, beta_c, Lq, m, L_pix, (hipStream_t)stream);
}

gpf_status gpf_camera_compose_backward(const float* dL_pix, int64_t n_pix, int samples,
                                       const int64_t* slot, const float* beta_c, int64_t m,
                                       float* dLq, void* stream) {
  if (!dL_pix || (m > 0 && (!slot || !beta_c || !dLq)))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  if (n_pix < 1 || samples < 1 || m < 0) return set_error(GPF_ERR_INVALID_ARGUMENT, "bad sizes");
  return launch_camera_compose_backward(dL_pix, n_pix, samples, slot, beta_c, m, dLq,
                                        (hipStream_t)stream);
}

gpf_status gpf_mse_loss(const float* L, const float* T, int64_t q, double* loss_sum, float* dL,
                        void* stream) {
  if (!L || !T || !loss_sum || !dL) return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  if (q < 1) return set_error(GPF_ERR_INVALID_ARGUMENT, "q must be >= 1");
  return launch_mse(L, T, q, loss_sum, dL, (hipStream_t)stream);
}

gpf_status gpf_adam_step(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                         float beta1, float beta2, float eps, int64_t step, const double* guard,
                         void* stream) {
  if (!p || !g || !m || !v) return set_error(GPF_ERR_INVALID_ARGUMENT, "NULL argument");
  if (n < 0) return set_error(GPF_ERR_INVALID_ARGUMENT, "n must be >= 0");
  if (step < 1) return set_error(GPF_ERR_INVALID_ARGUMENT, "step must be >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f))
    return set_error(GPF_ERR_INVALID_ARGUMENT, "bad Adam hyper-parameters");
  if (n == 0) return GPF_OK;
  return launch_adam(p, g, m, v, n, lr, beta1, beta2, eps, step, guard, (hipStream_t)stream);
}

}  // extern "C"
