// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/gpf.h"

namespace gpf {

// Queries per tile: one wave64 evaluates one tile.
constexpr int kTile = 64;
// Tiles per backward group: the backward accumulates each primitive's sums
// over a group of consecutive tiles of one cell before adding them to memory.
#ifndef GPF_GROUP_TILES
#define GPF_GROUP_TILES 2
#endif
constexpr int kGroupTiles = GPF_GROUP_TILES;
// Scale folded into the whitening rows: u' = kappa * u with kappa^2 = log2(e)/2,
// so that exp(-m^2/2) = exp2(-|u'|^2).
constexpr double kKappa2 = 0.72134752044448170368;  // 0.5 * log2(e)

// Primitive record (64 bytes): r0 = {mu, Phi_r}, r1 = {W'_0, Phi_g},
// r2 = {W'_1, Phi_b}, r3 = {W'_2, primitive index as int bits}; W'_k is row k
// of kappa * diag(1/s) R^T.
struct alignas(16) PrimRec {
  float4 r0, r1, r2, r3;
};

// Tile descriptor: queries [start, start+count) of the sorted order, all in
// occupied cell `cell`.
struct alignas(16) TileInfo {
  int start, count, cell, pad;
};

// Group of <= kGroupTiles consecutive tiles of one cell: queries
// [start, start+count), tiles [first_tile, first_tile + ntiles).
struct alignas(16) GroupInfo {
  int start, count, cell, first_tile;
};

}  // namespace gpf

struct gpf_queries {
  int device = 0;
  const float* x_user = nullptr;  // binned buffer (identity check only)
  int64_t q = 0;
  float origin[3] = {0, 0, 0};
  float cell = 0;
  int dims[3] = {0, 0, 0};
  int64_t ncells = 0;   // occupied cells
  int64_t ntiles = 0;
  uint64_t gen = 0;     // bumped by every (re)binning; grids record the value they were built on
  float4* xs = nullptr;          // [q] sorted points (w unused)
  int* perm = nullptr;           // [q] sorted position -> caller index
  int* occ_of_dense = nullptr;   // [dims product] dense cell -> occupied slot or -1
  int* occ_dense = nullptr;      // [ncells] occupied slot -> dense cell
  uint32_t* occ_bits = nullptr;  // [ceil(dims product / 32)] occupancy bit per dense cell
  gpf::TileInfo* tiles = nullptr;  // [ntiles]
  float4* tile_lo = nullptr;     // [ntiles] tight box of the tile's points
  float4* tile_hi = nullptr;
  int64_t ngroups = 0;
  gpf::GroupInfo* groups = nullptr;  // [ngroups]
  float4* group_lo = nullptr;        // [ngroups] box of the group's points
  float4* group_hi = nullptr;
  size_t bytes = 0;
  // allocated bytes of each array above, so that a rebin reuses them
  size_t xs_cap = 0, perm_cap = 0, occ_of_dense_cap = 0, occ_dense_cap = 0, occ_bits_cap = 0,
         tiles_cap = 0, tile_lo_cap = 0, tile_hi_cap = 0, groups_cap = 0, group_lo_cap = 0,
         group_hi_cap = 0;
  // binning scratch, kept between rebins (released after a one-off binning)
  uint64_t *keys = nullptr, *keys_s = nullptr;
  int *idx = nullptr, *flag = nullptr, *flag_s = nullptr, *cell_first = nullptr,
      *ntile = nullptr, *cell_first_g = nullptr;
  float* part = nullptr;
  void* tmp = nullptr;
  size_t keys_cap = 0, keys_s_cap = 0, idx_cap = 0, flag_cap = 0, flag_s_cap = 0,
         cell_first_cap = 0, ntile_cap = 0, cell_first_g_cap = 0, part_cap = 0, tmp_cap = 0;
};

struct gpf_grid {
  const gpf_queries* qs = nullptr;
  const float *mu = nullptr, *quat = nullptr, *log_scale = nullptr, *rgb = nullptr;
  int64_t n = 0;
  float cutoff = 3.f;
  gpf::PrimRec* rec = nullptr;  // [n]
  float4* ext = nullptr;        // [n] half-extents of the cutoff box; w = 1 if valid
  int64_t rec_cap = 0;
  int* prim_off = nullptr;      // per-(primitive, sub-thread) entry counts and their scan
  int64_t prim_off_len = 0;     // allocated entries of prim_off
  int* readback = nullptr;      // pinned host pair: entry total, degenerate primitives
  int* cell_start = nullptr;    // [ncells + 1]
  int64_t cell_start_cap = 0;   // allocated entries of cell_start
  uint64_t qs_gen = 0;          // query-set binning this grid was built on
  int* keys = nullptr;          // [cap] cell slot per entry (primitive-major)
  int* vals = nullptr;          // [cap] primitive per entry (primitive-major)
  int* keys_sorted = nullptr;   // [cap]
  int* cell_prims = nullptr;    // [cap] primitives of each cell, ascending
  gpf::PrimRec* cell_recs = nullptr;  // [cap] their records in the same order (truncated query)
  int64_t cell_recs_cap = 0;
  void* sort_tmp = nullptr;
  size_t sort_tmp_bytes = 0;
  int64_t cap = 0;
  int64_t entries = 0;
  float4* grad_rows = nullptr;  // [n][4] backward scratch: one 64-byte row per primitive
  int64_t grad_cap = 0;
  // Survivors of the forward's cull, per group (cell entry | tile mask << 30,
  // in cell-list order, at most kSurvPerGroup each) and their number, for the
  // backward of the same build; surv_ready is set by a forward and cleared by
  // a build.
  int* surv = nullptr;          // [surv_groups][kSurvPerGroup]
  int* surv_count = nullptr;    // [surv_groups]
  int64_t surv_groups = 0;
  bool surv_ready = false;
  // Hybrid query (ball > 0): ball radius r, nearest-centre top-up size, and a
  // uniform grid over the centres for the top-up search.
  float ball = 0.f;
  int k_min = 0;
  float cg_origin[3] = {0.f, 0.f, 0.f};
  float cg_h = 0.f;
  int cg_dims[3] = {0, 0, 0};
  int64_t cg_cells_cap = 0, cg_n_cap = 0;
  int* cg_start = nullptr;      // [cells + 1]
  unsigned* cg_key = nullptr;   // [n] cell of each centre, then [n] sorted
  int* cg_val = nullptr;        // [n] centre indices before the sort
  int* cg_sorted = nullptr;     // [n] centre indices by cell (index order within a cell)
  unsigned char* cg_near = nullptr;  // [cells] a centre lies within the top-up's rings
  float* cg_box = nullptr;      // [64 * 6] partial boxes
  void* cg_tmp = nullptr;
  size_t cg_tmp_bytes = 0;
  size_t cg_bytes = 0;
  size_t bytes = 0;
};

namespace gpf {

// Error plumbing (capi.cpp).
gpf_status set_error(gpf_status s, const std::string& msg);
gpf_status hip_fail(hipError_t e, const char* what);
#define GPF_HIP(call)                                         \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return ::gpf::hip_fail(e_, #call);  \
  } while (0)

// Device allocation under an optional byte budget (GPF_DEVICE_BYTES_LIMIT).
gpf_status dev_alloc(void** p, size_t bytes, const char* what);
void dev_free(void* p, size_t bytes);

// Launchers implemented in the .hip files.  They only enqueue work.
void release_bin_scratch(gpf_queries* qs);
void release_bin_outputs(gpf_queries* qs);
gpf_status launch_bin_queries(const float* x, int64_t q, float cell, bool keep_scratch, hipStream_t s,
                              gpf_queries* out);
gpf_status launch_build_grid(gpf_grid* g, hipStream_t s);
gpf_status launch_eval_fwd(const gpf_grid* g, float* L, hipStream_t s);
gpf_status launch_eval_bwd(const gpf_grid* g, const float* dL, gpf_field_grad* grad,
                           hipStream_t s);
// Primitives the allocation-free backward takes (its rows are a static
// device array of kNoAllocMaxPrims * 64 bytes).
constexpr int64_t kNoAllocMaxPrims = (int64_t)1 << 18;
gpf_status launch_eval_bwd_noalloc(const gpf_grid* g, const float* dL, gpf_field_grad* grad,
                                   hipStream_t s);
gpf_status launch_fit_pass(const gpf_grid* g, const float* T, float* L, double* loss,
                           gpf_field_grad* grad, hipStream_t s);
gpf_status launch_count_pairs(const gpf_grid* g, unsigned long long* d_count, hipStream_t s);
gpf_status ensure_grad_rows(gpf_grid* g, hipStream_t s);
void ensure_survivor_lists(gpf_grid* g);
gpf_status launch_grad_finalize(gpf_grid* g, float4* rows, gpf_field_grad* grad, hipStream_t s);
gpf_status build_centre_grid(gpf_grid* g, hipStream_t s);
void free_centre_grid(gpf_grid* g);
gpf_status launch_hybrid_fwd(const gpf_grid* g, float eps, float* L, float* Z, int* count,
                             hipStream_t s);
gpf_status launch_hybrid_bwd(const gpf_grid* g, float eps, const float* L, const float* Z,
                             const int* count, const float* dL, gpf_field_grad* grad,
                             hipStream_t s);
gpf_status launch_trace_photons(int64_t n, uint64_t seed, int E, float lo, float hi, int sphere,
                                float* pos, float* pw, int* surf, hipStream_t s);
gpf_status compact_photons(const float* pos, const float* pw, const int* surf, int64_t m,
                           float* opos, float* opw, int* osurf, int64_t* oslot, int64_t cap,
                           int64_t* count, hipStream_t s);
gpf_status photon_map_build(const float* ppos, const float* ppw, const int* psurf, int64_t np,
                            float r, gpf_photon_map** out, hipStream_t s);
gpf_status photon_map_fill(gpf_photon_map* m, const float* ppos, const float* ppw,
                           const int* psurf, int64_t np, float r, hipStream_t s);
gpf_status photon_map_gather(const gpf_photon_map* m, const float* x, const int* xs, int64_t q,
                             float weight, bool accumulate, float* L, int* count, hipStream_t s);
void photon_map_free(gpf_photon_map* m);
gpf_status photon_map_gather_binned(const gpf_photon_map* m, const gpf_queries* qs,
                                    const int* xs, float weight, bool accumulate, float* L,
                                    int* count, hipStream_t s);
gpf_status launch_camera_trace(const gpf_camera* cam, int samples, uint64_t seed, int max_depth,
                               float lo, float hi, int sphere, float* x, float* beta, int* face,
                               float* Le, hipStream_t s);
gpf_status launch_camera_compose(const float* Le, int64_t n_pix, int S, const int64_t* slot,
                                 const float* beta_c, const float* Lq, int64_t m, float* L,
                                 hipStream_t s);
gpf_status launch_camera_compose_backward(const float* dL, int64_t n_pix, int S,
                                          const int64_t* slot, const float* beta_c, int64_t m,
                                          float* dLq, hipStream_t s);
gpf_status launch_mse(const float* L, const float* T, int64_t q, double* loss, float* dL,
                      hipStream_t s);
gpf_status launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                       float b1, float b2, float eps, int64_t step, const double* guard,
                       hipStream_t s);

// Workgroup -> work-item remap.  Workgroups are dealt round-robin over the 8
// XCDs; this mapping hands each XCD whole chunks of kXcdChunk consecutive
// (spatially sorted) work items, so that the primitives a chunk touches stay
// hot in that XCD's L2, while consecutive chunks go to different XCDs so that
// dense regions of the scene are spread over the whole chip.  Launch
// xcd_grid(n) workgroups; work items >= n must return.
#ifndef GPF_XCD_CHUNK
#define GPF_XCD_CHUNK 16
#endif
constexpr int kXcd = 8;
// Survivors per group kept from the forward for the backward; a group with
// more culls again in the backward.
#ifndef GPF_SURV_PER_GROUP
#define GPF_SURV_PER_GROUP 2048
#endif
constexpr int kSurvPerGroup = GPF_SURV_PER_GROUP;
constexpr int kXcdChunk = GPF_XCD_CHUNK;

inline unsigned xcd_grid(int64_t n) {
  const int64_t per = (int64_t)kXcd * kXcdChunk;
  return (unsigned)(((n + per - 1) / per) * per);
}

__device__ __forceinline__ int xcd_remap(int bid) {
  const int xcd = bid % kXcd;
  const int idx = bid / kXcd;
  const int chunk = idx / kXcdChunk, within = idx % kXcdChunk;
  return (chunk * kXcd + xcd) * kXcdChunk + within;
}

}  // namespace gpf
