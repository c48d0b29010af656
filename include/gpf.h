/*
 * gpf.h -- C ABI of the Gaussian Photon Field radiance library (libgpf.so).
 *
 * The field (Sec. 4.1, Eq. gaussian_contribution) is a set of N anisotropic
 * 3-D Gaussians with centre mu, rotation quaternion q = (w,x,y,z) (Hamilton,
 * scalar first), per-axis scale s = exp(log_scale) and RGB flux Phi.  A query
 * at a surface point x (the first diffuse hit of a camera ray, Sec. 4.2) sums
 * the flux of every primitive within Mahalanobis distance `cutoff` (3 sigma),
 * each weighted by exp(-m^2/2), m^2 = |diag(1/s) R^T (x - mu)|^2 (the
 * aggregation equation of Sec. 4.2 with the local-frame evaluation of the
 * supplementary hybrid query, Alg. S3; un-normalised, no distance falloff,
 * no BSDF factor).
 *
 * Conventions for every call:
 *  - Array pointers are DEVICE pointers (hipMalloc'd or torch CUDA tensors),
 *    FP32, row-major, contiguous, unless a comment says "host".
 *  - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *    Calls enqueue work on it and return without synchronising, except where a
 *    comment says the call synchronises.
 *  - The caller owns every input, output and gradient buffer.  The library
 *    owns the opaque handles (query sets, grids, MLPs) and the device memory
 *    inside them; destroy them with the matching *_destroy call.
 *  - No call aborts or throws.  Arguments are validated on the host before any
 *    launch; failures return a non-zero gpf_status and leave a message for
 *    gpf_last_error() (thread-local).  Outputs are untouched on failure.
 */
#ifndef GPF_H
#define GPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GPF_OK = 0,
  GPF_ERR_INVALID_ARGUMENT = 1, /* null pointer, bad size, bad option        */
  GPF_ERR_OUT_OF_MEMORY = 2,    /* device allocation failed or over budget   */
  GPF_ERR_CAPACITY = 3,         /* a size exceeds a documented maximum       */
  GPF_ERR_HIP = 4,              /* a HIP runtime call failed                 */
  GPF_ERR_STALE = 5             /* handle built for a different field/query  */
} gpf_status;

typedef struct gpf_queries gpf_queries; /* binned query points (opaque)       */
typedef struct gpf_grid gpf_grid;       /* per-field cull structure (opaque)  */
typedef struct gpf_mlp gpf_mlp;         /* learned initialiser (opaque)       */
typedef struct gpf_photon_map gpf_photon_map; /* gridded photon map (opaque) */

/* A field of n primitives (1 <= n <= 2^30 - 1): mu[n][3], quat[n][4]
   (w,x,y,z; any non-zero norm, normalised inside), log_scale[n][3] (natural
   log of the per-axis standard deviation), rgb[n][3] (flux Phi). */
typedef struct {
  const float *mu, *quat, *log_scale, *rgb;
  int64_t n;
} gpf_field;

/* Gradient buffers with the shapes of gpf_field; calls ADD into them. */
typedef struct {
  float *mu, *quat, *log_scale, *rgb;
} gpf_field_grad;

/* Output field buffers with the shapes of gpf_field; calls OVERWRITE them. */
typedef struct {
  float *mu, *quat, *log_scale, *rgb;
} gpf_field_out;

/* ---- status ------------------------------------------------------------ */
const char *gpf_last_error(void);       /* message of the last failure (host) */
const char *gpf_version(void);

/* ---- query binning (supports the visible-point set of Sec. 4.3, which is
 * fixed during training, so it is binned once) ---------------------------
 * Bins q query points x[q][3] into a uniform grid of cubic cells of edge
 * `cell_size` (> 0) spanning their bounding box, sorts them by cell and by a
 * Morton code inside the cell, and cuts each cell's run into tiles of at most
 * 64 points.  The grid geometry of every later gpf_build_grid comes from this
 * set.  1 <= q <= 2^31 - 1.  Synchronises `stream` (reads back the bounding
 * box and the tile count).  *out receives a new handle. */
gpf_status gpf_bin_queries(const float *x, int64_t q, float cell_size, void *stream,
                           gpf_queries **out);
/* Re-bins new points x[q][3] into an existing handle, as gpf_bin_queries
 * would, reusing its device buffers (and its binning scratch, which a rebin
 * keeps): it allocates only when the new points need more room than any
 * earlier binning of the handle, so a loop over views or frames stops
 * allocating once the largest has been seen.  Every grid built on `qs`
 * before the call is stale afterwards (its queries return GPF_ERR_STALE)
 * until it is rebuilt with gpf_build_grid / gpf_build_grid_hybrid on the same
 * handle.  On failure the handle holds no binning (q = 0) until the next
 * successful rebin; it must still be destroyed.  Same limits on q and
 * cell_size as gpf_bin_queries; the current device must be the one `qs` was
 * created on.  Synchronises `stream`; work queued on other streams that reads
 * `qs` or a grid built on it must have finished before the call. */
gpf_status gpf_rebin_queries(gpf_queries *qs, const float *x, int64_t q, float cell_size,
                             void *stream);
/* Releases the query set.  Grids built on it keep a pointer to it: destroy
 * them first (or at least never use them afterwards). */
void gpf_queries_destroy(gpf_queries *qs);
/* Host-side facts about a query set: number of points, of occupied cells and
 * of tiles, and the device bytes the handle holds. */
gpf_status gpf_queries_info(const gpf_queries *qs, int64_t *q, int64_t *cells, int64_t *tiles,
                            size_t *device_bytes);

/* ---- grid build (replaces the KD-tree over Gaussian centres of the paper's
 * implementation, supplementary Sec. A.2) -----------------------------------
 * For every primitive: normalise q, build R(q), s = exp(log_scale) and the
 * whitening W = diag(1/s) R^T in FP64, rounded once to FP32; then register the
 * primitive in every occupied cell of `qs` whose box its `cutoff`-sigma
 * ellipsoid may touch (a conservative separating-axis test in the whitened
 * frame).  The grid keeps FP32 records {mu, W, Phi} of the field as it is now:
 * rebuild after any parameter change.  `cutoff` in (0, 16]; a zero-norm
 * quaternion or a non-finite position, quaternion, log-scale or flux is
 * GPF_ERR_INVALID_ARGUMENT (found on the device, reported after the one
 * synchronisation).  If *grid is
 * non-NULL it must come from an earlier call with the same `qs` and is
 * rebuilt in place (its buffers grow as needed); otherwise a new handle is
 * returned.  Synchronises `stream` once (reads back the number of
 * cell-primitive entries). */
gpf_status gpf_build_grid(const gpf_field *f, float cutoff, const gpf_queries *qs,
                          void *stream, gpf_grid **grid);
void gpf_grid_destroy(gpf_grid *grid);
/* Host-side facts about a built grid: cell-primitive entries, device bytes. */
gpf_status gpf_grid_info(const gpf_grid *grid, int64_t *entries, size_t *device_bytes);

/* ---- forward radiance query (Sec. 4.2 aggregation; Alg. S3 local frame) ---
 * L[i][c] = sum over primitives with m^2 <= cutoff^2 of exp(-m^2/2) rgb[c],
 * for the q points x[q][3] that were binned into the grid's query set (same
 * buffer, same contents).  L[q][3] is overwritten; a point with no
 * contributing primitive gets exactly 0.  `f` must be the field the grid was
 * built from (same pointers and n), else GPF_ERR_STALE.  The grid keeps the
 * primitives that survive the cull of each group of query points (up to 2048
 * per group, 4 bytes each; allocated on the first call and kept, not
 * allocated at all if the device byte budget refuses), which a backward on
 * the same build then reuses instead of culling again. */
gpf_status gpf_eval_radiance(const gpf_grid *grid, const gpf_field *f, const float *x, int64_t q,
                             float *L, void *stream);

/* ---- backward (Sec. 4.2 "Differentiable Accumulation") --------------------
 * Given dL[q][3] = d(loss)/dL, ADDS d(loss)/d(param) into grad for every
 * primitive parameter: mu, quat (through its normalisation), log_scale and
 * rgb.  Kernel weights are recomputed per pair, nothing per pair is stored.
 * The derivative of the cutoff indicator is taken as zero.  Gradient buffers
 * must not alias the field.  Accumulation order is not deterministic
 * (floating-point atomics).  After a gpf_eval_radiance on the same build the
 * backward reads that call's survivor lists rather than culling (same pairs);
 * on a stream other than the forward's the caller orders the two calls. */
gpf_status gpf_eval_radiance_backward(const gpf_grid *grid, const gpf_field *f, const float *x,
                                      int64_t q, const float *dL, gpf_field_grad *grad,
                                      void *stream);

/* ---- one fitting pass (Sec. 4.3 MSE loss; Sec. 4.2 forward and backward) -
 * The forward, the loss and the backward of one optimisation step in one
 * call, for the truncated query: L[q][3] as gpf_eval_radiance writes it,
 * loss_sum[0] (device, FP64) += sum_i sum_c (L - T)^2 over the q points
 * against the targets T[q][3] (device, same order as x), and d(loss)/d(param)
 * ADDED into grad as gpf_eval_radiance_backward would with
 * dL = 2 (L - T) / q, each dL value rounded to FP32 as gpf_mse_loss rounds it.
 * dL itself is never written to memory.  The caller zeroes loss_sum and grad.
 * The survivor lists are kept as by gpf_eval_radiance, so a later backward on
 * the same build reuses them.  Errors as for those two calls; L must not
 * alias T.  Loss and gradient accumulation order is not deterministic
 * (floating-point atomics). */
gpf_status gpf_fit_pass(const gpf_grid *grid, const gpf_field *f, const float *x, int64_t q,
                        const float *T, float *L, double *loss_sum, gpf_field_grad *grad,
                        void *stream);

/* ---- backward without device allocation ---------------------------------
 * For callers that cannot allocate device memory during the call: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, result and errors as gpf_eval_radiance_backward, but the
 * per-primitive gradient rows the backward gathers into are a static device
 * array of the library (16 MiB on every device it runs on, held until the
 * process ends) rather than memory of the grid handle, and the call never
 * allocates.  At most 262,144 primitives (f->n), else GPF_ERR_CAPACITY
 * before any launch.  The call clears the rows it uses with a fill kernel, so
 * nothing carries over from an earlier call; calls that overlap on one
 * device (other streams or threads) share the array and race, so the caller
 * orders them.  The first call on a device looks up the array's address. */
gpf_status gpf_eval_radiance_backward_noalloc(const gpf_grid *grid, const gpf_field *f,
                                              const float *x, int64_t q, const float *dL,
                                              gpf_field_grad *grad, void *stream);

/* ---- hybrid query: the paper's own neighbourhood (supplementary Alg. S3;
 * Sec. 4.2 neighbourhood search and aggregation) ----------------------------
 * Neighbourhood N(x) of a query point: the Gaussians whose centre lies within
 * Euclidean distance r of x (ball query); when the ball holds fewer than
 * k_min centres, the k_min centres nearest to x (which contain the ball).
 * Membership and nearest order are decided on single-precision squared
 * distances (dx*dx + dy*dy) + dz*dz, dx = x - mu, without fused multiply-add,
 * against r*r rounded to FP32; ties go to the lower index.  Weight
 * w = exp(-m^2/2) psi(|x - mu|) with no 3-sigma cut, psi = 1 within r and
 * exp(-3 t^2), t = (|x - mu| - r) / max(r, 1e-6), beyond.
 * L(x) = sum_N w Phi / max(sum_N w, eps).
 *
 * gpf_build_grid_hybrid: as gpf_build_grid, but every Gaussian is listed in
 * each occupied query cell its ball of radius r may reach, and a uniform grid
 * over the centres is built for the nearest-centre top-up.  r > 0 (finite),
 * 1 <= k_min <= 8.  Synchronises `stream` (two small readbacks).  A handle
 * keeps its query mode: rebuilding a truncated handle as hybrid (or the
 * reverse) is GPF_ERR_INVALID_ARGUMENT. */
gpf_status gpf_build_grid_hybrid(const gpf_field *f, float r, int k_min, const gpf_queries *qs,
                                 void *stream, gpf_grid **grid);

/* Forward: L[q][3] (overwritten, normalised), Z[q] = sum of the weights
 * before clamping, count[q] = number of centres in the ball of each point
 * (the top-up applies where count < k_min).  eps > 0.  Device pointers. */
gpf_status gpf_eval_hybrid(const gpf_grid *grid, const gpf_field *f, const float *x, int64_t q,
                           float eps, float *L, float *Z, int *count, void *stream);

/* Backward: adds to `grad` the gradient of sum_x dL(x) . L(x) with respect to
 * every Gaussian parameter, given this forward's L, Z and count for the same
 * grid, field and eps (per-point values, not per pair; weights are
 * recomputed).  With Zc = max(Z, eps): dPhi += w dL / Zc and, through w,
 * a = (dL . Phi - [Z >= eps] dL . L) / Zc per pair; changes of the
 * neighbourhoods contribute nothing.  Accumulation order is not
 * deterministic (floating-point atomics). */
gpf_status gpf_eval_hybrid_backward(const gpf_grid *grid, const gpf_field *f, const float *x,
                                    int64_t q, float eps, const float *L, const float *Z,
                                    const int *count, const float *dL, gpf_field_grad *grad,
                                    void *stream);

/* ---- photon tracing (Sec. 3.2 photon pass) and density estimate (Sec. 3
 * radiance estimation, Sec. 4.3 reference equation) ----------------------
 * Scene: the box [0,1]^3 with diffuse faces floor y=0 (0), ceiling y=1 (1),
 * x=0 (2), x=1 (3), back z=0 (4), open at z=1; a sphere of radius 0.2 at
 * (0.5,0.5,0.5) chosen by `sphere`: 0 none, 1 glass of index 1.5, 2 a mirror
 * of reflectance (0.95, 0.64, 0.54).  Albedos: white 0.73 for
 * 0, 1, 4; red (0.63, 0.06, 0.05) for 2; green (0.14, 0.45, 0.09) for 3.
 * Light: the ceiling square [light_lo, light_hi]^2 in x and z (a point when
 * equal), cosine distribution downwards, total power (12, 10, 8).
 *
 * gpf_trace_photons: n_paths photon paths, each with power (12,10,8)/n_paths
 * and uniforms from Philox4x64-10 (key (seed, 0), counter (path, event, 0,
 * 0), word -> (w >> 40) * 2^-24).  Event 0 emits; events 1..max_events
 * intersect sphere and box: the glass sphere reflects when u0 < F (exact
 * Fresnel) and refracts otherwise, the mirror reflects and scales the power
 * by its reflectance; a diffuse face stores a photon in slot
 * [path][event - 1] and continues when u0 < q = max(albedo) with power
 * * albedo / q in a cosine direction.  Outputs (device, caller-owned, written
 * whole): pos[n_paths][max_events][3], power[..][3], surface[..] (-1, with
 * zero position and power, where nothing was stored).  1 <= n_paths < 2^31, 1 <= max_events <= 16,
 * 0 <= light_lo <= light_hi <= 1, sphere in {0, 1, 2}. */
gpf_status gpf_trace_photons(int64_t n_paths, uint64_t seed, int max_events, float light_lo,
                             float light_hi, int sphere, float *pos, float *power, int *surface,
                             void *stream);

/* Order-preserving compaction of m photon records (surface >= 0 kept):
 * out_pos[count][3], out_power[count][3], out_surface[count], out_slot[count]
 * (record index; may be NULL).  *count (host) receives the number kept;
 * GPF_ERR_CAPACITY when it exceeds `capacity`.  m < 2^31.  Synchronises. */
gpf_status gpf_compact_photons(const float *pos, const float *power, const int *surface, int64_t m,
                               float *out_pos, float *out_power, int *out_surface, int64_t *out_slot,
                               int64_t capacity, int64_t *count, void *stream);

/* Photon map for the density estimate: the photons ppos[np][3],
 * ppower[np][3], psurface[np] (device; copied, so the caller may free them
 * afterwards) binned into a uniform grid of cells of edge >= r/2 in cell order.
 * 1 <= np < 2^31; r > 0 finite; non-finite positions are
 * GPF_ERR_INVALID_ARGUMENT.  Synchronises.  Release with
 * gpf_photon_map_destroy. */
gpf_status gpf_photon_map_build(const float *ppos, const float *ppower, const int *psurface,
                                int64_t np, float r, void *stream, gpf_photon_map **map);

/* Rebinds an existing map to new photons and radius (same arguments and
 * limits as gpf_photon_map_build), reusing its device buffers when they are
 * large enough: the progressive reference rebuilds one map per iteration.  On
 * failure the map holds no photons (gathers fail) until a rebuild succeeds.
 * Synchronises. */
gpf_status gpf_photon_map_rebuild(gpf_photon_map *map, const float *ppos, const float *ppower,
                                  const int *psurface, int64_t np, float r, void *stream);
void gpf_photon_map_destroy(gpf_photon_map *map);

/* Density estimate (Sec. 3.2 radiance estimation; the inner sum of the Sec. 4.3
 * reference equation with a Lambertian BSDF) at q points x[q][3] lying on
 * faces x_surface[q] (a point on the sphere, or any value outside 0..4, gets
 * 0): E = albedo / pi / (pi r^2) * sum of the powers of the photons of the
 * same face within the map's r, membership decided on FP32 squared distances
 * (dx*dx + dy*dy) + dz*dz without fused multiply-add.  L[q][3] = weight * E,
 * or L + weight * E when `accumulate` is non-zero (the progressive average of
 * the reference equation is a sum of such calls with weight 1/N_iter).  When
 * `count` is not NULL, count[q] (int32) receives the number of photons
 * gathered at each point.  All arrays are device memory; 1 <= q < 2^31.  One
 * kernel launch on `stream`; does not synchronise. */
gpf_status gpf_photon_map_gather(const gpf_photon_map *map, const float *x, const int *x_surface,
                                 int64_t q, float weight, int accumulate, float *L, int *count,
                                 void *stream);

/* The same estimate at the points of a binned query set (gpf_bin_queries),
 * x_surface[q] in the caller's order of those points, L[q][3] and count[q]
 * likewise: one wave per tile of points visits each photon of the cells near
 * the tile once, so the results are bit-identical to gpf_photon_map_gather's
 * at the same points.  Does not synchronise. */
gpf_status gpf_photon_map_gather_binned(const gpf_photon_map *map, const gpf_queries *queries,
                                        const int *x_surface, float weight, int accumulate,
                                        float *L, int *count, void *stream);

/* gpf_photon_map_build + gpf_photon_map_gather + destroy in one call.
 * Synchronises. */
gpf_status gpf_photon_density(const float *x, const int *x_surface, int64_t q, const float *ppos,
                              const float *ppower, const int *psurface, int64_t np, float r,
                              float weight, int accumulate, float *L, int *count, void *stream);

/* ---- hybrid camera integrator (Sec. 4.2 rendering with the field;
 * supplementary Alg. S2) ----------------------------------------------------
 * Pinhole camera: rays from `eye` through the pixel centres of a width x
 * height image (row 0 at the top) spanning vertical field of view vfov_deg
 * about the direction to `target`, `up` fixing the roll. */
typedef struct {
  float eye[3], target[3], up[3];
  float vfov_deg;
  int width, height;
} gpf_camera;

/* Camera paths in the scene of gpf_trace_photons, `samples` per pixel, path
 * k = pixel * samples + s.  Each follows the sphere's specular interactions
 * (glass: reflect when u0 < F, u0 from Philox counter (k, depth, 1, 0) with
 * key (seed, 0), throughput unchanged; refract otherwise with throughput *=
 * (eta_i / eta_t)^2; mirror: throughput *= reflectance) for at most
 * max_depth intersections and ends
 *  - on a diffuse face: x[k][3] = hit, face[k] = 0..4, beta[k][3] = throughput;
 *  - on the ceiling inside the light square: Le[k][3] = throughput * the
 *    light's radiance (12, 10, 8) / (pi * area), face[k] = -1;
 *  - through the open side or at max_depth: face[k] = -1.
 * Unused outputs are 0.  Outputs are device arrays of width*height*samples
 * rows, which must stay below 2^31; 1 <= samples <= 1024, 1 <= max_depth
 * <= 64, sphere in {0, 1, 2}; 0 <= light_lo <= light_hi <= 1; 0 < vfov_deg <
 * 180; eye != target and up not parallel to the view direction. */
gpf_status gpf_camera_trace(const gpf_camera *cam, int samples, uint64_t seed, int max_depth,
                            float light_lo, float light_hi, int sphere, float *x, float *beta,
                            int *face, float *Le, void *stream);

/* Pixel radiance L_pix[n_pix][3] = (1/samples) * sum over the pixel's paths
 * of Le + beta * L(x), from the diffuse hits compacted in path order
 * (gpf_compact_photons on (x, beta, face) gives them with slot = path index):
 * slot[m] ascending path indices, beta_c[m][3], and the field's radiance
 * Lq[m][3] at those hits.  Le[n_pix * samples][3].  Device arrays; m may be
 * 0.  Does not synchronise. */
gpf_status gpf_camera_compose(const float *Le, int64_t n_pix, int samples, const int64_t *slot,
                              const float *beta_c, const float *Lq, int64_t m, float *L_pix,
                              void *stream);

/* Gradient of a loss with respect to Lq from its gradient dL_pix[n_pix][3]
 * with respect to the pixels: dLq[k] = beta_c[k] * dL_pix[slot[k] / samples]
 * / samples (0 for a slot outside the image).  Does not synchronise. */
gpf_status gpf_camera_compose_backward(const float *dL_pix, int64_t n_pix, int samples,
                                       const int64_t *slot, const float *beta_c, int64_t m,
                                       float *dLq, void *stream);

/* ---- exact pair count (roofline numerator) --------------------------------
 * Writes to *pairs (host) the number of (query, primitive) pairs with
 * m^2 <= cutoff^2.  Synchronises `stream`. */
gpf_status gpf_count_pairs(const gpf_grid *grid, const gpf_field *f, int64_t *pairs, void *stream);

/* ---- loss (Sec. 4.3 MSE over visible points) ------------------------------
 * loss_sum[0] (device, FP64) += sum_i sum_c (L - T)^2 over the q points and
 * dL[q][3] = 2 (L - T) / q.  The caller zeroes loss_sum; MSE = loss_sum / q. */
gpf_status gpf_mse_loss(const float *L, const float *T, int64_t q, double *loss_sum, float *dL,
                        void *stream);

/* ---- optimiser (Adam, Kingma & Ba 2015; the paper trains with Adam) ------
 * One fused Adam update of n FP32 values: m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
 * `step` is the 1-based step count t.  p, g, m, v are distinct buffers of n.
 * `guard` (device, FP64, may be NULL), e.g. the loss sum of gpf_mse_loss:
 * when it is not finite the update is skipped on the device and p, m, v keep
 * their values, so a non-finite loss never reaches the parameters. */
gpf_status gpf_adam_step(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                         float beta1, float beta2, float eps, int64_t step, const double *guard,
                         void *stream);

/* ---- photon-to-Gaussian initialisation (Sec. 4.1 physically-inspired
 * initialisation: one Gaussian per photon, centre = photon position, flux =
 * photon flux; supplementary Sec. A.2 gives the paper's defaults) ---------- */

/* k nearest other photons of every photon: idx[p][k] (int32, device) and
 * FP32 squared distances d2[p][k], ordered by (distance, index); distances are
 * ((dx*dx + dy*dy) + dz*dz) with each operation rounded to FP32 (no fused
 * multiply-add).  pos[p][3].  3 <= k <= 32, p >= k + 1, p <= 2^28.
 * Synchronises `stream`. */
gpf_status gpf_photon_knn(const float *pos, int64_t p, int k, int32_t *idx, float *d2,
                          void *stream);

/* Network inputs X[p][96] (bfloat16 bits, device) from 16 neighbours (idx, d2
 * from gpf_photon_knn with k = 16): for each neighbour j in order,
 * (pos_j - pos_i) / r16 (3 values) then log(power_j / power_i) per channel. */
gpf_status gpf_photon_features(const float *pos, const float *power, int64_t p,
                               const int32_t *idx, const float *d2, uint16_t *X, void *stream);

/* Gaussians from photons, written to out (overwritten, p primitives):
 * mu = pos, rgb = power, and
 *  - mlp == NULL (plain initialisation): q = (1,0,0,0), isotropic
 *    log_scale = log(clamp(r3, 1e-4, 0.1)) with r3 the distance to the
 *    third-nearest photon (k >= 3);
 *  - mlp != NULL (learned initialisation, k must be 16): the network maps each
 *    photon's features to o[10]; q = normalise((1,0,0,0) + o[0:4]),
 *    log_scale = plain + o[4:7], rgb = power * exp(o[7:10]).
 * pos, power: [p][3] device.  Synchronises `stream`. */
gpf_status gpf_init_from_photons(const float *pos, const float *power, int64_t p, int k,
                                 const gpf_mlp *mlp, gpf_field_out *out, void *stream);

/* ---- learned initialiser network (not in the paper): 96 -> 128 -> 128 -> 10
 * with exact-erf GELU after both hidden layers, bfloat16 operands on MFMA with
 * FP32 accumulation, FP32 master parameters trained by Adam. --------------
 * Parameter vector (FP32, gpf_mlp_num_params() = 30218 values), matrices
 * W[in][out] row-major: W1[96][128] b1[128] W2[128][128] b2[128] W3[128][10]
 * b3[10]; a layer computes y = x W + b. */
int64_t gpf_mlp_num_params(void);
/* New network with all parameters zero (its outputs are zero: plain
 * initialisation).  Synchronises the device. */
gpf_status gpf_mlp_create(gpf_mlp **out);
void gpf_mlp_destroy(gpf_mlp *mlp);
/* Copies params (HOST, gpf_mlp_num_params() floats) into the network and
 * resets the optimiser state.  Synchronises the device. */
gpf_status gpf_mlp_set_params(gpf_mlp *mlp, const float *params);
/* Copies the FP32 parameters to params (HOST).  Synchronises the device. */
gpf_status gpf_mlp_get_params(const gpf_mlp *mlp, float *params);
/* Y[b][10] (FP32) = network(X[b][96] bfloat16 bits). */
gpf_status gpf_mlp_forward(const gpf_mlp *mlp, const uint16_t *X, int64_t b, float *Y,
                           void *stream);
/* Gradient of the mean squared error mean((Y - T)^2) over the b x 10 outputs:
 * grad[gpf_mlp_num_params()] (device) is overwritten; loss_sum (device FP64,
 * may be NULL) += sum of squared errors.  T[b][10] FP32. */
gpf_status gpf_mlp_gradient(gpf_mlp *mlp, const uint16_t *X, const float *T, int64_t b,
                            float *grad, double *loss_sum, void *stream);
/* One training step: the gradient above, then Adam (beta 0.9/0.999, eps 1e-8,
 * learning rate lr) on the FP32 parameters. */
gpf_status gpf_mlp_train_step(gpf_mlp *mlp, const uint16_t *X, const float *T, int64_t b, float lr,
                              double *loss_sum, void *stream);
/* Training targets T[p][10] that would map photon i onto Gaussian i of a
 * fitted field: o[0:4] = qhat - (1,0,0,0) (sign chosen so qhat_w >= 0),
 * o[4:7] = log_scale - log(clamp(r3)), o[7:10] = log(max(rgb, 1e-6 power) / power).
 * d2 from gpf_photon_knn (k columns). */
gpf_status gpf_mlp_targets(const float *power, int64_t p, const float *d2, int k,
                           const gpf_field *fitted, float *T, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GPF_H */
