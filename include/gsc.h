/* gsc.h -- C ABI of the GSCache hot path on MI355X (gfx950).
 *
 * GSCache (arXiv 2507.19718) caches path-space radiance of a volume path tracer in K levels of
 * 3D Gaussians, one level per path length (Method: "A Path Space Radiance Cache").  Each frame
 * the levels are splatted into cache images, the tracer runs with the early-termination
 * heuristic (Algorithm 1) and writes every terminated path's attenuated radiance into the
 * target buffer of its length (Method: "Cache Training"), and each level takes one AdamW step
 * against those noisy targets under the HDR loss (Eq. 4) with the viewport learning-rate
 * schedule (Eq. 5).  All the renderer gives the cache per path is the radiance it carried,
 * already attenuated, and the number of interactions of that path (Introduction); the library
 * is exposed through a C-style API (Method: "Implementation").
 *
 * Conventions
 *   - Pointers are DEVICE pointers unless marked HOST.  The caller owns every buffer it
 *     passes.  Opaque objects (gsc_ctx, gsc_binning, gsc_scene) are owned by the library,
 *     draw device memory through the context's allocator, and are released by the matching
 *     *_release / *_destroy call.
 *   - Every call returns a gsc_status; no C++ exception crosses the ABI.  On a non-OK status
 *     no output is valid.  Arguments are validated before anything is enqueued, so
 *     GSC_E_INVALID_ARG leaves the device untouched.  gsc_ctx_last_error() describes the last
 *     failure on a context.
 *   - Device work is enqueued on the context's HIP stream (on ROCm PyTorch: the caller's
 *     current stream).  A call synchronises only where stated.
 *   - Layouts: a level's Gaussians are SoA, pos [n][3], rot [n][4] (w, x, y, z; need not be
 *     normalised), log_scale [n][3], rgb [n][3], opacity_logit [n]: 14 fp32 per Gaussian
 *     (Appendix "Memory Footprint").  Images are [K][h][w][3] fp32, row-major, level-major.
 *   - Frames: the volume occupies the unit cube [0,1]^3.  Cameras map world to camera by
 *     x_c = R x_w + t with camera axes x right, y down, z forward; intrinsics are in full-frame
 *     pixels where pixel i spans [i, i+1).  (x0, y0, w, h) is the rendered window; every
 *     per-pixel quantity is computed in full-frame coordinates, so a crop reproduces the full
 *     frame's pixels exactly.  Tiles are 16x16 pixels laid out from (x0, y0).
 *   - Limits: 1 <= w, h <= 16384; 1 <= K <= 8 levels per request; 0 <= n < 2^31 Gaussians per
 *     level; 2 <= tf_points <= 64; 0 <= n_lights, n_spheres <= 8 with at least one light;
 *     instance counts are 64-bit.
 *   - Threading: a context is used by one host thread at a time; several contexts may share a
 *     device (one per concurrently running stream).
 *   - Determinism: every output is deterministic except, by default, the float-atomic sums of
 *     the splat adjoint (gsc_splat_backward and the training step of the frame calls), whose
 *     order of accumulation across tiles varies from run to run.  gsc_ctx_set_deterministic
 *     makes them reproducible bit for bit.
 */
#ifndef GSC_H_
#define GSC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GSC_OK = 0,
  GSC_E_INVALID_ARG = 1,   /* bad pointer, size or limit; nothing was enqueued            */
  GSC_E_CAPACITY = 2,      /* instance capacity exceeded; gsc_ctx_required_capacity() says  *
                            * how many were needed; retry with a larger hint                */
  GSC_E_OUT_OF_MEMORY = 3, /* the allocator returned NULL                                   */
  GSC_E_DEVICE = 4,        /* a HIP runtime error; sticky for the context                   */
  GSC_E_UNSUPPORTED = 5     /* the call needs a debug build (gsc_debug_selftest)            */
} gsc_status;

typedef struct gsc_ctx gsc_ctx;
typedef struct gsc_binning gsc_binning;
typedef struct gsc_scene gsc_scene;

/* Device-memory hooks.  alloc(bytes, user) returns device memory usable on the context's
 * stream or NULL; release(ptr, user) returns it.  With no allocator the library uses
 * hipMalloc / hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*release)(void* ptr, void* user);
  void* user;
} gsc_allocator;

/* HOST.  Pinhole camera, see the conventions above. */
typedef struct {
  float R[9];              /* world -> camera rotation, row-major                          */
  float t[3];
  float fx, fy, cx, cy;    /* full-frame pixels                                            */
  int32_t full_w, full_h;  /* full frame (the 1.3x frustum clamp of the EWA Jacobian)      */
  int32_t x0, y0, w, h;    /* rendered window                                              */
  float znear;             /* Gaussians at z <= znear are culled (0.2)                     */
} gsc_camera;

/* One cache level.  DEVICE arrays, layouts as in the conventions. */
typedef struct {
  const float* pos;
  const float* rot;
  const float* log_scale;
  const float* rgb;
  const float* opacity_logit;
  int64_t n;
} gsc_gaussians;

/* Writable parameter arrays of one level (cache initialisation output).  DEVICE, overwritten. */
typedef struct {
  float* pos;
  float* rot;
  float* log_scale;
  float* rgb;
  float* opacity_logit;
  int64_t n;
} gsc_level_buffers;

/* Parameter gradients of one level, same shapes as gsc_gaussians.  DEVICE, overwritten. */
typedef struct {
  float* pos;
  float* rot;
  float* log_scale;
  float* rgb;
  float* opacity_logit;
} gsc_grads;

/* A scalar volume and its optics.  density: DEVICE [nz][ny][nx] fp32 over [0,1]^3 (trilinear,
 * cell-centred, clamp-to-edge).  tf_rgba: HOST [tf_points][4], control point i at density
 * i/(tf_points-1) * density_max; sigma_t = d * A(d), albedo = RGB(d); the delta-tracking
 * majorant is density_max * max_i A_i (Evaluation: a predefined 1D transfer function per
 * dataset).  lights: HOST [n_lights][6] point lights (position xyz, radiant intensity rgb),
 * NULL when n_lights is 0.  spheres: HOST [n_spheres][7] spherical area lights (centre xyz,
 * radius > 0, emitted radiance rgb, uniform over the surface and outgoing directions), NULL
 * when n_spheres is 0; each must lie entirely outside the unit cube (the paper lights its
 * scenes with two small spherical lights placed outside the volume, Evaluation), otherwise
 * GSC_E_INVALID_ARG.  Lights are not seen directly by camera rays (paths of length 0 carry no
 * radiance to the cache). */
typedef struct {
  const float* density;
  int32_t nx, ny, nz;
  float density_max;
  const float* tf_rgba;
  int32_t tf_points;
  const float* lights;
  int32_t n_lights;
  const float* spheres;
  int32_t n_spheres;
} gsc_volume;

/* Light-transport estimator of the tracer (Method: "Path Termination Heuristics"; the
 * evaluation's uniform and next-event-estimation baselines). */
enum {
  /* Next-event estimation at every real collision: each point light directly; each sphere
   * light by one direction uniform in the cone it subtends (solid-angle pdf
   * 1 / (2 pi (1 - cos theta_max))), blocked if another sphere light is nearer along it, else
   * ratio-tracked; combined with the phase-sampled continuation (pdf 1/(4 pi)) that leaves the
   * volume and hits the light, by the power heuristic. */
  GSC_STRATEGY_NEE = 0,
  /* Phase sampling only: radiance is gathered only when a continuation leaves the volume and
   * hits a sphere light (weight 1); point lights contribute nothing. */
  GSC_STRATEGY_UNIFORM = 1
};

/* HOST.  Tracer parameters.  Random numbers: Philox4x32-10 with key (lo32(seed), hi32(seed))
 * and counter (y * full_w + x, sample, frame, j); draw k of a path is word k mod 4 of block
 * j = k / 4; u = (word >> 8) * 2^-24.  Draw order at a real collision: the point lights'
 * shadow rays, then per sphere light two draws for the cone direction and (unless blocked)
 * its shadow ray, then Algorithm 1's draw, then two for the phase direction.  C: the
 * termination coefficient of Algorithm 1 (C_inf != 0 disables the heuristic); eps: the epsilon
 * of Algorithm 1 (0 by default).  With sphere lights, the B-th collision still samples a
 * continuation (no Algorithm 1 there): if it leaves the volume it may hit a light, if it
 * collides the path ends with n = B. */
typedef struct {
  uint64_t seed;
  uint32_t frame;
  uint32_t spp;            /* >= 1; targets are the mean over samples                      */
  uint32_t max_bounces;    /* B >= 1: paths stop after B real collisions                   */
  uint32_t num_levels;     /* K: paths of length n >= K write level K-1                    */
  float C;
  int32_t C_inf;
  float eps;
  uint32_t strategy;       /* GSC_STRATEGY_NEE (0) or GSC_STRATEGY_UNIFORM (1)             */
} gsc_trace_params;

/* DEVICE, one per path ([spp][h][w], sample-major): the path's accumulated radiance L, the product
 * beta of the survival probabilities of Algorithm 1 at termination (Eq. 3), its length n
 * (real collisions) in the low 16 bits of n_kind and the termination kind in the high 16 bits:
 * 0 no interaction, 1 left the volume, 2 reached max_bounces, 3 terminated early. */
typedef struct {
  float L[3];
  float beta;
  uint32_t n_kind;
} gsc_path_record;

enum { GSC_KIND_ESCAPE0 = 0, GSC_KIND_ESCAPE = 1, GSC_KIND_MAXDEPTH = 2, GSC_KIND_EARLY = 3 };

/* HOST.  Per-call counters and stage times (milliseconds, from HIP events). */
typedef struct {
  double ms_project_bin, ms_forward, ms_trace, ms_loss, ms_backward, ms_adam, ms_total;
  uint64_t gaussians, instances, tiles, pixels, paths, path_vertices;
  double loss;
  int32_t adam_skipped;    /* 1 when the loss was not finite and no parameter was written  */
} gsc_frame_stats;

/* HOST.  Counts plus DEVICE pointers into a binning object, for inspection.  Per-Gaussian
 * arrays are indexed by the concatenation of the levels (level l starts at gauss_offset[l]). */
typedef struct {
  uint64_t n_instances;
  uint64_t n_tiles;        /* sum over levels of TX * TY                                   */
  int32_t num_levels, tiles_x, tiles_y;
  int64_t gauss_offset[9];
  const uint32_t* values;  /* [n_instances] level-local Gaussian ids, sorted by (tile, depth, id) */
  const uint64_t* ranges;  /* [n_tiles][2] per-tile [start, end); (0, 0) when empty          */
  const int32_t* window;   /* [sum n][4] inclusive pixel window px0, px1, py0, py1 (0 if culled) */
  const uint32_t* tiles_touched; /* [sum n]; 0 when culled                                  */
  const uint32_t* depth_key; /* [sum n] bits of the camera-space z; 0xFFFFFFFF when culled   */
  const float* screen;     /* [sum n][6] u, v, conic A, B, C, opacity                        */
} gsc_binning_info;

/* HOST.  AdamW hyper-parameters of one parameter group; lr already includes the Eq. 5 factor.
 * Doubles: the step factors are formed in double on the host before rounding to fp32. */
typedef struct {
  double lr, beta1, beta2, eps, weight_decay;
  int64_t step;            /* >= 1: the bias-correction step                                */
} gsc_adam_hparams;

/* HOST.  One frame of one viewer of one scene. */
typedef struct {
  gsc_camera cam;
  gsc_trace_params trace;  /* num_levels must equal the scene's K; 1 <= spp <= 4096: the   *
                            * splat, loss and optimiser step run once whatever spp is       */
  int32_t loss;            /* 0 = L2, 1 = HDR (Eq. 4)                                      */
  int32_t train;           /* 0: render only (no backward, no optimiser step)              */
  uint32_t viewport_frames;/* t >= 1 of Eq. 5                                               */
  double lr[5];            /* pos, rot, log_scale, rgb, opacity_logit (before Eq. 5)       */
  double beta1, beta2, eps, weight_decay;
} gsc_frame_request;

/* ---- context ------------------------------------------------------------------------- */
/* Creates a context on `device` that enqueues on `hip_stream` (NULL: the null stream).
 * `alloc` may be NULL.  Synchronises nothing. */
gsc_status gsc_ctx_create(int device, void* hip_stream, const gsc_allocator* alloc, gsc_ctx** out);
void gsc_ctx_destroy(gsc_ctx* ctx);
/* HOST string, valid until the next call on ctx. */
const char* gsc_ctx_last_error(const gsc_ctx* ctx);
gsc_status gsc_ctx_set_stream(gsc_ctx* ctx, void* hip_stream);
/* on != 0: the splat adjoint (gsc_splat_backward, and the training step of gsc_render_frame /
 * gsc_render_frames) sums each Gaussian's per-tile gradient partials as 64-bit fixed-point
 * integers instead of float atomics, so its gradients, and the parameters AdamW then writes, are
 * the same bit for bit on every run.  A first pass over the tiles finds the largest |partial| of
 * each gradient component of each Gaussian; a second rounds every partial to 2^-41 of that and
 * adds the integers; the sum converts back to float.  The result differs from the float-atomic
 * one by the rounding of the partials (a relative 2^-41 of the largest partial each) and of the
 * float sums.  Costs a second pass of the adjoint and 108 bytes of device memory per Gaussian.
 * Off by default; the setting stays until changed.  Returns GSC_E_INVALID_ARG for a NULL ctx. */
gsc_status gsc_ctx_set_deterministic(gsc_ctx* ctx, int32_t on);
/* Frames (gsc_render_frame / gsc_render_frames) bin each tile's list only up to the depth by
 * which every pixel of the tile has surely stopped blending (on by default): a Gaussian whose
 * splat gives alpha >= o/2 over all pixels of a tile multiplies their transmittance by at most
 * 1 - o/2, and once these factors reach 0.5e-4 no later entry can be blended (blending stops
 * below 1e-4), so the cut lists give the same images, gradients and parameter updates as the
 * full ones with fewer instances.  gsc_project_bin builds full lists unless
 * gsc_ctx_set_frame_binning is on. */
gsc_status gsc_ctx_set_list_cut(gsc_ctx* ctx, int32_t on);
/* on != 0: gsc_project_bin bins the way the frame calls do: 32x32-pixel tiles (the views then
 * report tiles of that size and the keys carry those tile indices) and, when the list cut is
 * on, cut tile lists.  The splat forward and adjoint results do not depend on the tiling, so
 * this is how the frames' binning and kernels are compared with the oracle at full size.
 * Default off: 16x16 tiles, full lists (the binning the oracle's keys and ranges follow). */
gsc_status gsc_ctx_set_frame_binning(gsc_ctx* ctx, int32_t on);
/* The tile edge, in pixels, that frames (gsc_render_frame / gsc_render_frames) bin with: 16,
 * 32, or 0 for automatic (the default): 32 when every request of the batch spans at least
 * 6144 tiles of 32x32 pixels over its levels (1920x1080 with four levels spans 8160), else 16.
 * Larger tiles give shorter binning (fewer instances), smaller ones more parallel work and
 * shorter lists for the splat kernels.  Images, gradients and
 * parameter updates do not depend on the tiling beyond float summation order.  Returns
 * GSC_E_INVALID_ARG for a NULL ctx or any other size. */
gsc_status gsc_ctx_set_frame_tiles(gsc_ctx* ctx, int32_t tile_px);
/* After GSC_E_CAPACITY: the instance count the failed call needed. */
uint64_t gsc_ctx_required_capacity(const gsc_ctx* ctx);
/* Per-kernel timing: while on, every kernel launch of the context is bracketed by HIP events
 * recorded on the stream it is launched on; turning it on clears the totals.  Costs two event
 * records per launch. */
gsc_status gsc_ctx_profile(gsc_ctx* ctx, int32_t on);
/* Synchronises on the recorded events and returns kernel `index`'s name (HOST buffer of
 * name_len bytes), total milliseconds and launch count since profiling was turned on;
 * GSC_E_INVALID_ARG past the last index. */
gsc_status gsc_ctx_profile_read(gsc_ctx* ctx, int32_t index, char* name, size_t name_len,
                                double* total_ms, int64_t* launches);
/* Work counters since profiling was last turned on (HOST struct).  The splat counters count
 * pairs of the cache-image forward (the front-to-back blend): per pixel, `contributors` sums the
 * position of its last blended entry (the length of the adjoint's walk); `tile_entries` sums,
 * per tile wavefront, the entries it evaluated after the tile-ellipse cull.  While
 * gsc_ctx_set_work_counters is on, also `evaluations` (per pixel, the list entries it examined
 * before it finished: its termination position, or the list length), `blended` (the entries it
 * blended, alpha >= 1/255 before termination) and the fwd_* and bwd_* counters. */
typedef struct gsc_counters {
  uint64_t instances;      /* (tile, Gaussian) instances binned */
  uint64_t binnings;       /* binnings run */
  uint64_t evaluations;
  uint64_t blended;
  uint64_t contributors;
  uint64_t tile_entries;
  /* Counted only while gsc_ctx_set_work_counters is on (the kernels' counting variants): */
  uint64_t fwd_tested;     /* forward: (pixel, entry) pairs evaluated (pixels live in the
                              Gaussian's window when the entry was walked) */
  uint64_t fwd_slots;      /* forward: 64-pixel slot evaluations (one wave instruction stream) */
  uint64_t bwd_tested;     /* adjoint: (pixel, entry) pairs evaluated */
  uint64_t bwd_blended;    /* adjoint: pairs that blended (alpha >= 1/255, before the stop) */
  uint64_t bwd_slots;      /* adjoint: 64-pixel slot evaluations */
  uint64_t bwd_entries;    /* adjoint: (tile, entry) pairs walked after the tile-ellipse cull */
  uint64_t bwd_atomics;    /* adjoint: float atomics issued into the screen-space gradients */
  uint64_t bwd_records;    /* adjoint: (tile, Gaussian) partials flushed, each as up to nine
                              atomics into one 64-byte record (one memory request) */
  uint64_t frame_retries;  /* frames run again because their binning outgrew the capacity sized
                              from the previous frame (see gsc_render_frame) */
} gsc_counters;
/* Fills *out; synchronises the context's stream.  GSC_E_INVALID_ARG for NULL. */
gsc_status gsc_ctx_counters(gsc_ctx* ctx, gsc_counters* out);
/* on != 0: later splat launches on ctx run counting variants of the forward and adjoint kernels
 * that also fill the fwd_* and bwd_* counters (a few scalar instructions per slot; the default
 * kernels do not count them).  For measurement only; results are unchanged. */
gsc_status gsc_ctx_set_work_counters(gsc_ctx* ctx, int32_t on);
/* Frees the context's cached workspace (binning buffers, frame scratch). */
gsc_status gsc_ctx_trim(gsc_ctx* ctx);

/* ---- ceiling micro-benchmarks (measurement only) ----------------------------------------
 * Each enqueues one kernel on the context's stream between two events, waits for it, and
 * writes its duration in milliseconds to *ms (HOST).  threads: a positive multiple of 256.
 * They measure the ceilings the hot-path kernels are compared with: the tracer's random reads
 * of a density grid, the adjoint's float atomics, and the splat kernels' vector ALU. */
/* threads x per_thread random 32-byte reads (per_thread a multiple of 8) from `cells`, an array
 * of n_cells 32-byte cells; out [threads] receives one sum per thread. */
gsc_status gsc_probe_gather(gsc_ctx* ctx, const void* cells, uint64_t n_cells, uint32_t threads,
                            int32_t per_thread, float* out, double* ms);
/* threads x per_thread float atomic adds of 1 to random elements of buf [n]. */
gsc_status gsc_probe_atomics(gsc_ctx* ctx, float* buf, uint64_t n, uint32_t threads,
                             int32_t per_thread, double* ms);
/* threads x iters x 8 independent fp32 FMAs (mode 0) or exponentials exp(x) evaluated as
 * 2^(x log2 e) (mode 1); out [threads] receives one value per thread. */
gsc_status gsc_probe_valu(gsc_ctx* ctx, float* out, uint32_t threads, int32_t iters, int32_t mode,
                          double* ms);

/* ---- the hot path ----------------------------------------------------------------------- */
/* Delta-tracking volume path tracer with next-event estimation to every light (ratio-tracked
 * shadow transmittance, isotropic phase 1/(4 pi); sphere lights combined with phase sampling
 * by MIS) or phase sampling only (params->strategy), Algorithm 1 early termination with the
 * cumulative throughput reading and beta of Eq. 3, at most max_bounces real collisions; one
 * path per pixel of the camera window per sample (Method: "Path Termination Heuristics",
 * "Cache Sampling", "Cache Training").
 * targets: [K][h][w][3], written completely: level min(n,K)-1 of pixel p receives the
 * path's accumulated radiance (next-event estimates plus light hits on leaving the volume),
 * every other level 0; mean over spp.
 * records: [spp][h][w] gsc_path_record (sample s of pixel p at s h w + p), or NULL.
 * stats: HOST or NULL; non-NULL synchronises the stream and fills ms_trace, paths and
 * path_vertices. */
gsc_status gsc_trace_targets(gsc_ctx* ctx, const gsc_volume* vol, const gsc_camera* cam,
                             const gsc_trace_params* params, float* targets,
                             gsc_path_record* records, gsc_frame_stats* stats);

/* Projects every Gaussian of num_levels levels to a screen-space conic (3D Gaussian
 * splatting, the rasteriser the paper adapts; Method: "A Path Space Radiance Cache") and bins
 * them into 16x16 tiles: all levels share one tile-key space (level l's tiles follow level
 * l-1's), and each tile's list is sorted by (depth, id), i.e. the instances come out sorted by
 * the 64-bit key (tile << 32) | bits(depth) with ties broken by Gaussian id.
 * capacity_hint: 0 sizes the instance buffer exactly (one device->host read of the count);
 * otherwise it is used as the capacity and GSC_E_CAPACITY is returned (after synchronising)
 * if the frame needs more.  On success *out holds a binning object that must be released
 * with gsc_binning_release. */
gsc_status gsc_project_bin(gsc_ctx* ctx, const gsc_gaussians* levels, int32_t num_levels,
                           const gsc_camera* cam, uint64_t capacity_hint, gsc_binning** out);
/* Synchronises; fills HOST counts and DEVICE pointers (valid until the object is released). */
gsc_status gsc_binning_view(gsc_ctx* ctx, const gsc_binning* bin, gsc_binning_info* out);
/* Writes the 64-bit sort keys [n_instances] ((global tile << 32) | bits(depth)) of the
 * binned instances to `keys` (DEVICE, caller-owned).  The sort itself never materialises
 * them. */
gsc_status gsc_binning_keys(gsc_ctx* ctx, const gsc_binning* bin, uint64_t* keys);
void gsc_binning_release(gsc_ctx* ctx, gsc_binning* bin);

/* Rasterisation of the cache images (Method: "A Path Space Radiance Cache": every frame each
 * level is splatted with the 3D Gaussian splatting rasteriser before the tracer runs).
 * Front-to-back alpha blending of every level's tiles: per pixel, over the tile list in
 * order, alpha = min(0.99, o exp(power)), pairs with power > 0, alpha < 1/255 or the pixel
 * outside the Gaussian's window are skipped, and blending stops before T (1 - alpha) < 1e-4;
 * background 0.  images [K][h][w][3], final_T [K][h][w], last_id [K][h][w] (level-local id of
 * the last blended Gaussian, -1 when none).  The object keeps each pixel's list position of
 * its last contributor for gsc_splat_backward. */
gsc_status gsc_splat_forward(gsc_ctx* ctx, gsc_binning* bin, float* images, float* final_T,
                             int32_t* last_id);

/* The gradient step of cache training (Method: "Cache Training": the levels are optimised
 * every frame against the traced per-length targets; "Optimization and Hyperparameters").
 * Adjoint of gsc_splat_forward followed by the adjoint of the projection: given dL/dimages
 * [K][h][w][3], writes the gradients of all 14 parameters of every Gaussian of every level
 * (grads[l] has the shapes of levels[l]; overwritten).  Walks each tile back to front from
 * the stored last contributor, recovering transmittance from final_T by division (no
 * per-pixel lists).  levels and cam must be those given to gsc_project_bin. */
gsc_status gsc_splat_backward(gsc_ctx* ctx, const gsc_binning* bin, const gsc_gaussians* levels,
                              int32_t num_levels, const gsc_camera* cam, const float* final_T,
                              const int32_t* last_id, const float* dL_dimages,
                              const gsc_grads* grads);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same adjoint as gsc_splat_backward, same
 * arguments and results, but its temporaries (screen-space and parameter gradients before they
 * are copied out, the tile schedule) live in one static device array of the library, 64.0 MB
 * per device, held until the process ends; it calls no hipMalloc / hipFree and no allocator
 * hook.  Limits: at most 524,288 Gaussians (all levels together) and 262,144 tiles per call,
 * else GSC_E_INVALID_ARG with a message and nothing enqueued.  Sums with float atomics:
 * GSC_E_INVALID_ARG while the deterministic mode is on.  Every call on a device shares that
 * device's array, so calls that overlap on one device (several contexts or streams) race; calls
 * ordered on one stream do not.  GSC_E_DEVICE if the array's address could not be obtained. */
gsc_status gsc_splat_backward_noalloc(gsc_ctx* ctx, const gsc_binning* bin,
                                      const gsc_gaussians* levels, int32_t num_levels,
                                      const gsc_camera* cam, const float* final_T,
                                      const int32_t* last_id, const float* dL_dimages,
                                      const gsc_grads* grads);

/* Per level l, with prediction y = images[l] and noisy target x = targets[l]: L2 (loss 0) or
 * the HDR loss of Eq. 4, (y - x)^2 / (sg(max(y,0)) + 0.01)^2 (loss 1), averaged over the
 * 3 w h elements of the level and summed over levels; writes dL/dimages [K][h][w][3] and the
 * loss (DEVICE scalar, fp32).  If records is not NULL also writes the cached composite image
 * [h][w][3]: early termination -> max(cache, 0) / beta; natural termination with nonzero
 * radiance -> the radiance, with zero radiance -> max(cache, 0) / beta; no interaction -> 0,
 * where cache = images[min(n,K)-1] (Method: "Natural Path Termination", Eq. 3).  records
 * holds spp >= 1 samples per pixel ([spp][h][w]); the composite pixel is the mean of its
 * samples' values, summed in sample order. */
gsc_status gsc_loss_composite(gsc_ctx* ctx, const float* images, const float* targets,
                              const gsc_path_record* records, int32_t spp, int32_t num_levels,
                              int32_t w, int32_t h, int32_t loss, float* dL_dimages,
                              float* loss_out, float* composite);

/* One AdamW step over `count` elements (Method: "Regularization"): m = b1 m + (1-b1) g;
 * v = b2 v + (1-b2) g^2; p = p (1 - lr wd); p = p - s1 m / (sqrt(v) s2 + eps) with
 * s1 = lr / (1 - b1^step), s2 = 1 / sqrt(1 - b2^step) computed in double on the host; every
 * fp32 operation separately rounded.  In-place on param, m, v. */
gsc_status gsc_adam_step(gsc_ctx* ctx, float* param, float* m, float* v, const float* grad,
                         int64_t count, const gsc_adam_hparams* hp);

/* ---- cache initialisation (Method: "Cache Initialization", Eq. 2) ------------------------ */
/* n points of first interaction of random rays with the volume (delta tracking against the
 * majorant; a ray that leaves the cube is replaced by a new one, up to 4096 per point), with
 * the transfer function's colour at the point as albedo.  Point i's attempt a draws from the
 * Philox4x32-10 stream keyed by seed with counter (i, a, 0x494E4954, block): a point p uniform
 * in the cube, a direction w uniform on the sphere, the ray starting at p - 2 w.  vol: density
 * DEVICE, TF HOST (lights unused).  pos, albedo: DEVICE [n][3] fp32, caller-owned.
 * GSC_E_INVALID_ARG for bad arguments or if some point found no interaction (a volume that is
 * transparent under its TF); then pos/albedo are partially written. */
gsc_status gsc_init_points(gsc_ctx* ctx, const gsc_volume* vol, int64_t n, uint64_t seed,
                           float* pos, float* albedo);
/* For each of n points (DEVICE [n][3], in the unit cube) the mean Euclidean distance to its 3
 * nearest other points (uniform grid, rings searched outward until exact).  mean3: DEVICE [n].
 * n >= 4. */
gsc_status gsc_knn_mean3(gsc_ctx* ctx, const float* pos, int64_t n, float* mean3);
/* K cache levels from one sampling pass: n points as gsc_init_points; level l takes the first
 * n >> l of them (the points are i.i.d., so a prefix is a uniform sub-sample, sum_l n / 2^l in
 * total), isotropic scale s_i = min(mu + 2 sigma, m_i) / 2 (Eq. 2; m_i the mean 3-NN distance
 * within the level, mu and sigma its mean and population standard deviation), identity
 * rotation, log-scale log(s_i) on all axes, the albedo as colour, opacity 0.1 (logit).
 * levels[l].n must equal n >> l, and n >> (K - 1) >= 4.  Arrays DEVICE, caller-owned. */
gsc_status gsc_cache_init(gsc_ctx* ctx, const gsc_volume* vol, int64_t n, int32_t K, uint64_t seed,
                          const gsc_level_buffers* levels);

/* ---- scenes and frames ------------------------------------------------------------------ */
/* A scene keeps resident on the device: its volume grid in a cell-corner layout (for every
 * trilinear cell the eight clamped corner values, 32 bytes, (nx+1)(ny+1)(nz+1) cells, so a
 * tracer lookup reads one aligned 32-byte block; built from vol->density, which the caller may
 * free once the call's stream work is done), its TF and lights, and K levels of parameters with
 * their Adam moments and step counter (copied from init_levels). */
gsc_status gsc_scene_create(gsc_ctx* ctx, const gsc_volume* vol, const gsc_gaussians* init_levels,
                            int32_t K, gsc_scene** out);
void gsc_scene_destroy(gsc_ctx* ctx, gsc_scene* scene);
/* Replaces the TF, point lights and sphere lights (HOST arrays as in gsc_volume; a
 * transfer-function edit or a light move). */
gsc_status gsc_scene_set_optics(gsc_ctx* ctx, gsc_scene* scene, const float* tf_rgba,
                                int32_t tf_points, const float* lights, int32_t n_lights,
                                const float* spheres, int32_t n_spheres);
/* DEVICE pointers to the scene's current parameters of level l. */
gsc_status gsc_scene_level(const gsc_scene* scene, int32_t l, gsc_gaussians* out);
/* DEVICE pointers to level l's optimiser state: params, m and v are each [14 n] floats laid out
 * [pos 3n][rot 4n][log_scale 3n][rgb 3n][opacity_logit n]; *step (HOST) is the number of AdamW
 * steps taken.  The step count is kept on the device, where a frame advances it only when its
 * update ran (a frame with a non-finite loss skips AdamW and leaves moments and count as they
 * were), so this call waits for the device before it reads the count.  The pointers are valid
 * until the scene is destroyed. */
gsc_status gsc_scene_state(const gsc_scene* scene, int32_t l, float** params, float** m, float** v,
                           int64_t* n, int64_t* step);
/* Copies parameters, moments and step counters from src to dst (same level sizes). */
gsc_status gsc_scene_copy_state(gsc_ctx* ctx, gsc_scene* dst, const gsc_scene* src);
/* Checkpoint of the cache's optimiser state (all levels' parameters, AdamW moments and step
 * counts) to the HOST file `path`: one JSON header line
 *   {"format":"gsc-scene-state","version":1,"dtype":"float32","byte_order":"little",
 *    "levels":[{"n":N,"step":S},...]}
 * (written without the line break shown here) and a newline, then per level params, m and v,
 * each 14 n little-endian float32 in the layout of gsc_scene_state.  The volume, transfer
 * function and lights are not saved (they belong to the scene's creation and gsc_scene_set_optics),
 * nor is Eq. 5's viewport count, which each frame request carries.  Waits for the work already
 * enqueued on the context's stream, then copies through host memory; synchronous.  A failed write
 * returns GSC_E_INVALID_ARG and leaves an incomplete file. */
gsc_status gsc_scene_save(gsc_ctx* ctx, const gsc_scene* scene, const char* path);
/* Restores a state written by gsc_scene_save into `scene`, whose level count and sizes must
 * equal the file's.  The header, the level sizes and the file length are checked before the
 * device is touched (GSC_E_INVALID_ARG, scene unchanged); the copies are ordered after the
 * work already enqueued on the context's stream and complete before the call returns. */
gsc_status gsc_scene_load(gsc_ctx* ctx, gsc_scene* scene, const char* path);
/* Resident bytes: the cell-corner grid (32 (nx+1)(ny+1)(nz+1)) + 3 x 14 fp32 per Gaussian
 * (parameters and two moments). */
size_t gsc_scene_footprint_bytes(const gsc_scene* scene);
/* Transient bytes one frame of w x h at one sample per pixel needs, for an instance
 * estimate; each further sample per pixel adds 20 bytes per pixel (its path records). */
size_t gsc_frame_footprint_bytes(const gsc_scene* scene, int32_t w, int32_t h,
                                 uint64_t instance_estimate);

/* One frame (Method, per-frame protocol): splat all K levels into cache images (one key
 * space, one launch per stage), trace the targets on a second stream meanwhile, then the
 * loss, the cached composite into `image` ([h][w][3]), and -- when req->train -- the splat
 * backward and one AdamW step per parameter group with lr x 1/(1 + ln t) (Eq. 5).  A
 * non-finite loss skips the step.  stats: HOST or NULL (non-NULL synchronises).
 * Sizing: a context's first frame reads its instance count back before placing; later frames
 * size the tile lists from the previous frame's count plus a quarter, enqueue the whole frame,
 * and then wait only for the placement's count to reach the host (no stream synchronisation;
 * the device has the rest of the frame queued).  If the lists did not fit, the splats and the
 * AdamW step skip themselves on the device and the call runs the frame again with room for
 * the count (counted in gsc_counters.frame_retries); results equal those of a frame sized
 * exactly. */
gsc_status gsc_render_frame(gsc_ctx* ctx, gsc_scene* scene, const gsc_frame_request* req,
                            float* image, gsc_frame_stats* stats);

/* A batch of n frames of distinct scenes, executed stage by stage with one launch per stage
 * over all (request, level) pairs.  The scenes must be pairwise distinct (one training step
 * per scene per batch).  images[i] is request i's composite [h_i][w_i][3]; stats: HOST array
 * of n or NULL.  Results equal n separate gsc_render_frame calls up to float-atomic order,
 * and bit for bit with gsc_ctx_set_deterministic. */
gsc_status gsc_render_frames(gsc_ctx* ctx, gsc_scene* const* scenes,
                             const gsc_frame_request* reqs, float* const* images, int32_t n,
                             gsc_frame_stats* stats);

/* Enqueues a copy of `bytes` bytes between two device (or pinned host) buffers on the
 * context's stream.  A convenience for bindings that read the DEVICE pointers of a view. */
gsc_status gsc_copy(gsc_ctx* ctx, void* dst, const void* src, size_t bytes);
/* Waits for all work enqueued on the context's stream. */
gsc_status gsc_ctx_synchronize(gsc_ctx* ctx);

/* ---- debug builds ---------------------------------------------------------------------- */
/* A library built with -DGSC_DEBUG (libgsc_debug.so) checks on the device the accesses whose
 * indices come from data: each instance store of the binning against the tile lists' capacity,
 * the placement's compaction queue against its ring, and each tile-list entry the splat kernels
 * read against the capacity and its level's Gaussian count.  A failed check skips the access and
 * records itself; after every call the library waits for the device, and a call during which a
 * check failed returns GSC_E_DEVICE with gsc_ctx_last_error() naming the checks.  Other builds
 * compile no check.  This call makes the check path fire on purpose (one flag set by a kernel,
 * no access skipped): GSC_E_DEVICE naming "self-test" in a debug build, GSC_E_UNSUPPORTED in
 * others. */
gsc_status gsc_debug_selftest(gsc_ctx* ctx);

/* HOST, side-effect free: sizes of the structs above, for bindings to check their layouts:
 * which = 0 camera, 1 gaussians, 2 grads, 3 volume, 4 trace_params, 5 path_record,
 * 6 frame_stats, 7 binning_info, 8 adam_hparams, 9 frame_request, 10 allocator, 11 counters,
 * 12 level_buffers;
 * 0 for any other value. */
size_t gsc_abi_struct_size(int32_t which);

#ifdef __cplusplus
}
#endif
#endif /* GSC_H_ */
