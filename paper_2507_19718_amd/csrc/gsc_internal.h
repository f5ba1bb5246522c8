// gsc_internal.h -- structures shared by the host runtime and the HIP kernels of the GSCache
// hot path (not part of the public ABI).
//
// A *batch* is a list of segments; a segment is one cache level of one frame request.  Every
// kernel of the splat path runs once per stage over all segments of a batch: per-Gaussian
// arrays are concatenated (segment s owns [g_off, g_off + n)), per-pixel arrays likewise
// ([pix_off, pix_off + w h)), and the tiles of all segments share one key space
// ([tile_base, tile_base + TX TY)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gsc.h"

namespace gsc {

constexpr int kTile = 16;               // 16x16 pixel tiles (gsc_project_bin and its views)
constexpr int kTileShift = 4;
// Large frames bin 32x32 tiles.  The adjoint walks one with two independent wavefronts, each a
// 16x32 half with eight pixels per lane (the per-entry work, record broadcast, window masks and
// reductions, is shared by eight pixels); the forward walks it with four independent 16x16
// wavefronts.  The tile lists hold about a third of the instances of 16x16 tiles.
constexpr int kFrameTileShiftX = 5;
constexpr int kFrameTileShiftY = 5;
// Frames bin 32x32 tiles when each request of the batch spans at least this many of them over
// its levels (1920x1080 with four levels: 8160), else 16x16.  Measured on 1M-Gaussian levels:
// 32x32 tiles win 10 % at 1080p with four levels, tie at 1080p with three, and lose 20-110 %
// at 720p and 360p, where the longest tile list sets the splat adjoint's time.
constexpr int64_t kAutoTiles32 = 6144;
// The adjoint's screen-space gradients: one 64-byte record of 16 floats per Gaussian, [G][16]
// (du, dv, dA, dB, dC, do, dr, dg, db, then 7 unused).  The nine float atomics of a (tile,
// Gaussian) partial then fall in one aligned 64-byte line, and the adjoint issues them from nine
// lanes of one instruction, which the memory system carries as one request.
constexpr int kGrad2dStride = 16;
constexpr int kMaxTf = 64;
constexpr int kMaxLights = 8;
constexpr int kChunk = 1024;            // depth-ordered Gaussians per binning chunk

struct DevCam {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t full_w, full_h, x0, y0, w, h;
  float znear;
};

struct Seg {
  const float* pos;
  const float* rot;
  const float* ls;
  const float* rgb;
  const float* logit;
  int64_t n;
  int64_t g_off;        // per-Gaussian offset
  int64_t tile_base;    // first global tile
  int64_t pix_off;      // per-pixel offset (w h per segment)
  int64_t chunk_off;    // first binning chunk (chunks of kChunk depth-ordered Gaussians)
  int32_t n_chunks;
  int32_t cam;
  int32_t TX, TY;
  int32_t level;
  int32_t request;
  int32_t tsx, tsy;     // log2 of the tile width and height: 16x16 (4, 4) or, in frames, 32x32
};

// Per request of a trace launch.
struct TraceDesc {
  const float* density;   // [nz][ny][nx], used when cells is NULL
  const float4* cells;    // cell-corner layout (see launch_build_cells) or NULL
  int32_t nx, ny, nz;
  float dmax, majorant;
  int32_t P, n_lights, n_spheres;
  uint32_t strategy;      // GSC_STRATEGY_NEE or GSC_STRATEGY_UNIFORM
  float tf[kMaxTf * 4];
  float lights[kMaxLights * 6];
  float spheres[kMaxLights * 7];   // centre xyz, radius, radiance rgb
  DevCam cam;
  uint64_t seed;
  uint32_t frame, spp, max_bounces, K;
  float C;
  int32_t C_inf;
  float eps;
  int64_t pix_off;      // first launch index of this request (a multiple of the block size)
  float* targets;       // [K][h][w][3]
  void* records;        // [spp][h][w] x 20 B or NULL
};

// Per-Gaussian projected record, 48 B, gathered by the splat kernels:
//   q0 = (u, v, A, B), q1 = (Cc, o, r, g), q2 = (b, px0|px1<<16, py0|py1<<16, id)
struct alignas(16) SplatRec {
  float4 q0, q1, q2;
};

// ---- launchers (all enqueue on `st`) ---------------------------------------------------------
// Cell-corner layout of a density grid: for every trilinear cell (x0, y0, z0) in [-1, n-1]^3 the
// eight clamped corner values, 32 bytes, so one lookup reads one aligned 32-byte block.
size_t cells_bytes(int nx, int ny, int nz);
hipError_t launch_build_cells(hipStream_t st, const float* density, int nx, int ny, int nz,
                              float4* cells);
// Cache initialisation (k_trace.hip: points; k_init.hip: neighbours, Eq. 2, levels).
hipError_t launch_init_points(hipStream_t st, const TraceDesc* desc, int64_t n, int max_attempts,
                              float* pos, float* albedo, int32_t* tries);
int init_grid_side(int64_t n);
hipError_t launch_grid_keys(hipStream_t st, const float* pos, int64_t n, int G, uint32_t* key,
                            uint32_t* id);
hipError_t launch_cell_ranges(hipStream_t st, const uint32_t* key, const uint32_t* id, const float* pos,
                              int64_t n, uint32_t* start, uint32_t* end, float4* spos);
hipError_t launch_knn3(hipStream_t st, const float4* spos, const uint32_t* id, int64_t n, int G,
                       const uint32_t* start, const uint32_t* end, float* mean3);
int init_moment_blocks();
size_t init_partial_doubles();
hipError_t launch_count_failed(hipStream_t st, const int32_t* tries, int64_t n,
                               unsigned long long* out);
hipError_t launch_init_level(hipStream_t st, const float* mean3, int64_t n, const float* pos,
                             const float* albedo, float opacity_logit, double* partial, float* gpos,
                             float* grot, float* gls, float* grgb, float* glogit);
hipError_t launch_project(hipStream_t st, const Seg* segs, const int64_t* seg_gstart, int S,
                          const DevCam* cams, int64_t G, SplatRec* rec, uint32_t* depth_key,
                          uint64_t* rect, uint32_t* tiles, uint32_t* ids, uint64_t* core);
hipError_t launch_project_backward(hipStream_t st, const Seg* segs, const int64_t* seg_gstart, int S,
                                   const DevCam* cams, int64_t G, const float* grad2d,
                                   float* grads14);
struct AdamGroup;
// The same chain rule followed, per Gaussian, by its AdamW step: groups[5 s + k] holds parameter
// group k (pos, rot, log_scale, rgb, opacity_logit) of segment s, with p, m, v at the group's
// base; segments whose p is NULL are not trained.  No gradient array is written.
hipError_t launch_project_backward_adam(hipStream_t st, const Seg* segs, const int64_t* seg_gstart,
                                        int S, const DevCam* cams, int64_t G, const float* grad2d,
                                        const AdamGroup* groups);
hipError_t launch_fill_u32(hipStream_t st, uint32_t* p, uint32_t value, int64_t count);

size_t sort_table_bytes(int n_blocks, int S);
size_t sort_hist_words(int n_blocks, int S);
int sort_count_blocks(const int64_t* seg_n, int S);
void sort_fill_table(void* host, const int64_t* seg_n, const int64_t* seg_off, int S);
hipError_t launch_segmented_sort(hipStream_t st, const void* table_dev, int n_blocks, int S,
                                 uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp,
                                 uint32_t* vals_tmp, uint32_t* hist);

size_t bin_work_bytes(int S);
int64_t bin_fill_work(void* host, const Seg* segs, int S, int64_t* total_chunk_tiles,
                      int64_t* total_count_blocks, int64_t* total_regions);
size_t bin_scan_partials(int64_t n_tiles);
hipError_t launch_gather_rect(hipStream_t st, const int64_t* seg_gstart, int S, int64_t G,
                              const uint32_t* sorted_ids, const uint64_t* rect,
                              uint64_t* rect_sorted, const uint64_t* core, uint64_t* core_sorted);
hipError_t launch_bin_count(hipStream_t st, const void* work_dev, int S, int64_t total_blocks,
                            const uint64_t* rect_sorted, uint32_t* counts,
                            const uint64_t* core_sorted, uint32_t* wsum);
hipError_t launch_bin_scan(hipStream_t st, const void* work_dev, int S, const int64_t* seg_tstart,
                           int64_t n_tiles, uint32_t* counts, uint32_t* tile_total,
                           uint64_t* partial, uint64_t* tile_start, uint64_t* ranges,
                           uint64_t* n_instances, const uint32_t* wsum, int32_t* cut,
                           int32_t* region_n);
hipError_t launch_bin_regions(hipStream_t st, int64_t n_regions, const int32_t* region_n,
                              uint64_t* region_start, uint64_t* n_blocks);
hipError_t launch_bin_place(hipStream_t st, const void* work_dev, int S, int64_t n_regions,
                            const uint64_t* region_start, const uint64_t* n_blocks,
                            int64_t grid_blocks, const uint32_t* sorted_ids,
                            const uint64_t* rect_sorted, const uint32_t* counts,
                            const uint64_t* tile_start, const uint64_t* n_instances,
                            uint64_t capacity, uint32_t* values, const int32_t* cut);
hipError_t launch_binning_keys(hipStream_t st, const int64_t* seg_tstart, int S,
                               const int64_t* seg_goff, int64_t n_tiles, const uint64_t* tile_start,
                               const uint64_t* n_instances, uint64_t n_host,
                               const uint32_t* values, const uint32_t* depth_key, uint64_t* keys);
hipError_t launch_view(hipStream_t st, int64_t G, const SplatRec* rec, const uint32_t* tiles,
                       int32_t* window, float* screen);

hipError_t launch_splat_forward(hipStream_t st, const Seg* segs, const int64_t* seg_tstart, int S,
                                const DevCam* cams, int64_t n_tiles, const uint64_t* ranges,
                                const uint32_t* values, const SplatRec* rec, float* images,
                                float* final_T, int32_t* last_id, uint32_t* n_contrib,
                                unsigned long long* stats, const uint32_t* order,
                                uint32_t* tile_work, bool count, int tsx, int tsy,
                                const uint64_t* n_inst, uint64_t capacity);
// Keys ordering tiles by decreasing work (work NULL: list length from ranges).
hipError_t launch_tile_order(hipStream_t st, const uint64_t* ranges, const uint32_t* work,
                             int64_t n_tiles, uint32_t* order);
// gmax NULL: float atomics into grad2d (zeroed by the caller).  Otherwise the deterministic
// fixed-point accumulation (gmax[9 G] and gfix[9 G] zeroed by the caller); grad2d is overwritten.
hipError_t launch_splat_backward(hipStream_t st, const Seg* segs, const int64_t* seg_tstart, int S,
                                 const DevCam* cams, int64_t n_tiles, const uint64_t* ranges,
                                 const uint32_t* values, const SplatRec* rec, const float* final_T,
                                 const uint32_t* n_contrib, const float* dL_dimages,
                                 float* grad2d, int64_t G, const uint32_t* order, uint32_t* gmax,
                                 unsigned long long* gfix, unsigned long long* stats, bool count,
                                 int tsx, int tsy, const uint64_t* n_inst, uint64_t capacity);

int64_t trace_align(int64_t pixels);
hipError_t launch_trace(hipStream_t st, const TraceDesc* descs, const int64_t* req_pstart, int R,
                        int64_t total_launch, unsigned long long* path_vertices);

int loss_num_partials(int64_t pixels);
hipError_t launch_loss_composite(hipStream_t st, const float* images, const float* targets,
                                 const void* records, int spp, int K, int w, int h, int loss,
                                 float* dL_dimages, double* partials, float* loss_out,
                                 float* composite);
// One AdamW parameter group of a fused multi-group step (hyper-parameters prepared on the host).
struct AdamGroup {
  float* p;
  float* m;
  float* v;
  const float* g;
  int64_t n;
  const float* guard;     // the step is skipped when *guard is not finite (nullptr: never)
  float b1, b2, omb1, omb2, s1, s2, wdf, eps;
  // Frames: the level's AdamW step count lives on the device.  launch_adam_factors sets s1, s2
  // from t = *step + 1 (in double from lr, beta1, beta2); launch_adam_commit advances *step
  // once the update ran, i.e. only when *guard is finite.  nullptr: s1, s2 given by the host.
  int64_t* step;
  double lr, b1d, b2d;
};
// Bias corrections of every group of the table from its device step count (groups whose p or
// step is NULL are left alone).
hipError_t launch_adam_factors(hipStream_t st, AdamGroup* groups, int n_groups);
// Advances the step count of each segment's level (groups[5 s]) whose update ran.
hipError_t launch_adam_commit(hipStream_t st, const AdamGroup* groups, int S);
// losses[0 .. n) = NaN when *n_inst > capacity, so the AdamW step that follows is skipped.
hipError_t launch_capacity_guard(hipStream_t st, const uint64_t* n_inst, uint64_t capacity,
                                 float* losses, int n);
hipError_t launch_adam(hipStream_t st, float* param, float* m, float* v, const float* grad,
                       int64_t count, float b1, float b2, float omb1, float omb2, float s1,
                       float s2, float wdf, float eps, const float* guard);

// Ceiling micro-benchmarks (k_probe.hip).  threads: a multiple of 256.
hipError_t launch_probe_gather(hipStream_t st, const float4* cells, uint64_t n_cells,
                               uint32_t threads, int per_thread, float* out);
hipError_t launch_probe_atomic(hipStream_t st, float* buf, uint64_t n, uint32_t threads,
                               int per_thread);
hipError_t launch_probe_valu(hipStream_t st, float* out, uint32_t threads, int iters, int mode);

// Device bounds checks of a debug build (-DGSC_DEBUG): the bits a failed check sets, and per
// translation unit that holds checks, the reader of its flag word (returns the bits set since
// the last read and clears them; ~0u if the word could not be read; always 0 in other builds).
enum : uint32_t {
  kDbgInstanceStore = 1u << 0,   // an instance id stored past the tile lists' capacity
  kDbgPlaceQueue = 1u << 1,      // the placement's compaction queue held more than its ring
  kDbgListEntry = 1u << 2,       // a tile list past the capacity, or naming a Gaussian past its level
  kDbgSelfTest = 1u << 31,       // set on purpose by gsc_debug_selftest
};
uint32_t debug_flags_bin();
uint32_t debug_flags_splat();
uint32_t debug_flags_probe();
hipError_t launch_debug_selftest(hipStream_t st);

}  // namespace gsc
