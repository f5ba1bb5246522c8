// runtime.hip -- host runtime behind the C ABI in include/gsc.h: contexts, device memory via the
// caller's allocator hook, argument validation, descriptor tables, stage orchestration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <mutex>
#include <vector>

#include "gsc_internal.h"

using namespace gsc;

namespace {

// ---------------------------------------------------------------------------------------------
// Memory
// ---------------------------------------------------------------------------------------------
struct Alloc {
  gsc_allocator hook{};
  bool has = false;
  void* get(size_t bytes) const {
    if (bytes == 0) bytes = 256;
    if (has) return hook.alloc(bytes, hook.user);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
  }
  void put(void* p) const {
    if (!p) return;
    if (has) hook.release(p, hook.user);
    else (void)hipFree(p);
  }
};

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  // Grow-only; contents are not preserved.
  bool ensure(const Alloc& a, size_t bytes) {
    if (bytes <= cap && p) return true;
    a.put(p);
    p = nullptr;
    cap = 0;
    size_t want = std::max<size_t>(bytes, 256);
    p = a.get(want);
    if (!p) return false;
    cap = want;
    return true;
  }
  void release(const Alloc& a) { a.put(p); p = nullptr; cap = 0; }
  template <typename T> T* as() const { return (T*)p; }
};

struct Fail {
  gsc_status st;
};

}  // namespace

// ---------------------------------------------------------------------------------------------
// Opaque objects
// ---------------------------------------------------------------------------------------------
struct gsc_binning {
  Alloc alloc;
  int S = 0;
  int R = 0;                       // requests
  std::vector<Seg> segs;
  std::vector<DevCam> cams;
  std::vector<int64_t> seg_gstart, seg_tstart;
  int64_t G = 0, n_tiles = 0, pixels = 0;
  int n_sort_blocks = 0;
  int64_t bin_waves = 0, count_blocks = 0, chunk_tiles = 0, n_regions = 0;
  // device tables: [Seg x S][DevCam x R][int64 gstart x S][int64 tstart x S][sort table][bin work]
  DevBuf tables;
  size_t off_cams = 0, off_gstart = 0, off_tstart = 0, off_sort = 0, off_work = 0;
  DevBuf rec, depth_key, rect, tiles, ids, keys_tmp, ids_tmp, hist, rect_sorted;
  DevBuf counts, tile_total, partial, tile_start, ranges, scalars, values, n_contrib, grad2d;
  // heaviest-first tile schedules of the splat kernels
  DevBuf ord_val, tile_work;
  // list cut: per-Gaussian saturation cores (with their weights), [chunk][tile] weight sums,
  // per-tile last kept chunk, per-region placement chunk counts and first workgroups
  DevBuf core, core_sorted, wsum, cut, region_start, region_n;
  DevBuf gfix;                     // deterministic adjoint: [9][G] fixed-point sums, [9][G] maxima
  bool list_cut = false;
  uint64_t n_instances = 0;
  uint64_t capacity = 0;
  bool forward_done = false;
  int K = 0;
  int TX = 0, TY = 0;
  int tsx = kTileShift, tsy = kTileShift;   // log2 tile size: 16x16 (gsc_project_bin), 32x32 (frames)
  // views
  DevBuf view_window, view_screen;

  const Seg* d_segs() const { return tables.as<Seg>(); }
  const DevCam* d_cams() const { return (const DevCam*)((char*)tables.p + off_cams); }
  const int64_t* d_gstart() const { return (const int64_t*)((char*)tables.p + off_gstart); }
  const int64_t* d_tstart() const { return (const int64_t*)((char*)tables.p + off_tstart); }
  const void* d_sort() const { return (char*)tables.p + off_sort; }
  const void* d_work() const { return (char*)tables.p + off_work; }
  uint64_t* d_ninst() const { return scalars.as<uint64_t>(); }

  void free_all() {
    DevBuf* all[] = {&tables, &rec, &depth_key, &rect, &tiles, &ids, &keys_tmp, &ids_tmp, &hist,
                     &rect_sorted, &counts, &tile_total, &partial, &tile_start, &ranges, &scalars,
                     &values, &n_contrib, &grad2d, &view_window, &view_screen, &ord_val,
                     &tile_work, &core,
                     &core_sorted, &wsum, &cut, &region_start, &region_n, &gfix};
    for (DevBuf* b : all) b->release(alloc);
  }
};

struct gsc_scene {
  Alloc alloc;
  int K = 0;
  std::vector<int64_t> n;
  std::vector<float*> params;      // per level: [pos 3n][rot 4n][ls 3n][rgb 3n][logit n]
  std::vector<float*> m, v;
  int64_t* d_step = nullptr;       // DEVICE [K]: AdamW steps taken per level (advanced only by
                                   // updates that ran, i.e. with a finite loss)
  float4* cells = nullptr;         // density in the cell-corner layout (32 B per trilinear cell)
  int32_t nx = 0, ny = 0, nz = 0;
  float dmax = 1.0f;
  std::vector<float> tf, lights, spheres;
};

struct gsc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;      // tracer stream (default priority)
  Alloc alloc;
  std::string err;
  bool sticky = false;
  uint64_t required = 0;
  int deterministic = 0;
  int list_cut = 1;                // frames bin only the list prefixes that can reach a pixel
  int frame_binning = 0;           // gsc_project_bin bins like the frames (32x32 tiles, list cut)
  int frame_tiles = 0;             // frames' tile edge in pixels: 16, 32, or 0 (by batch size)
  // pinned staging ring for descriptor uploads
  char* pinned = nullptr;
  size_t pinned_cap = 0, pinned_head = 0;
  hipEvent_t upload_ev = nullptr;
  bool upload_pending = false;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_place = nullptr;   // frames: the placement's instance count has reached the host
  uint64_t frame_capacity = 0;     // frames: instance capacity (0: size the next binning exactly)
  hipEvent_t tev[8] = {};
  // frame workspace
  gsc_binning* frame_bin = nullptr;
  DevBuf targets, records, dL, partials, losses, grads14, images, final_T, last_id, trace_tab,
      vertices, composite_tmp;
  // cache initialisation workspace
  DevBuf ini_tries, ini_key, ini_id, ini_key_tmp, ini_id_tmp, ini_hist, ini_sort_tab, ini_start,
      ini_end, ini_spos, ini_partial, ini_pos, ini_alb, ini_mean3, ini_count;
  uint64_t* host_u64 = nullptr;    // pinned scalars for readback
  // per-kernel event timing (gsc_ctx_profile)
  bool prof_on = false;
  struct ProfRec { int id; hipEvent_t a, b; };
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  double prof_ms[16] = {};
  int64_t prof_n[16] = {};
  uint64_t acc_instances = 0, acc_frames = 0, acc_retries = 0;
  DevBuf adam_tab;                 // fused AdamW group table
  DevBuf d_stats;                  // splat work counters (kStatWords words)
  void* scratch = nullptr;         // this device's address of the allocation-free adjoint's array
  hipError_t scratch_err = hipSuccess;
  bool work_counters = false;      // detailed counting variants of the splat kernels
};

namespace {

#define GSC_TRY(expr)                                                     \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess) throw_hip(ctx, e_, #expr, __LINE__);            \
  } while (0)

[[noreturn]] void throw_hip(gsc_ctx* ctx, hipError_t e, const char* what, int line) {
  char buf[512];
  snprintf(buf, sizeof(buf), "HIP error %d (%s) at runtime.hip:%d: %s", (int)e,
           hipGetErrorString(e), line, what);
  ctx->err = buf;
  ctx->sticky = true;
  throw Fail{GSC_E_DEVICE};
}

[[noreturn]] void invalid(gsc_ctx* ctx, const std::string& msg) {
  ctx->err = msg;
  throw Fail{GSC_E_INVALID_ARG};
}

[[noreturn]] void oom(gsc_ctx* ctx, const char* what, size_t bytes) {
  char buf[256];
  snprintf(buf, sizeof(buf), "allocation of %zu bytes for %s failed", bytes, what);
  ctx->err = buf;
  throw Fail{GSC_E_OUT_OF_MEMORY};
}

void need(gsc_ctx* ctx, DevBuf& b, const Alloc& a, size_t bytes, const char* what) {
  if (!b.ensure(a, bytes)) oom(ctx, what, bytes);
}

#ifdef GSC_DEBUG
// Debug builds: after every call, wait for the device and read (and clear) the flag words of
// the device bounds checks; a failed check fails the call with GSC_E_DEVICE, naming the checks.
void debug_after_call(gsc_ctx* ctx) {
  GSC_TRY(hipDeviceSynchronize());
  const uint32_t f = debug_flags_bin() | debug_flags_splat() | debug_flags_probe();
  if (f == 0u) return;
  std::string msg = "device bounds check failed:";
  if (f == ~0u) msg += " (flag word unreadable)";
  else {
    if (f & kDbgInstanceStore) msg += " instance store past the list capacity;";
    if (f & kDbgPlaceQueue) msg += " placement queue overflow;";
    if (f & kDbgListEntry) msg += " tile-list entry out of range;";
    if (f & kDbgSelfTest) msg += " self-test;";
  }
  ctx->err = msg;
  throw Fail{GSC_E_DEVICE};
}
#endif

template <typename F>
gsc_status guarded(gsc_ctx* ctx, F&& f) {
  if (!ctx) return GSC_E_INVALID_ARG;
  if (ctx->sticky) return GSC_E_DEVICE;
  try {
    ctx->err.clear();
    GSC_TRY(hipSetDevice(ctx->device));
#ifdef GSC_DEBUG
    const gsc_status st = f();
    if (st == GSC_OK) debug_after_call(ctx);
    return st;
#else
    return f();
#endif
  } catch (const Fail& fl) {
    return fl.st;
  } catch (const std::bad_alloc&) {
    ctx->err = "host allocation failed";
    return GSC_E_OUT_OF_MEMORY;
  } catch (...) {
    ctx->err = "unexpected exception";
    return GSC_E_DEVICE;
  }
}

// Copies host bytes to device through the pinned ring, on the context stream.
void upload(gsc_ctx* ctx, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return;
  if (bytes > ctx->pinned_cap) {
    // Rare: very large tables go through a synchronous copy.
    GSC_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream));
    GSC_TRY(hipStreamSynchronize(ctx->stream));
    return;
  }
  size_t off = (ctx->pinned_head + 255) & ~size_t(255);
  if (off + bytes > ctx->pinned_cap) {
    if (ctx->upload_pending) GSC_TRY(hipEventSynchronize(ctx->upload_ev));
    off = 0;
  }
  std::memcpy(ctx->pinned + off, src, bytes);
  GSC_TRY(hipMemcpyAsync(dst, ctx->pinned + off, bytes, hipMemcpyHostToDevice, ctx->stream));
  GSC_TRY(hipEventRecord(ctx->upload_ev, ctx->stream));
  ctx->upload_pending = true;
  ctx->pinned_head = off + bytes;
}

uint64_t read_u64(gsc_ctx* ctx, const uint64_t* dev) {
  GSC_TRY(hipMemcpyAsync(ctx->host_u64, dev, sizeof(uint64_t), hipMemcpyDeviceToHost, ctx->stream));
  GSC_TRY(hipStreamSynchronize(ctx->stream));
  return ctx->host_u64[0];
}

// Two consecutive device words in one synchronising read.
void read_u64x2(gsc_ctx* ctx, const uint64_t* dev, uint64_t* a, uint64_t* b) {
  GSC_TRY(hipMemcpyAsync(ctx->host_u64 + 2, dev, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost,
                         ctx->stream));
  GSC_TRY(hipStreamSynchronize(ctx->stream));
  *a = ctx->host_u64[2];
  *b = ctx->host_u64[3];
}

const char* const kProfNames[] = {"project", "depth_sort", "bin_count", "bin_scan", "bin_place",
                                  "splat_forward", "trace", "loss_composite", "splat_backward",
                                  "project_backward", "adam", "gather_rect",
                                  "project_backward_adam"};
constexpr int kProfCount = 13;
constexpr int kStatWords = 12;  // splat work counters (gsc_counters; see k_splat.hip)
enum { P_PROJECT, P_SORT, P_COUNT, P_SCAN, P_PLACE, P_FWD, P_TRACE, P_LOSS, P_BWD, P_PBWD, P_ADAM,
       P_GATHER, P_PBADAM };

hipEvent_t pool_event(gsc_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  GSC_TRY(hipEventCreate(&e));
  return e;
}

// Records HIP events around one launch on its own stream when profiling is on.
struct ProfScope {
  gsc_ctx* ctx;
  hipStream_t st;
  int id;
  hipEvent_t a = nullptr;
  ProfScope(gsc_ctx* c, int i, hipStream_t s) : ctx(c), st(s), id(i) {
    if (ctx->prof_on) {
      a = pool_event(ctx);
      GSC_TRY(hipEventRecord(a, st));
    }
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = nullptr;
    if (!ctx->ev_pool.empty()) { b = ctx->ev_pool.back(); ctx->ev_pool.pop_back(); }
    else if (hipEventCreate(&b) != hipSuccess) b = nullptr;
    if (b && hipEventRecord(b, st) == hipSuccess) ctx->prof_pending.push_back({id, a, b});
    else { ctx->ev_pool.push_back(a); if (b) ctx->ev_pool.push_back(b); }
  }
};

void prof_resolve(gsc_ctx* ctx) {
  for (auto& p : ctx->prof_pending) {
    GSC_TRY(hipEventSynchronize(p.b));
    float ms = 0.0f;
    GSC_TRY(hipEventElapsedTime(&ms, p.a, p.b));
    ctx->prof_ms[p.id] += (double)ms;
    ctx->prof_n[p.id] += 1;
    ctx->ev_pool.push_back(p.a);
    ctx->ev_pool.push_back(p.b);
  }
  ctx->prof_pending.clear();
}

DevCam to_dev(const gsc_camera& c) {
  DevCam d;
  std::memcpy(d.R, c.R, sizeof(d.R));
  std::memcpy(d.t, c.t, sizeof(d.t));
  d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
  d.full_w = c.full_w; d.full_h = c.full_h;
  d.x0 = c.x0; d.y0 = c.y0; d.w = c.w; d.h = c.h;
  d.znear = c.znear;
  return d;
}

void check_camera(gsc_ctx* ctx, const gsc_camera* c) {
  if (!c) invalid(ctx, "camera is NULL");
  if (c->w < 1 || c->h < 1 || c->w > 16384 || c->h > 16384) invalid(ctx, "camera window size out of range");
  if (c->full_w < 1 || c->full_h < 1 || c->full_w > 65535 || c->full_h > 65535) invalid(ctx, "full frame size out of range");
  if (c->x0 < 0 || c->y0 < 0 || c->x0 + c->w > c->full_w || c->y0 + c->h > c->full_h)
    invalid(ctx, "camera window outside the full frame");
  if (!(c->fx > 0.0f) || !(c->fy > 0.0f) || !std::isfinite(c->cx) || !std::isfinite(c->cy))
    invalid(ctx, "camera intrinsics invalid");
  for (float r : c->R) if (!std::isfinite(r)) invalid(ctx, "camera rotation not finite");
  for (float t : c->t) if (!std::isfinite(t)) invalid(ctx, "camera translation not finite");
  if (!(c->znear > 0.0f)) invalid(ctx, "znear must be positive");
}

void check_levels(gsc_ctx* ctx, const gsc_gaussians* lv, int K) {
  if (K < 1 || K > 8) invalid(ctx, "num_levels must be in [1, 8]");
  if (!lv) invalid(ctx, "levels is NULL");
  for (int l = 0; l < K; ++l) {
    if (lv[l].n < 0 || lv[l].n >= (int64_t(1) << 31)) invalid(ctx, "level size out of range");
    if (lv[l].n > 0 && (!lv[l].pos || !lv[l].rot || !lv[l].log_scale || !lv[l].rgb || !lv[l].opacity_logit))
      invalid(ctx, "level parameter pointer is NULL");
  }
}

// One request of a batch: a camera and K levels.
struct ReqSpec {
  gsc_camera cam;
  std::vector<gsc_gaussians> levels;
};

// Builds (or rebuilds) a binning object's tables for a list of requests and uploads them.
void plan_batch(gsc_ctx* ctx, gsc_binning* b, const std::vector<ReqSpec>& reqs, int tsx, int tsy) {
  b->tsx = tsx;
  b->tsy = tsy;
  const int tw = 1 << tsx, th = 1 << tsy;  // tiles are tw x th pixels
  b->segs.clear();
  b->cams.clear();
  b->seg_gstart.clear();
  b->seg_tstart.clear();
  int64_t g = 0, tiles = 0, pix = 0;
  for (size_t r = 0; r < reqs.size(); ++r) {
    const gsc_camera& c = reqs[r].cam;
    b->cams.push_back(to_dev(c));
    const int TX = (c.w + tw - 1) / tw, TY = (c.h + th - 1) / th;
    for (size_t l = 0; l < reqs[r].levels.size(); ++l) {
      const gsc_gaussians& lv = reqs[r].levels[l];
      Seg s{};
      s.pos = lv.pos; s.rot = lv.rot; s.ls = lv.log_scale; s.rgb = lv.rgb; s.logit = lv.opacity_logit;
      s.n = lv.n;
      s.g_off = g;
      s.tile_base = tiles;
      s.pix_off = pix;
      s.cam = (int32_t)r;
      s.TX = TX; s.TY = TY;
      s.level = (int32_t)l;
      s.request = (int32_t)r;
      s.tsx = tsx;
      s.tsy = tsy;
      s.n_chunks = (int32_t)((lv.n + kChunk - 1) / kChunk);
      b->segs.push_back(s);
      b->seg_gstart.push_back(g);
      b->seg_tstart.push_back(tiles);
      g += lv.n;
      tiles += (int64_t)TX * TY;
      pix += (int64_t)c.w * c.h;
    }
  }
  b->S = (int)b->segs.size();
  b->R = (int)reqs.size();
  b->G = g;
  b->n_tiles = tiles;
  b->pixels = pix;
  std::vector<int64_t> seg_n(b->S), seg_off(b->S);
  for (int s = 0; s < b->S; ++s) { seg_n[s] = b->segs[s].n; seg_off[s] = b->segs[s].g_off; }
  b->n_sort_blocks = sort_count_blocks(seg_n.data(), b->S);
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  size_t off = al(sizeof(Seg) * b->S);
  b->off_cams = off;
  off = al(off + sizeof(DevCam) * b->R);
  b->off_gstart = off;
  off = al(off + sizeof(int64_t) * b->S);
  b->off_tstart = off;
  off = al(off + sizeof(int64_t) * b->S);
  b->off_sort = off;
  off = al(off + sort_table_bytes(b->n_sort_blocks, b->S));
  b->off_work = off;
  off = al(off + bin_work_bytes(b->S));
  std::vector<char> host(off, 0);
  std::memcpy(host.data(), b->segs.data(), sizeof(Seg) * b->S);
  std::memcpy(host.data() + b->off_cams, b->cams.data(), sizeof(DevCam) * b->R);
  std::memcpy(host.data() + b->off_gstart, b->seg_gstart.data(), sizeof(int64_t) * b->S);
  std::memcpy(host.data() + b->off_tstart, b->seg_tstart.data(), sizeof(int64_t) * b->S);
  sort_fill_table(host.data() + b->off_sort, seg_n.data(), seg_off.data(), b->S);
  b->bin_waves = bin_fill_work(host.data() + b->off_work, b->segs.data(), b->S, &b->chunk_tiles,
                                &b->count_blocks, &b->n_regions);
  need(ctx, b->tables, b->alloc, off, "descriptor tables");
  upload(ctx, b->tables.p, host.data(), off);
  b->forward_done = false;
}

// Projection, depth sort and binning of a planned batch.  capacity_hint 0: exact sizing with one
// read-back of the instance count.
// after_count, if set, is called once the per-(chunk, tile) counts are enqueued.  Frames start
// the tracer there: it then overlaps the scans, the placement and the forward splat, and stays
// off the LDS-heavy sort and count kernels.
constexpr int kHostDeferredCount = 16;   // slot of ctx->host_u64 for a frame's instance count

gsc_status run_project_bin(gsc_ctx* ctx, gsc_binning* b, uint64_t capacity_hint,
                           const std::function<void()>& after_count = {}, bool deferred = false) {
  const Alloc& a = b->alloc;
  const int64_t G = b->G;
  const int64_t Gp = std::max<int64_t>(G, 1);
  need(ctx, b->rec, a, sizeof(SplatRec) * Gp, "projected records");
  need(ctx, b->depth_key, a, 4 * Gp, "depth keys");
  need(ctx, b->rect, a, 8 * Gp, "tile rects");
  need(ctx, b->tiles, a, 4 * Gp, "tiles touched");
  need(ctx, b->ids, a, 4 * Gp, "ids");
  need(ctx, b->keys_tmp, a, 4 * Gp, "sort keys");
  need(ctx, b->ids_tmp, a, 4 * Gp, "sort values");
  need(ctx, b->hist, a, 4 * sort_hist_words(std::max(b->n_sort_blocks, 1), b->S), "sort histograms");
  need(ctx, b->rect_sorted, a, 8 * Gp, "sorted rects");
  need(ctx, b->counts, a, 4 * (size_t)std::max<int64_t>(b->chunk_tiles, 1), "chunk counts");
  need(ctx, b->tile_total, a, 4 * (size_t)std::max<int64_t>(b->n_tiles, 1), "tile totals");
  need(ctx, b->partial, a, 8 * bin_scan_partials(b->n_tiles), "scan partials");
  need(ctx, b->tile_start, a, 8 * (size_t)std::max<int64_t>(b->n_tiles, 1), "tile starts");
  need(ctx, b->ranges, a, 16 * (size_t)std::max<int64_t>(b->n_tiles, 1), "tile ranges");
  need(ctx, b->scalars, a, 64, "scalars");
  const bool lc = b->list_cut;
  if (lc) {
    need(ctx, b->core, a, 8 * Gp, "saturation cores");
    need(ctx, b->core_sorted, a, 8 * Gp, "sorted saturation cores");
    need(ctx, b->wsum, a, 4 * (size_t)std::max<int64_t>(b->chunk_tiles, 1), "chunk weight sums");
  }
  need(ctx, b->cut, a, 4 * (size_t)std::max<int64_t>(b->n_tiles, 1), "tile cuts");
  need(ctx, b->region_start, a, 8 * (size_t)std::max<int64_t>(b->n_regions, 1), "region starts");
  need(ctx, b->region_n, a, 4 * (size_t)std::max<int64_t>(b->n_regions, 1), "region chunk counts");
  uint64_t* core = lc ? b->core.as<uint64_t>() : nullptr;
  uint64_t* core_sorted = lc ? b->core_sorted.as<uint64_t>() : nullptr;
  uint32_t* wsum = lc ? b->wsum.as<uint32_t>() : nullptr;
  int32_t* cut = b->cut.as<int32_t>();
  hipStream_t st = ctx->stream;
  GSC_TRY(hipMemsetAsync(b->scalars.p, 0, 64, st));
  GSC_TRY(hipMemsetAsync(b->region_n.p, 0, 4 * (size_t)b->n_regions, st));
  { ProfScope ps_(ctx, P_PROJECT, st);
  GSC_TRY(launch_project(st, b->d_segs(), b->d_gstart(), b->S, b->d_cams(), G, b->rec.as<SplatRec>(),
                         b->depth_key.as<uint32_t>(), b->rect.as<uint64_t>(), b->tiles.as<uint32_t>(),
                         b->ids.as<uint32_t>(), core));
  }
  // The sort consumes a copy of the depth keys (the originals serve the key view); the odd
  // passes of the sort use rect_sorted as key scratch before the gather fills it.
  GSC_TRY(hipMemcpyAsync(b->keys_tmp.p, b->depth_key.p, 4 * G, hipMemcpyDeviceToDevice, st));
  { ProfScope ps_(ctx, P_SORT, st);
  GSC_TRY(launch_segmented_sort(st, b->d_sort(), b->n_sort_blocks, b->S, b->keys_tmp.as<uint32_t>(),
                                b->ids.as<uint32_t>(), b->rect_sorted.as<uint32_t>(),
                                b->ids_tmp.as<uint32_t>(), b->hist.as<uint32_t>()));
  }
  { ProfScope ps_(ctx, P_GATHER, st);
  GSC_TRY(launch_gather_rect(st, b->d_gstart(), b->S, G, b->ids.as<uint32_t>(), b->rect.as<uint64_t>(),
                             b->rect_sorted.as<uint64_t>(), core, core_sorted));
  }
  { ProfScope ps_(ctx, P_COUNT, st);
  GSC_TRY(launch_bin_count(st, b->d_work(), b->S, b->count_blocks, b->rect_sorted.as<uint64_t>(),
                           b->counts.as<uint32_t>(), core_sorted, wsum));
  }
  if (after_count) after_count();
  { ProfScope ps_(ctx, P_SCAN, st);
  GSC_TRY(launch_bin_scan(st, b->d_work(), b->S, b->d_tstart(), b->n_tiles, b->counts.as<uint32_t>(),
                          b->tile_total.as<uint32_t>(), b->partial.as<uint64_t>(),
                          b->tile_start.as<uint64_t>(), b->ranges.as<uint64_t>(), b->d_ninst(),
                          wsum, cut, b->region_n.as<int32_t>()));
  GSC_TRY(launch_bin_regions(st, b->n_regions, b->region_n.as<int32_t>(), b->region_start.as<uint64_t>(),
                             b->d_ninst() + 1));
  }
  uint64_t cap = capacity_hint;
  uint64_t n_inst = 0;
  // Placement workgroups: the exact count when the sizes are read back anyway, else the bound
  // of every region visiting every chunk (the surplus workgroups exit at once).
  uint64_t place_blocks = (uint64_t)b->bin_waves;
  if (cap == 0) {
    read_u64x2(ctx, b->d_ninst(), &n_inst, &place_blocks);
    cap = n_inst;
  }
  need(ctx, b->values, a, 4 * (size_t)std::max<uint64_t>(cap, 1), "instance values");
  b->capacity = cap;
  { ProfScope ps_(ctx, P_PLACE, st);
  GSC_TRY(launch_bin_place(st, b->d_work(), b->S, b->n_regions, b->region_start.as<uint64_t>(),
                           b->d_ninst() + 1, (int64_t)place_blocks, b->ids.as<uint32_t>(),
                           b->rect_sorted.as<uint64_t>(), b->counts.as<uint32_t>(),
                           b->tile_start.as<uint64_t>(), b->d_ninst(), cap, b->values.as<uint32_t>(),
                           cut));
  }
  if (deferred && capacity_hint != 0) {
    // Frames: the count reaches the host while the rest of the frame is enqueued; the splat
    // kernels and the AdamW step skip a binning that overflowed, and the frame call checks the
    // count once everything is enqueued (render_batch).
    GSC_TRY(hipMemcpyAsync(ctx->host_u64 + kHostDeferredCount, b->d_ninst(), 8,
                           hipMemcpyDeviceToHost, st));
    GSC_TRY(hipEventRecord(ctx->ev_place, st));
    b->n_instances = 0;
    return GSC_OK;
  }
  if (capacity_hint != 0) n_inst = read_u64(ctx, b->d_ninst());
  b->n_instances = n_inst;
  ctx->acc_instances += n_inst;
  ctx->acc_frames += 1;
  if (n_inst > cap) {
    ctx->required = n_inst;
    char buf[160];
    snprintf(buf, sizeof(buf), "instance capacity %llu exceeded: %llu needed",
             (unsigned long long)cap, (unsigned long long)n_inst);
    ctx->err = buf;
    return GSC_E_CAPACITY;
  }
  return GSC_OK;
}

// Heaviest-first tile schedule for a splat launch: tiles in decreasing buckets of a work estimate
// (work NULL: list length).  Single-wave workgroups start in that order, so the long tiles do not
// end up in the launch's tail.
const uint32_t* tile_order(gsc_ctx* ctx, gsc_binning* b, const uint32_t* work) {
  need(ctx, b->ord_val, b->alloc, 4 * (size_t)std::max<int64_t>(b->n_tiles, 1), "tile order");
  GSC_TRY(launch_tile_order(ctx->stream, b->ranges.as<uint64_t>(), work, b->n_tiles,
                            b->ord_val.as<uint32_t>()));
  return b->ord_val.as<uint32_t>();
}

void run_forward(gsc_ctx* ctx, gsc_binning* b, float* images, float* final_T, int32_t* last_id) {
  need(ctx, b->n_contrib, b->alloc, 4 * (size_t)std::max<int64_t>(b->pixels, 1), "n_contrib");
  need(ctx, b->tile_work, b->alloc, 4 * (size_t)std::max<int64_t>(b->n_tiles, 1), "tile work");
  if (!ctx->d_stats.p) {
    need(ctx, ctx->d_stats, ctx->alloc, kStatWords * 8, "splat counters");
    GSC_TRY(hipMemsetAsync(ctx->d_stats.p, 0, kStatWords * 8, ctx->stream));
  }
  const uint32_t* order = tile_order(ctx, b, nullptr);
  if (b->tsx != kTileShift || b->tsy != kTileShift)   // larger tiles: the forward sums its blocks' work
    GSC_TRY(launch_fill_u32(ctx->stream, b->tile_work.as<uint32_t>(), 0u, b->n_tiles));
  { ProfScope ps_(ctx, P_FWD, ctx->stream);
  GSC_TRY(launch_splat_forward(ctx->stream, b->d_segs(), b->d_tstart(), b->S, b->d_cams(), b->n_tiles,
                               b->ranges.as<uint64_t>(), b->values.as<uint32_t>(),
                               b->rec.as<SplatRec>(), images, final_T, last_id,
                               b->n_contrib.as<uint32_t>(), ctx->d_stats.as<unsigned long long>(),
                               order, b->tile_work.as<uint32_t>(), ctx->work_counters, b->tsx, b->tsy,
                               b->d_ninst(), b->capacity));
  }
  b->forward_done = true;
}

// The splat adjoint into b->grad2d ([G][kGrad2dStride] screen-space gradients).
void run_splat_adjoint(gsc_ctx* ctx, gsc_binning* b, const float* final_T, const float* dL) {
  need(ctx, b->grad2d, b->alloc, 4 * kGrad2dStride * (size_t)std::max<int64_t>(b->G, 1),
       "2D gradients");
  uint32_t* gmax = nullptr;
  unsigned long long* gfix = nullptr;
  if (ctx->deterministic) {
    need(ctx, b->gfix, b->alloc, 12 * 9 * (size_t)std::max<int64_t>(b->G, 1), "fixed-point gradients");
    GSC_TRY(hipMemsetAsync(b->gfix.p, 0, 12 * 9 * (size_t)b->G, ctx->stream));
    gfix = b->gfix.as<unsigned long long>();
    gmax = (uint32_t*)(gfix + 9 * (size_t)b->G);
  } else {
    GSC_TRY(hipMemsetAsync(b->grad2d.p, 0, 4 * kGrad2dStride * (size_t)b->G, ctx->stream));
  }
  const uint32_t* order = tile_order(ctx, b, b->tile_work.as<uint32_t>());
  if (ctx->work_counters && !ctx->d_stats.p) {
    need(ctx, ctx->d_stats, ctx->alloc, kStatWords * 8, "splat counters");
    GSC_TRY(hipMemsetAsync(ctx->d_stats.p, 0, kStatWords * 8, ctx->stream));
  }
  { ProfScope ps_(ctx, P_BWD, ctx->stream);
  GSC_TRY(launch_splat_backward(ctx->stream, b->d_segs(), b->d_tstart(), b->S, b->d_cams(), b->n_tiles,
                                b->ranges.as<uint64_t>(), b->values.as<uint32_t>(),
                                b->rec.as<SplatRec>(), final_T, b->n_contrib.as<uint32_t>(), dL,
                                b->grad2d.as<float>(), b->G, order, gmax, gfix,
                                ctx->d_stats.as<unsigned long long>(), ctx->work_counters,
                                b->tsx, b->tsy, b->d_ninst(), b->capacity));
  }
}

// The splat adjoint and the chain rule to the 14 parameter gradients per Gaussian.
void run_backward(gsc_ctx* ctx, gsc_binning* b, const float* final_T, const float* dL,
                  float* grads14) {
  run_splat_adjoint(ctx, b, final_T, dL);
  { ProfScope ps_(ctx, P_PBWD, ctx->stream);
  GSC_TRY(launch_project_backward(ctx->stream, b->d_segs(), b->d_gstart(), b->S, b->d_cams(), b->G,
                                  b->grad2d.as<float>(), grads14));
  }
}


float max_alpha(const float* tf, int P) {
  float m = 0.0f;
  for (int i = 0; i < P; ++i) m = std::fmax(m, tf[4 * i + 3]);
  return m;
}

void check_volume_host(gsc_ctx* ctx, const float* tf, int P, const float* lights, int nl,
                       const float* spheres, int ns) {
  if (P < 2 || P > kMaxTf) invalid(ctx, "tf_points must be in [2, 64]");
  if (nl < 0 || nl > kMaxLights) invalid(ctx, "n_lights must be in [0, 8]");
  if (ns < 0 || ns > kMaxLights) invalid(ctx, "n_spheres must be in [0, 8]");
  if (nl + ns < 1) invalid(ctx, "the scene needs at least one light");
  if (!tf) invalid(ctx, "tf_rgba is NULL");
  if (nl > 0 && !lights) invalid(ctx, "lights is NULL");
  if (ns > 0 && !spheres) invalid(ctx, "spheres is NULL");
  for (int i = 0; i < 4 * P; ++i) if (!std::isfinite(tf[i])) invalid(ctx, "transfer function not finite");
  if (!(max_alpha(tf, P) > 0.0f)) invalid(ctx, "transfer function opacity is zero everywhere (no majorant)");
  for (int i = 0; i < 6 * nl; ++i) if (!std::isfinite(lights[i])) invalid(ctx, "lights not finite");
  for (int s = 0; s < ns; ++s) {
    const float* sp = spheres + 7 * s;
    for (int i = 0; i < 7; ++i) if (!std::isfinite(sp[i])) invalid(ctx, "spheres not finite");
    if (!(sp[3] > 0.0f)) invalid(ctx, "sphere light radius must be positive");
    // Squared distance from the centre to the unit cube must exceed r^2.
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double c = sp[a], q = std::min(std::max(c, 0.0), 1.0);
      d2 += (c - q) * (c - q);
    }
    if (!(d2 > (double)sp[3] * sp[3])) invalid(ctx, "sphere lights must lie outside the unit cube");
  }
}

TraceDesc make_trace_desc(const float* density, const float4* cells, int nx, int ny, int nz, float dmax,
                          const float* tf,
                          int P, const float* lights, int nl, const float* spheres, int ns,
                          const gsc_camera& cam, const gsc_trace_params& tp) {
  TraceDesc d;
  std::memset(&d, 0, sizeof(d));
  d.density = density;
  d.cells = cells;
  d.nx = nx; d.ny = ny; d.nz = nz;
  d.dmax = dmax;
  d.majorant = dmax * max_alpha(tf, P);
  d.P = P;
  d.n_lights = nl;
  d.n_spheres = ns;
  d.strategy = tp.strategy;
  std::memcpy(d.tf, tf, sizeof(float) * 4 * P);
  if (nl > 0) std::memcpy(d.lights, lights, sizeof(float) * 6 * nl);
  if (ns > 0) std::memcpy(d.spheres, spheres, sizeof(float) * 7 * ns);
  d.cam = to_dev(cam);
  d.seed = tp.seed;
  d.frame = tp.frame;
  d.spp = tp.spp;
  d.max_bounces = tp.max_bounces;
  d.K = tp.num_levels;
  d.C = tp.C;
  d.C_inf = tp.C_inf;
  d.eps = tp.eps;
  return d;
}

void check_trace_params(gsc_ctx* ctx, const gsc_trace_params* tp) {
  if (!tp) invalid(ctx, "trace params NULL");
  if (tp->spp < 1) invalid(ctx, "spp must be >= 1");
  if (tp->max_bounces < 1) invalid(ctx, "max_bounces must be >= 1");
  if (tp->num_levels < 1 || tp->num_levels > 8) invalid(ctx, "num_levels must be in [1, 8]");
  if (!tp->C_inf && !std::isfinite(tp->C)) invalid(ctx, "C must be finite unless C_inf is set");
  if (!std::isfinite(tp->eps) || tp->eps < 0.0f) invalid(ctx, "eps must be finite and >= 0");
  if (tp->strategy != GSC_STRATEGY_NEE && tp->strategy != GSC_STRATEGY_UNIFORM)
    invalid(ctx, "strategy must be GSC_STRATEGY_NEE or GSC_STRATEGY_UNIFORM");
}

// AdamW hyper-parameters of one group at `step`: bias corrections s1 = lr / (1 - b1^t) and
// s2 = 1 / sqrt(1 - b2^t) and the decoupled decay factor 1 - lr wd, in double, then rounded.
AdamGroup adam_params(float* p, float* m, float* v, const float* g, int64_t count, double lr,
                      double b1, double b2, double eps, double wd, int64_t step, const float* guard) {
  AdamGroup a;
  a.p = p; a.m = m; a.v = v; a.g = g; a.n = count; a.guard = guard;
  a.b1 = (float)b1; a.b2 = (float)b2;
  a.omb1 = (float)(1.0 - b1); a.omb2 = (float)(1.0 - b2);
  a.s1 = (float)(lr / (1.0 - std::pow(b1, (double)step)));
  a.s2 = (float)(1.0 / std::sqrt(1.0 - std::pow(b2, (double)step)));
  a.wdf = (float)(1.0 - lr * wd);
  a.eps = (float)eps;
  a.step = nullptr;
  a.lr = lr; a.b1d = b1; a.b2d = b2;
  return a;
}

void adam_group(gsc_ctx* ctx, float* p, float* m, float* v, const float* g, int64_t count, double lr,
                double b1, double b2, double eps, double wd, int64_t step, const float* guard) {
  const AdamGroup a = adam_params(p, m, v, g, count, lr, b1, b2, eps, wd, step, guard);
  { ProfScope ps_(ctx, P_ADAM, ctx->stream);
  GSC_TRY(launch_adam(ctx->stream, p, m, v, g, count, a.b1, a.b2, a.omb1, a.omb2, a.s1, a.s2,
                      a.wdf, a.eps, guard));
  }
}

double elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
  return (double)ms;
}

// The frame pipeline over a batch of (distinct) scenes.
// *retry is set when the frame's binning overflowed the capacity sized from the previous frame:
// nothing persistent was written, and the caller runs the frame again.
// The frames' tile edge (as a shift): the setting, or by the requests' sizes.  32x32 tiles
// bin fewer instances than 16x16 ones (a third at 1080p), but the splat kernels walk each list
// with two or four wavefronts instead of one per 16x16 tile, so a frame's heaviest tile takes
// longer; only a request with at least kAutoTiles32 of them over its levels has the parallel
// work to hide that.  Every request of the batch must have it.
int frame_tile_shift(const gsc_ctx* ctx, gsc_scene* const* scenes, const gsc_frame_request* reqs,
                     int n) {
  if (ctx->frame_tiles == 16) return kTileShift;
  if (ctx->frame_tiles == 32) return kFrameTileShiftX;
  for (int i = 0; i < n; ++i) {
    const int64_t tiles = (int64_t)scenes[i]->K * ((reqs[i].cam.w + 31) / 32) * ((reqs[i].cam.h + 31) / 32);
    if (tiles < kAutoTiles32) return kTileShift;
  }
  return kFrameTileShiftX;
}

gsc_status render_batch(gsc_ctx* ctx, gsc_scene* const* scenes, const gsc_frame_request* reqs,
                        float* const* images, int n, gsc_frame_stats* stats, bool* retry) {
  *retry = false;
  if (n < 1) invalid(ctx, "batch is empty");
  if (!scenes || !reqs || !images) invalid(ctx, "NULL argument");
  for (int i = 0; i < n; ++i) {
    if (!scenes[i]) invalid(ctx, "scene is NULL");
    if (!images[i]) invalid(ctx, "image is NULL");
    for (int j = 0; j < i; ++j) if (scenes[j] == scenes[i]) invalid(ctx, "scenes of a batch must be distinct");
    check_camera(ctx, &reqs[i].cam);
    check_trace_params(ctx, &reqs[i].trace);
    if ((int)reqs[i].trace.num_levels != scenes[i]->K) invalid(ctx, "trace.num_levels must equal the scene's K");
    if (reqs[i].trace.spp > 4096) invalid(ctx, "frames trace at most 4096 samples per pixel");
    if (reqs[i].loss != 0 && reqs[i].loss != 1) invalid(ctx, "loss must be 0 (L2) or 1 (HDR)");
    if (reqs[i].viewport_frames < 1) invalid(ctx, "viewport_frames must be >= 1");
  }
  hipStream_t st = ctx->stream;
  const bool timing = stats != nullptr;
  if (timing) GSC_TRY(hipEventRecord(ctx->tev[0], st));
  // ---- plan -----------------------------------------------------------------------------------
  if (!ctx->frame_bin) {
    ctx->frame_bin = new gsc_binning();
    ctx->frame_bin->alloc = ctx->alloc;
  }
  gsc_binning* b = ctx->frame_bin;
  std::vector<ReqSpec> specs(n);
  std::vector<int64_t> pix_base(n), rec_base(n);
  int64_t pix = 0, rpix = 0;
  for (int i = 0; i < n; ++i) {
    specs[i].cam = reqs[i].cam;
    gsc_scene* sc = scenes[i];
    for (int l = 0; l < sc->K; ++l) {
      gsc_gaussians lv;
      float* p = sc->params[l];
      const int64_t nn = sc->n[l];
      lv.pos = p; lv.rot = p + 3 * nn; lv.log_scale = p + 7 * nn; lv.rgb = p + 10 * nn;
      lv.opacity_logit = p + 13 * nn; lv.n = nn;
      specs[i].levels.push_back(lv);
    }
    pix_base[i] = pix;
    rec_base[i] = rpix;
    pix += (int64_t)sc->K * reqs[i].cam.w * reqs[i].cam.h;
    rpix += (int64_t)reqs[i].trace.spp * reqs[i].cam.w * reqs[i].cam.h;
  }
  const int fshift = frame_tile_shift(ctx, scenes, reqs, n);
  plan_batch(ctx, b, specs, fshift, fshift);
  const Alloc& a = ctx->alloc;
  need(ctx, ctx->images, a, 12 * (size_t)pix, "cache images");
  need(ctx, ctx->targets, a, 12 * (size_t)pix, "targets");
  need(ctx, ctx->dL, a, 12 * (size_t)pix, "dL/dimages");
  need(ctx, ctx->final_T, a, 4 * (size_t)pix, "final T");
  need(ctx, ctx->last_id, a, 4 * (size_t)pix, "last id");
  need(ctx, ctx->records, a, sizeof(gsc_path_record) * (size_t)rpix, "records");
  int max_partials = 1;
  for (int i = 0; i < n; ++i) max_partials = std::max(max_partials, loss_num_partials((int64_t)reqs[i].cam.w * reqs[i].cam.h));
  need(ctx, ctx->partials, a, 8 * (size_t)max_partials * n, "loss partials");
  need(ctx, ctx->losses, a, 4 * (size_t)n, "losses");
  need(ctx, ctx->vertices, a, 8, "vertex counter");
  // ---- trace on the side stream (independent of the cache) --------------------------------------
  std::vector<TraceDesc> td(n);
  std::vector<int64_t> tstart(n);
  int64_t tlaunch = 0;
  for (int i = 0; i < n; ++i) {
    gsc_scene* sc = scenes[i];
    td[i] = make_trace_desc(nullptr, sc->cells, sc->nx, sc->ny, sc->nz, sc->dmax, sc->tf.data(),
                            (int)sc->tf.size() / 4, sc->lights.data(), (int)sc->lights.size() / 6,
                            sc->spheres.data(), (int)sc->spheres.size() / 7, reqs[i].cam,
                            reqs[i].trace);
    td[i].pix_off = tlaunch;
    td[i].targets = ctx->targets.as<float>() + 3 * pix_base[i];
    td[i].records = (char*)ctx->records.p + sizeof(gsc_path_record) * rec_base[i];
    tstart[i] = tlaunch;
    tlaunch += trace_align((int64_t)reqs[i].cam.w * reqs[i].cam.h);
  }
  const size_t tbytes = sizeof(TraceDesc) * n + sizeof(int64_t) * n;
  need(ctx, ctx->trace_tab, a, tbytes, "trace descriptors");
  std::vector<char> th(tbytes);
  std::memcpy(th.data(), td.data(), sizeof(TraceDesc) * n);
  std::memcpy(th.data() + sizeof(TraceDesc) * n, tstart.data(), sizeof(int64_t) * n);
  upload(ctx, ctx->trace_tab.p, th.data(), tbytes);
  // The trace is independent of the cache; it runs on the side stream from the end of the
  // binning counts, overlapping the scans, the placement and the forward splat (measured faster
  // than starting it with the frame, after the depth sort, before the placement or after the
  // binning: 93.4 against 91.5, 91.0, 92.2 and 91.5 frames/s at 1080p).
  bool traced = false;
  auto start_trace = [&]() {
    GSC_TRY(hipMemsetAsync(ctx->vertices.p, 0, 8, st));
    GSC_TRY(hipEventRecord(ctx->ev_fork, st));
    GSC_TRY(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
    if (timing) GSC_TRY(hipEventRecord(ctx->tev[6], ctx->side));
    { ProfScope ps_(ctx, P_TRACE, ctx->side);
    GSC_TRY(launch_trace(ctx->side, ctx->trace_tab.as<TraceDesc>(),
                         (const int64_t*)((char*)ctx->trace_tab.p + sizeof(TraceDesc) * n), n, tlaunch,
                         ctx->vertices.as<unsigned long long>()));
    }
    if (timing) GSC_TRY(hipEventRecord(ctx->tev[7], ctx->side));
    GSC_TRY(hipEventRecord(ctx->ev_join, ctx->side));
    traced = true;
  };
  // ---- splat the cache images ---------------------------------------------------------------------
  b->list_cut = ctx->list_cut != 0;
  // Sized from the previous frame's count (no host round trip inside the frame); the first
  // frame of a context is sized exactly.
  const bool deferred = ctx->frame_capacity != 0;
  gsc_status s = run_project_bin(ctx, b, ctx->frame_capacity, start_trace, true);
  if (s != GSC_OK) {
    if (traced) GSC_TRY(hipStreamWaitEvent(st, ctx->ev_join, 0));
    return s;
  }
  if (!traced) start_trace();
  if (timing) GSC_TRY(hipEventRecord(ctx->tev[1], st));
  run_forward(ctx, b, ctx->images.as<float>(), ctx->final_T.as<float>(), ctx->last_id.as<int32_t>());
  if (timing) GSC_TRY(hipEventRecord(ctx->tev[2], st));
  GSC_TRY(hipStreamWaitEvent(st, ctx->ev_join, 0));
  // ---- loss, composite ----------------------------------------------------------------------------
  for (int i = 0; i < n; ++i) {
    const int w = reqs[i].cam.w, h = reqs[i].cam.h;
  { ProfScope ps_(ctx, P_LOSS, st);
  GSC_TRY(launch_loss_composite(st, ctx->images.as<float>() + 3 * pix_base[i],
                                  ctx->targets.as<float>() + 3 * pix_base[i],
                                  (char*)ctx->records.p + sizeof(gsc_path_record) * rec_base[i],
                                  (int)reqs[i].trace.spp, scenes[i]->K, w, h, reqs[i].loss,
                                  ctx->dL.as<float>() + 3 * pix_base[i],
                                  ctx->partials.as<double>() + (size_t)max_partials * i,
                                  ctx->losses.as<float>() + i, images[i]));
  }
  }
  // A binning that overflowed its capacity skips the splats; its frame takes no AdamW step.
  if (deferred) GSC_TRY(launch_capacity_guard(st, b->d_ninst(), b->capacity, ctx->losses.as<float>(), n));
  if (timing) GSC_TRY(hipEventRecord(ctx->tev[3], st));
  // ---- backward + AdamW ---------------------------------------------------------------------------
  bool any_train = false;
  for (int i = 0; i < n; ++i) any_train = any_train || reqs[i].train;
  if (any_train) {
    run_splat_adjoint(ctx, b, ctx->final_T.as<float>(), ctx->dL.as<float>());
    if (timing) GSC_TRY(hipEventRecord(ctx->tev[4], st));
    // One launch over every Gaussian of the batch: chain rule, then AdamW on its 14 parameters
    // with the group's learning rate (Eq. 5 factor included).  groups[5 s + k]: segment s, group k.
    std::vector<AdamGroup> groups(5 * (size_t)b->S);
    int si = 0;
    for (int i = 0; i < n; ++i) {
      gsc_scene* sc = scenes[i];
      const double eta = 1.0 / (1.0 + std::log((double)reqs[i].viewport_frames));
      for (int l = 0; l < sc->K; ++l, ++si) {
        const int64_t nn = sc->n[l];
        if (!reqs[i].train || nn == 0) {
          for (int grp = 0; grp < 5; ++grp) groups[5 * si + grp].p = nullptr;
          continue;
        }
        const int64_t off[6] = {0, 3 * nn, 7 * nn, 10 * nn, 13 * nn, 14 * nn};
        // The bias corrections come from the level's device step count (set on the device
        // below), so a frame whose loss is not finite leaves moments and count untouched.
        for (int grp = 0; grp < 5; ++grp) {
          groups[5 * si + grp] = adam_params(sc->params[l] + off[grp], sc->m[l] + off[grp],
                                             sc->v[l] + off[grp], nullptr, off[grp + 1] - off[grp],
                                             (double)reqs[i].lr[grp] * eta, reqs[i].beta1,
                                             reqs[i].beta2, reqs[i].eps, reqs[i].weight_decay, 1,
                                             ctx->losses.as<float>() + i);
          groups[5 * si + grp].step = sc->d_step + l;
        }
      }
    }
    need(ctx, ctx->adam_tab, ctx->alloc, sizeof(AdamGroup) * groups.size(), "AdamW groups");
    upload(ctx, ctx->adam_tab.p, groups.data(), sizeof(AdamGroup) * groups.size());
    GSC_TRY(launch_adam_factors(st, ctx->adam_tab.as<AdamGroup>(), (int)groups.size()));
    { ProfScope ps_(ctx, P_PBADAM, st);
    GSC_TRY(launch_project_backward_adam(st, b->d_segs(), b->d_gstart(), b->S, b->d_cams(), b->G,
                                         b->grad2d.as<float>(), ctx->adam_tab.as<AdamGroup>()));
    }
    GSC_TRY(launch_adam_commit(st, ctx->adam_tab.as<AdamGroup>(), b->S));
  } else if (timing) {
    GSC_TRY(hipEventRecord(ctx->tev[4], st));
  }
  // The whole frame is enqueued; confirm the capacity (the host waits for the placement's count
  // only, the device has the rest of the frame queued).  An overflowed frame wrote nothing that
  // persists (no AdamW step, no step count) and is run again with room for its count.
  const uint64_t frame_cap = b->capacity;
  if (deferred) {
    GSC_TRY(hipEventSynchronize(ctx->ev_place));
    const uint64_t got = ctx->host_u64[kHostDeferredCount];
    if (got > frame_cap) {
      ctx->frame_capacity = got + got / 4 + 1024;
      ctx->acc_retries += 1;
      *retry = true;
      return GSC_OK;
    }
    b->n_instances = got;
    ctx->acc_instances += got;
    ctx->acc_frames += 1;
  }
  if (b->n_instances > ctx->frame_capacity - ctx->frame_capacity / 8)
    ctx->frame_capacity = b->n_instances + b->n_instances / 4 + 1024;
  if (timing) {
    GSC_TRY(hipEventRecord(ctx->tev[5], st));
    std::vector<float> losses(n);
    GSC_TRY(hipMemcpyAsync(losses.data(), ctx->losses.p, 4 * n, hipMemcpyDeviceToHost, st));
    GSC_TRY(hipMemcpyAsync(ctx->host_u64 + 1, ctx->vertices.p, 8, hipMemcpyDeviceToHost, st));
    GSC_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) {
      gsc_frame_stats& fs = stats[i];
      std::memset(&fs, 0, sizeof(fs));
      fs.ms_project_bin = elapsed(ctx->tev[0], ctx->tev[1]);
      fs.ms_forward = elapsed(ctx->tev[1], ctx->tev[2]);
      fs.ms_trace = elapsed(ctx->tev[6], ctx->tev[7]);
      fs.ms_loss = elapsed(ctx->tev[2], ctx->tev[3]);
      fs.ms_backward = any_train ? elapsed(ctx->tev[3], ctx->tev[4]) : 0.0;
      fs.ms_adam = any_train ? elapsed(ctx->tev[4], ctx->tev[5]) : 0.0;
      fs.ms_total = elapsed(ctx->tev[0], ctx->tev[5]);
      int64_t gi = 0;
      for (int l = 0; l < scenes[i]->K; ++l) gi += scenes[i]->n[l];
      fs.gaussians = (uint64_t)gi;
      fs.instances = b->n_instances;
      fs.tiles = (uint64_t)b->n_tiles;
      fs.pixels = (uint64_t)reqs[i].cam.w * reqs[i].cam.h;
      fs.paths = fs.pixels * reqs[i].trace.spp;
      fs.path_vertices = ctx->host_u64[1];
      fs.loss = (double)losses[i];
      fs.adam_skipped = (reqs[i].train && !std::isfinite(losses[i])) ? 1 : 0;
    }
  }
  return GSC_OK;
}

}  // namespace

// ---- checkpoint of the cache state ---------------------------------------------------------
// File: one header line of JSON written in exactly this form,
//   {"format":"gsc-scene-state","version":1,"dtype":"float32","byte_order":"little","levels":[{"n":N,"step":S},...]}\n
// then, per level, params, m and v, each 14 n float32 in the [pos][rot][log_scale][rgb][opacity]
// layout of the scene.  The loader accepts exactly what the writer produces.
namespace {

constexpr const char* kStateMagic = "{\"format\":\"gsc-scene-state\",\"version\":1,\"dtype\":\"float32\","
                                    "\"byte_order\":\"little\",\"levels\":[";

bool host_is_little_endian() {
  const uint32_t one = 1u;
  unsigned char b;
  std::memcpy(&b, &one, 1);
  return b == 1;
}

struct File {
  FILE* f = nullptr;
  ~File() { if (f) std::fclose(f); }
};

// Parses the header line; returns the per-level (n, step) pairs or fails with a message.
std::vector<std::pair<int64_t, int64_t>> parse_state_header(gsc_ctx* ctx, const std::string& line) {
  const size_t m = std::strlen(kStateMagic);
  if (line.compare(0, m, kStateMagic) != 0) invalid(ctx, "not a scene state file (header mismatch)");
  std::vector<std::pair<int64_t, int64_t>> lv;
  size_t pos = m;
  for (;;) {
    if (pos < line.size() && line[pos] == ']') break;
    if (!lv.empty()) {
      if (pos >= line.size() || line[pos] != ',') invalid(ctx, "malformed level list in scene state header");
      ++pos;
    }
    long long n = -1, step = -1;
    int used = 0;
    if (std::sscanf(line.c_str() + pos, "{\"n\":%lld,\"step\":%lld}%n", &n, &step, &used) != 2 || used == 0)
      invalid(ctx, "malformed level entry in scene state header");
    if (n < 0 || step < 0) invalid(ctx, "negative size or step in scene state header");
    lv.emplace_back((int64_t)n, (int64_t)step);
    pos += (size_t)used;
    if (lv.size() > 64) invalid(ctx, "too many levels in scene state header");
  }
  if (line.compare(pos, std::string::npos, "]}") != 0) invalid(ctx, "malformed end of scene state header");
  return lv;
}

}  // namespace

// =============================================================================================
// C ABI
// =============================================================================================
// ---- the allocation-free adjoint's scratch ------------------------------------------------------
// gsc_splat_backward_noalloc keeps its temporaries (the [G][16] screen-space gradients, the
// [14][G] parameter gradients before they are copied out, the tile schedule) in one file-scope
// device array instead of allocating them.  Every device the library runs on holds its own copy
// until the process ends; host code uses only the address hipGetSymbolAddress gives for the
// current device, looked up once per device.
constexpr int64_t kNoAllocMaxGaussians = int64_t(1) << 19;     // 524,288 Gaussians per call
constexpr int64_t kNoAllocMaxTiles = int64_t(1) << 18;         // 262,144 tiles per call
constexpr size_t kNoAllocScratchBytes =
    (size_t)(kGrad2dStride + 14) * 4 * (size_t)kNoAllocMaxGaussians + 4 * (size_t)kNoAllocMaxTiles;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
struct ScratchSlot {
  std::once_flag once;
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
};
ScratchSlot g_scratch[kMaxDevices];

// Called with `device` current.
void lookup_scratch(int device, void** ptr, hipError_t* err) {
  if (device < 0 || device >= kMaxDevices) {
    *ptr = nullptr;
    *err = hipErrorInvalidDevice;
    return;
  }
  ScratchSlot& slot = g_scratch[device];
  std::call_once(slot.once, [&]() {
    void* p = nullptr;
    slot.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    slot.ptr = slot.err == hipSuccess ? p : nullptr;
  });
  *ptr = slot.ptr;
  *err = slot.err;
}

// Ceiling micro-benchmarks: one launch between two events on the context stream.
namespace {
template <typename F>
gsc_status timed_probe(gsc_ctx* ctx, double* ms, F&& launch) {
  hipEvent_t a = pool_event(ctx), b = pool_event(ctx);
  GSC_TRY(hipEventRecord(a, ctx->stream));
  GSC_TRY(launch());
  GSC_TRY(hipEventRecord(b, ctx->stream));
  GSC_TRY(hipEventSynchronize(b));
  *ms = elapsed(a, b);
  ctx->ev_pool.push_back(a);
  ctx->ev_pool.push_back(b);
  return GSC_OK;
}

void check_probe_threads(gsc_ctx* ctx, uint32_t threads, int32_t per_thread) {
  if (threads == 0 || threads % 256 != 0) invalid(ctx, "threads must be a positive multiple of 256");
  if (per_thread < 1) invalid(ctx, "per_thread must be >= 1");
}
}  // namespace

extern "C" {

gsc_status gsc_ctx_create(int device, void* hip_stream, const gsc_allocator* alloc, gsc_ctx** out) {
  if (!out) return GSC_E_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return GSC_E_DEVICE;
  if (device < 0 || device >= count) return GSC_E_INVALID_ARG;
  if (alloc && (!alloc->alloc || !alloc->release)) return GSC_E_INVALID_ARG;
  gsc_ctx* c = new (std::nothrow) gsc_ctx();
  if (!c) return GSC_E_OUT_OF_MEMORY;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (alloc) { c->alloc.hook = *alloc; c->alloc.has = true; }
  bool ok = hipSetDevice(device) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&c->upload_ev, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&c->ev_place, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; i < 8 && ok; ++i) ok = hipEventCreate(&c->tev[i]) == hipSuccess;
  c->pinned_cap = size_t(4) << 20;
  ok = ok && hipHostMalloc((void**)&c->pinned, c->pinned_cap, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&c->host_u64, 8 * 32, hipHostMallocDefault) == hipSuccess;
  if (ok) lookup_scratch(device, &c->scratch, &c->scratch_err);
  if (!ok) {
    gsc_ctx_destroy(c);
    return GSC_E_DEVICE;
  }
  *out = c;
  return GSC_OK;
}

void gsc_ctx_destroy(gsc_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->side) (void)hipStreamSynchronize(c->side);
  if (c->frame_bin) { c->frame_bin->free_all(); delete c->frame_bin; }
  DevBuf* all[] = {&c->targets, &c->records, &c->dL, &c->partials, &c->losses, &c->grads14,
                   &c->images, &c->final_T, &c->last_id, &c->trace_tab, &c->vertices,
                   &c->composite_tmp, &c->d_stats, &c->adam_tab, &c->ini_tries, &c->ini_key,
                   &c->ini_id, &c->ini_key_tmp, &c->ini_id_tmp, &c->ini_hist, &c->ini_sort_tab,
                   &c->ini_start, &c->ini_end, &c->ini_spos, &c->ini_partial, &c->ini_pos,
                   &c->ini_alb, &c->ini_mean3, &c->ini_count};
  for (DevBuf* b : all) b->release(c->alloc);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->host_u64) (void)hipHostFree(c->host_u64);
  if (c->upload_ev) (void)hipEventDestroy(c->upload_ev);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->ev_place) (void)hipEventDestroy(c->ev_place);
  for (hipEvent_t e : c->tev) if (e) (void)hipEventDestroy(e);
  for (auto& p : c->prof_pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->side) (void)hipStreamDestroy(c->side);
  delete c;
}

const char* gsc_ctx_last_error(const gsc_ctx* ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

gsc_status gsc_ctx_set_stream(gsc_ctx* ctx, void* hip_stream) {
  if (!ctx) return GSC_E_INVALID_ARG;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->upload_pending = false;
  return guarded(ctx, [&]() -> gsc_status {
    // Make sure no staged upload on the previous stream is still reading the ring.
    GSC_TRY(hipDeviceSynchronize());
    return GSC_OK;
  });
}

gsc_status gsc_ctx_set_deterministic(gsc_ctx* ctx, int32_t on) {
  if (!ctx) return GSC_E_INVALID_ARG;
  ctx->deterministic = on ? 1 : 0;
  return GSC_OK;
}

gsc_status gsc_ctx_set_work_counters(gsc_ctx* ctx, int32_t on) {
  if (!ctx) return GSC_E_INVALID_ARG;
  ctx->work_counters = on != 0;
  return GSC_OK;
}

gsc_status gsc_ctx_set_frame_binning(gsc_ctx* ctx, int32_t on) {
  if (!ctx) return GSC_E_INVALID_ARG;
  ctx->frame_binning = on != 0;
  return GSC_OK;
}

gsc_status gsc_ctx_set_frame_tiles(gsc_ctx* ctx, int32_t tile_px) {
  if (!ctx) return GSC_E_INVALID_ARG;
  if (tile_px != 0 && tile_px != 16 && tile_px != 32) {
    ctx->err = "frame tile size must be 0 (automatic), 16 or 32";
    return GSC_E_INVALID_ARG;
  }
  ctx->frame_tiles = tile_px;
  return GSC_OK;
}

gsc_status gsc_ctx_set_list_cut(gsc_ctx* ctx, int32_t on) {
  if (!ctx) return GSC_E_INVALID_ARG;
  ctx->list_cut = on ? 1 : 0;
  return GSC_OK;
}

uint64_t gsc_ctx_required_capacity(const gsc_ctx* ctx) { return ctx ? ctx->required : 0; }

gsc_status gsc_ctx_trim(gsc_ctx* ctx) {
  return guarded(ctx, [&]() -> gsc_status {
    GSC_TRY(hipStreamSynchronize(ctx->stream));
    if (ctx->frame_bin) { ctx->frame_bin->free_all(); delete ctx->frame_bin; ctx->frame_bin = nullptr; }
    DevBuf* all[] = {&ctx->targets, &ctx->records, &ctx->dL, &ctx->partials, &ctx->losses,
                     &ctx->grads14, &ctx->images, &ctx->final_T, &ctx->last_id, &ctx->trace_tab,
                     &ctx->vertices, &ctx->composite_tmp, &ctx->adam_tab, &ctx->ini_tries,
                     &ctx->ini_key, &ctx->ini_id, &ctx->ini_key_tmp, &ctx->ini_id_tmp,
                     &ctx->ini_hist, &ctx->ini_sort_tab, &ctx->ini_start, &ctx->ini_end,
                     &ctx->ini_spos, &ctx->ini_partial, &ctx->ini_pos, &ctx->ini_alb,
                     &ctx->ini_mean3, &ctx->ini_count};
    for (DevBuf* b : all) b->release(ctx->alloc);
    return GSC_OK;
  });
}

gsc_status gsc_trace_targets(gsc_ctx* ctx, const gsc_volume* vol, const gsc_camera* cam,
                             const gsc_trace_params* params, float* targets,
                             gsc_path_record* records, gsc_frame_stats* stats) {
  return guarded(ctx, [&]() -> gsc_status {
    if (!vol || !vol->density) invalid(ctx, "volume or density is NULL");
    if (vol->nx < 1 || vol->ny < 1 || vol->nz < 1) invalid(ctx, "volume dimensions must be >= 1");
    if (!(vol->density_max > 0.0f) || !std::isfinite(vol->density_max)) invalid(ctx, "density_max must be positive");
    check_volume_host(ctx, vol->tf_rgba, vol->tf_points, vol->lights, vol->n_lights, vol->spheres,
                      vol->n_spheres);
    check_camera(ctx, cam);
    check_trace_params(ctx, params);
    if (!targets) invalid(ctx, "targets is NULL");
    TraceDesc d = make_trace_desc(vol->density, nullptr, vol->nx, vol->ny, vol->nz, vol->density_max,
                                  vol->tf_rgba, vol->tf_points, vol->lights, vol->n_lights,
                                  vol->spheres, vol->n_spheres, *cam, *params);
    d.pix_off = 0;
    d.targets = targets;
    d.records = records;
    const size_t bytes = sizeof(TraceDesc) + sizeof(int64_t);
    need(ctx, ctx->trace_tab, ctx->alloc, bytes, "trace descriptor");
    need(ctx, ctx->vertices, ctx->alloc, 8, "vertex counter");
    std::vector<char> h(bytes, 0);
    std::memcpy(h.data(), &d, sizeof(TraceDesc));
    upload(ctx, ctx->trace_tab.p, h.data(), bytes);
    hipStream_t st = ctx->stream;
    GSC_TRY(hipMemsetAsync(ctx->vertices.p, 0, 8, st));
    if (stats) GSC_TRY(hipEventRecord(ctx->tev[6], st));
    const int64_t P = (int64_t)cam->w * cam->h;
  { ProfScope ps_(ctx, P_TRACE, st);
  GSC_TRY(launch_trace(st, ctx->trace_tab.as<TraceDesc>(),
                         (const int64_t*)((char*)ctx->trace_tab.p + sizeof(TraceDesc)), 1,
                         trace_align(P), ctx->vertices.as<unsigned long long>()));
  }
    if (stats) {
      GSC_TRY(hipEventRecord(ctx->tev[7], st));
      GSC_TRY(hipMemcpyAsync(ctx->host_u64 + 1, ctx->vertices.p, 8, hipMemcpyDeviceToHost, st));
      GSC_TRY(hipStreamSynchronize(st));
      std::memset(stats, 0, sizeof(*stats));
      stats->ms_trace = elapsed(ctx->tev[6], ctx->tev[7]);
      stats->paths = (uint64_t)P * params->spp;
      stats->pixels = (uint64_t)P;
      stats->path_vertices = ctx->host_u64[1];
    }
    return GSC_OK;
  });
}

gsc_status gsc_project_bin(gsc_ctx* ctx, const gsc_gaussians* levels, int32_t num_levels,
                           const gsc_camera* cam, uint64_t capacity_hint, gsc_binning** out) {
  return guarded(ctx, [&]() -> gsc_status {
    if (!out) invalid(ctx, "out is NULL");
    *out = nullptr;
    check_levels(ctx, levels, num_levels);
    check_camera(ctx, cam);
    gsc_binning* b = new gsc_binning();
    b->alloc = ctx->alloc;
    std::vector<ReqSpec> specs(1);
    specs[0].cam = *cam;
    specs[0].levels.assign(levels, levels + num_levels);
    b->K = num_levels;
    const bool fb = ctx->frame_binning != 0;
    const int tsx = fb ? kFrameTileShiftX : kTileShift, tsy = fb ? kFrameTileShiftY : kTileShift;
    b->TX = (cam->w + (1 << tsx) - 1) >> tsx;
    b->TY = (cam->h + (1 << tsy) - 1) >> tsy;
    b->list_cut = fb && ctx->list_cut != 0;
    gsc_status s;
    try {
      plan_batch(ctx, b, specs, tsx, tsy);
      s = run_project_bin(ctx, b, capacity_hint);
    } catch (...) {
      b->free_all();
      delete b;
      throw;
    }
    if (s != GSC_OK) {
      (void)hipStreamSynchronize(ctx->stream);
      b->free_all();
      delete b;
      return s;
    }
    *out = b;
    return GSC_OK;
  });
}

gsc_status gsc_binning_view(gsc_ctx* ctx, const gsc_binning* bin, gsc_binning_info* out) {
  return guarded(ctx, [&]() -> gsc_status {
    if (!bin || !out) invalid(ctx, "NULL argument");
    gsc_binning* b = const_cast<gsc_binning*>(bin);
    need(ctx, b->view_window, b->alloc, 16 * (size_t)std::max<int64_t>(b->G, 1), "window view");
    need(ctx, b->view_screen, b->alloc, 24 * (size_t)std::max<int64_t>(b->G, 1), "screen view");
    GSC_TRY(launch_view(ctx->stream, b->G, b->rec.as<SplatRec>(), b->tiles.as<uint32_t>(),
                        b->view_window.as<int32_t>(), b->view_screen.as<float>()));
    GSC_TRY(hipStreamSynchronize(ctx->stream));
    std::memset(out, 0, sizeof(*out));
    out->n_instances = b->n_instances;
    out->n_tiles = (uint64_t)b->n_tiles;
    out->num_levels = b->S;
    out->tiles_x = b->TX;
    out->tiles_y = b->TY;
    for (int s = 0; s < b->S && s < 8; ++s) out->gauss_offset[s] = b->segs[s].g_off;
    out->gauss_offset[std::min(b->S, 8)] = b->G;
    out->values = b->values.as<uint32_t>();
    out->ranges = b->ranges.as<uint64_t>();
    out->window = b->view_window.as<int32_t>();
    out->tiles_touched = b->tiles.as<uint32_t>();
    out->depth_key = b->depth_key.as<uint32_t>();
    out->screen = b->view_screen.as<float>();
    return GSC_OK;
  });
}

gsc_status gsc_binning_keys(gsc_ctx* ctx, const gsc_binning* bin, uint64_t* keys) {
  return guarded(ctx, [&]() -> gsc_status {
    if (!bin) invalid(ctx, "NULL binning");
    const gsc_binning* b = bin;
    if (b->n_instances == 0) return GSC_OK;
    if (!keys) invalid(ctx, "keys is NULL");
    GSC_TRY(launch_binning_keys(ctx->stream, b->d_tstart(), b->S, b->d_gstart(), b->n_tiles,
                                b->tile_start.as<uint64_t>(), b->d_ninst(), b->n_instances,
                                b->values.as<uint32_t>(), b->depth_key.as<uint32_t>(), keys));
    return GSC_OK;
  });
}

void gsc_binning_release(gsc_ctx* ctx, gsc_binning* bin) {
  if (!bin) return;
  if (ctx) {
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
  }
  bin->free_all();
  delete bin;
}

gsc_status gsc_splat_forward(gsc_ctx* ctx, gsc_binning* bin, float* images, float* final_T,
                             int32_t* last_id) {
  return guarded(ctx, [&]() -> gsc_status {
    if (!bin || !images || !final_T || !last_id) invalid(ctx, "NULL argument");
    run_forward(ctx, bin, images, final_T, last_id);
    return GSC_OK;
  });
}

namespace {
gsc_binning* check_backward_args(gsc_ctx* ctx, const gsc_binning* bin, const gsc_gaussians* levels,
                                 int32_t num_levels, const gsc_camera* cam, const float* final_T,
                                 const int32_t* last_id, const float* dL_dimages,
                                 const gsc_grads* grads) {
  if (!bin || !final_T || !last_id || !dL_dimages || !grads) invalid(ctx, "NULL argument");
  gsc_binning* b = const_cast<gsc_binning*>(bin);
  if (!b->forward_done) invalid(ctx, "gsc_splat_forward has not run on this binning");
  check_levels(ctx, levels, num_levels);
  check_camera(ctx, cam);
  if (num_levels != b->S) invalid(ctx, "num_levels differs from the binning's");
  for (int l = 0; l < num_levels; ++l) {
    const Seg& sg = b->segs[l];
    if (levels[l].n != sg.n || levels[l].pos != sg.pos || levels[l].rot != sg.rot ||
        levels[l].log_scale != sg.ls || levels[l].rgb != sg.rgb ||
        levels[l].opacity_logit != sg.logit)
      invalid(ctx, "levels differ from those given to gsc_project_bin");
    if (levels[l].n > 0 && (!grads[l].pos || !grads[l].rot || !grads[l].log_scale ||
                            !grads[l].rgb || !grads[l].opacity_logit))
      invalid(ctx, "gradient pointer is NULL");
  }
  return b;
}

// Copies each level's 14 gradients ([14 n] in the binning's segment order) to the caller's arrays.
void copy_out_grads(gsc_ctx* ctx, const gsc_binning* b, const gsc_gaussians* levels, int num_levels,
                    const float* grads14, const gsc_grads* grads) {
  for (int l = 0; l < num_levels; ++l) {
    const int64_t nn = levels[l].n;
    if (nn == 0) continue;
    const float* g = grads14 + 14 * b->segs[l].g_off;
    GSC_TRY(hipMemcpyAsync(grads[l].pos, g, 12 * nn, hipMemcpyDeviceToDevice, ctx->stream));
    GSC_TRY(hipMemcpyAsync(grads[l].rot, g + 3 * nn, 16 * nn, hipMemcpyDeviceToDevice, ctx->stream));
    GSC_TRY(hipMemcpyAsync(grads[l].log_scale, g + 7 * nn, 12 * nn, hipMemcpyDeviceToDevice, ctx->stream));
    GSC_TRY(hipMemcpyAsync(grads[l].rgb, g + 10 * nn, 12 * nn, hipMemcpyDeviceToDevice, ctx->stream));
    GSC_TRY(hipMemcpyAsync(grads[l].opacity_logit, g + 13 * nn, 4 * nn, hipMemcpyDeviceToDevice, ctx->stream));
  }
}
}  // namespace

gsc_status gsc_splat_backward(gsc_ctx* ctx, const gsc_binning* bin, const gsc_gaussians* levels,
                              int32_t num_levels, const gsc_camera* cam, const float* final_T,
                              const int32_t* last_id, const float* dL_dimages,
                              const gsc_grads* grads) {
  return guarded(ctx, [&]() -> gsc_status {
    gsc_binning* b = check_backward_args(ctx, bin, levels, num_levels, cam, final_T, last_id,
                                         dL_dimages, grads);
    need(ctx, ctx->grads14, ctx->alloc, 4 * 14 * (size_t)std::max<int64_t>(b->G, 1), "parameter gradients");
    run_backward(ctx, b, final_T, dL_dimages, ctx->grads14.as<float>());
    copy_out_grads(ctx, b, levels, num_levels, ctx->grads14.as<float>(), grads);
    return GSC_OK;
  });
}

gsc_status gsc_splat_backward_noalloc(gsc_ctx* ctx, const gsc_binning* bin,
                                      const gsc_gaussians* levels, int32_t num_levels,
                                      const gsc_camera* cam, const float* final_T,
                                      const int32_t* last_id, const float* dL_dimages,
                                      const gsc_grads* grads) {
  return guarded(ctx, [&]() -> gsc_status {
    gsc_binning* b = check_backward_args(ctx, bin, levels, num_levels, cam, final_T, last_id,
                                         dL_dimages, grads);
    if (ctx->deterministic)
      invalid(ctx, "gsc_splat_backward_noalloc sums with float atomics; switch the deterministic "
                   "mode off (gsc_ctx_set_deterministic)");
    if (b->G > kNoAllocMaxGaussians) {
      char buf[200];
      snprintf(buf, sizeof(buf), "gsc_splat_backward_noalloc takes at most %lld Gaussians per call; "
               "the binning holds %lld", (long long)kNoAllocMaxGaussians, (long long)b->G);
      invalid(ctx, buf);
    }
    if (b->n_tiles > kNoAllocMaxTiles) {
      char buf[200];
      snprintf(buf, sizeof(buf), "gsc_splat_backward_noalloc takes at most %lld tiles per call; "
               "the binning holds %lld", (long long)kNoAllocMaxTiles, (long long)b->n_tiles);
      invalid(ctx, buf);
    }
    if (!ctx->scratch) {
      char buf[200];
      snprintf(buf, sizeof(buf), "no address for the allocation-free adjoint's device array on "
               "device %d (hipGetSymbolAddress: %s)", ctx->device, hipGetErrorString(ctx->scratch_err));
      ctx->err = buf;
      return GSC_E_DEVICE;
    }
    hipStream_t st = ctx->stream;
    const int64_t G = b->G;
    float* g2d = (float*)ctx->scratch;
    float* g14 = g2d + kGrad2dStride * kNoAllocMaxGaussians;
    uint32_t* order = (uint32_t*)(g14 + 14 * kNoAllocMaxGaussians);
    // Cleared by a kernel (no memset node), so the call can be captured in a graph.
    GSC_TRY(launch_fill_u32(st, (uint32_t*)g2d, 0u, kGrad2dStride * G));
    GSC_TRY(launch_tile_order(st, b->ranges.as<uint64_t>(), b->tile_work.as<uint32_t>(), b->n_tiles,
                              order));
    GSC_TRY(launch_splat_backward(st, b->d_segs(), b->d_tstart(), b->S, b->d_cams(), b->n_tiles,
                                  b->ranges.as<uint64_t>(), b->values.as<uint32_t>(),
                                  b->rec.as<SplatRec>(), final_T, b->n_contrib.as<uint32_t>(),
                                  dL_dimages, g2d, G, order, nullptr, nullptr, nullptr, false,
                                  b->tsx, b->tsy, b->d_ninst(), b->capacity));
    GSC_TRY(launch_project_backward(st, b->d_segs(), b->d_gstart(), b->S, b->d_cams(), G, g2d, g14));
    copy_out_grads(ctx, b, levels, num_levels, g14, grads);
    return GSC_OK;
  });
}

gsc_status gsc_loss_composite(gsc_ctx* ctx, const float* images, const float* targets,
                              const gsc_path_record* records, int32_t spp, int32_t num_levels,
                              int32_t w, int32_t h, int32_t loss, float* dL_dimages,
                              float* loss_out, float* composite) {
  return guarded(ctx, [&]() -> gsc_status {
    if (!images || !targets || !dL_dimages || !loss_out) invalid(ctx, "NULL argument");
    if (spp < 1) invalid(ctx, "spp must be >= 1");
    if (num_levels < 1 || num_levels > 8) invalid(ctx, "num_levels must be in [1, 8]");
    if (w < 1 || h < 1 || w > 16384 || h > 16384) invalid(ctx, "image size out of range");
    if (loss != 0 && loss != 1) invalid(ctx, "loss must be 0 or 1");
    if ((records == nullptr) != (composite == nullptr)) invalid(ctx, "records and composite go together");
    const int np = loss_num_partials((int64_t)w * h);
    need(ctx, ctx->partials, ctx->alloc, 8 * (size_t)np, "loss partials");
    GSC_TRY(launch_loss_composite(ctx->stream, images, targets, records, spp, num_levels, w, h, loss,
                                  dL_dimages, ctx->partials.as<double>(), loss_out, composite));
    return GSC_OK;
  });
}

gsc_status gsc_adam_step(gsc_ctx* ctx, float* param, float* m, float* v, const float* grad,
                         int64_t count, const gsc_adam_hparams* hp) {
  return guarded(ctx, [&]() -> gsc_status {
    if (!hp) invalid(ctx, "hparams NULL");
    if (count < 0) invalid(ctx, "count must be >= 0");
    if (count > 0 && (!param || !m || !v || !grad)) invalid(ctx, "NULL argument");
    if (hp->step < 1) invalid(ctx, "step must be >= 1");
    if (!(hp->beta1 >= 0.0 && hp->beta1 < 1.0) || !(hp->beta2 >= 0.0 && hp->beta2 < 1.0))
      invalid(ctx, "betas must be in [0, 1)");
    if (!std::isfinite(hp->lr) || !std::isfinite(hp->eps) || !std::isfinite(hp->weight_decay))
      invalid(ctx, "hyper-parameters must be finite");
    adam_group(ctx, param, m, v, grad, count, hp->lr, hp->beta1, hp->beta2, hp->eps,
               hp->weight_decay, hp->step, nullptr);
    return GSC_OK;
  });
}

gsc_status gsc_scene_create(gsc_ctx* ctx, const gsc_volume* vol, const gsc_gaussians* init_levels,
                            int32_t K, gsc_scene** out) {
  return guarded(ctx, [&]() -> gsc_status {
    if (!out) invalid(ctx, "out is NULL");
    *out = nullptr;
    if (!vol || !vol->density) invalid(ctx, "volume or density is NULL");
    if (vol->nx < 1 || vol->ny < 1 || vol->nz < 1) invalid(ctx, "volume dimensions must be >= 1");
    if (!(vol->density_max > 0.0f)) invalid(ctx, "density_max must be positive");
    check_volume_host(ctx, vol->tf_rgba, vol->tf_points, vol->lights, vol->n_lights, vol->spheres,
                      vol->n_spheres);
    check_levels(ctx, init_levels, K);
    gsc_scene* sc = new gsc_scene();
    sc->alloc = ctx->alloc;
    auto cleanup = [&]() {
      for (float* p : sc->params) sc->alloc.put(p);
      for (float* p : sc->m) sc->alloc.put(p);
      for (float* p : sc->v) sc->alloc.put(p);
      sc->alloc.put(sc->cells);
      sc->alloc.put(sc->d_step);
      delete sc;
    };
    try {
      sc->K = K;
      sc->nx = vol->nx; sc->ny = vol->ny; sc->nz = vol->nz;
      sc->dmax = vol->density_max;
      sc->tf.assign(vol->tf_rgba, vol->tf_rgba + 4 * vol->tf_points);
      sc->lights.assign(vol->lights, vol->lights + 6 * vol->n_lights);
      sc->spheres.assign(vol->spheres, vol->spheres + 7 * vol->n_spheres);
      const size_t vb = cells_bytes(vol->nx, vol->ny, vol->nz);
      sc->cells = (float4*)sc->alloc.get(vb);
      if (!sc->cells) oom(ctx, "scene volume", vb);
      GSC_TRY(launch_build_cells(ctx->stream, vol->density, vol->nx, vol->ny, vol->nz, sc->cells));
      sc->d_step = (int64_t*)sc->alloc.get(8 * (size_t)K);
      if (!sc->d_step) oom(ctx, "scene step counts", 8 * (size_t)K);
      GSC_TRY(hipMemsetAsync(sc->d_step, 0, 8 * (size_t)K, ctx->stream));
      for (int l = 0; l < K; ++l) {
        const int64_t nn = init_levels[l].n;
        const size_t bytes = 4 * 14 * (size_t)std::max<int64_t>(nn, 1);
        float* p = (float*)sc->alloc.get(bytes);
        float* m = (float*)sc->alloc.get(bytes);
        float* v = (float*)sc->alloc.get(bytes);
        sc->params.push_back(p); sc->m.push_back(m); sc->v.push_back(v);
        if (!p || !m || !v) oom(ctx, "scene parameters", bytes);
        sc->n.push_back(nn);
        if (nn > 0) {
          const gsc_gaussians& g = init_levels[l];
          GSC_TRY(hipMemcpyAsync(p, g.pos, 12 * nn, hipMemcpyDeviceToDevice, ctx->stream));
          GSC_TRY(hipMemcpyAsync(p + 3 * nn, g.rot, 16 * nn, hipMemcpyDeviceToDevice, ctx->stream));
          GSC_TRY(hipMemcpyAsync(p + 7 * nn, g.log_scale, 12 * nn, hipMemcpyDeviceToDevice, ctx->stream));
          GSC_TRY(hipMemcpyAsync(p + 10 * nn, g.rgb, 12 * nn, hipMemcpyDeviceToDevice, ctx->stream));
          GSC_TRY(hipMemcpyAsync(p + 13 * nn, g.opacity_logit, 4 * nn, hipMemcpyDeviceToDevice, ctx->stream));
        }
        GSC_TRY(hipMemsetAsync(m, 0, bytes, ctx->stream));
        GSC_TRY(hipMemsetAsync(v, 0, bytes, ctx->stream));
      }
    } catch (...) {
      cleanup();
      throw;
    }
    *out = sc;
    return GSC_OK;
  });
}

void gsc_scene_destroy(gsc_ctx* ctx, gsc_scene* sc) {
  if (!sc) return;
  if (ctx) {
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
  }
  for (float* p : sc->params) sc->alloc.put(p);
  for (float* p : sc->m) sc->alloc.put(p);
  for (float* p : sc->v) sc->alloc.put(p);
  sc->alloc.put(sc->cells);
  sc->alloc.put(sc->d_step);
  delete sc;
}

gsc_status gsc_scene_set_optics(gsc_ctx* ctx, gsc_scene* sc, const float* tf_rgba, int32_t tf_points,
                                const float* lights, int32_t n_lights, const float* spheres,
                                int32_t n_spheres) {
  return guarded(ctx, [&]() -> gsc_status {
    if (!sc) invalid(ctx, "scene is NULL");
    check_volume_host(ctx, tf_rgba, tf_points, lights, n_lights, spheres, n_spheres);
    sc->tf.assign(tf_rgba, tf_rgba + 4 * tf_points);
    sc->lights.assign(lights, lights + 6 * n_lights);
    sc->spheres.assign(spheres, spheres + 7 * n_spheres);
    return GSC_OK;
  });
}

gsc_status gsc_scene_level(const gsc_scene* sc, int32_t l, gsc_gaussians* out) {
  if (!sc || !out || l < 0 || l >= sc->K) return GSC_E_INVALID_ARG;
  float* p = sc->params[l];
  const int64_t nn = sc->n[l];
  out->pos = p; out->rot = p + 3 * nn; out->log_scale = p + 7 * nn; out->rgb = p + 10 * nn;
  out->opacity_logit = p + 13 * nn; out->n = nn;
  return GSC_OK;
}

gsc_status gsc_scene_state(const gsc_scene* sc, int32_t l, float** params, float** m, float** v,
                           int64_t* n, int64_t* step) {
  if (!sc || l < 0 || l >= sc->K || !params || !m || !v || !n || !step) return GSC_E_INVALID_ARG;
  *params = sc->params[l];
  *m = sc->m[l];
  *v = sc->v[l];
  *n = sc->n[l];
  // The count lives on the device and advances with the frames' updates: wait for the device.
  if (hipDeviceSynchronize() != hipSuccess) return GSC_E_DEVICE;
  if (hipMemcpy(step, sc->d_step + l, 8, hipMemcpyDeviceToHost) != hipSuccess) return GSC_E_DEVICE;
  return GSC_OK;
}

gsc_status gsc_scene_copy_state(gsc_ctx* ctx, gsc_scene* dst, const gsc_scene* src) {
  return guarded(ctx, [&]() -> gsc_status {
    if (!dst || !src) invalid(ctx, "NULL scene");
    if (dst->K != src->K) invalid(ctx, "level counts differ");
    for (int l = 0; l < src->K; ++l) if (dst->n[l] != src->n[l]) invalid(ctx, "level sizes differ");
    for (int l = 0; l < src->K; ++l) {
      const size_t bytes = 4 * 14 * (size_t)src->n[l];
      if (bytes == 0) continue;
      GSC_TRY(hipMemcpyAsync(dst->params[l], src->params[l], bytes, hipMemcpyDeviceToDevice, ctx->stream));
      GSC_TRY(hipMemcpyAsync(dst->m[l], src->m[l], bytes, hipMemcpyDeviceToDevice, ctx->stream));
      GSC_TRY(hipMemcpyAsync(dst->v[l], src->v[l], bytes, hipMemcpyDeviceToDevice, ctx->stream));
    }
    GSC_TRY(hipMemcpyAsync(dst->d_step, src->d_step, 8 * (size_t)src->K, hipMemcpyDeviceToDevice,
                           ctx->stream));
    return GSC_OK;
  });
}


gsc_status gsc_scene_save(gsc_ctx* ctx, const gsc_scene* sc, const char* path) {
  return guarded(ctx, [&]() -> gsc_status {
    if (!sc || !path) invalid(ctx, "NULL scene or path");
    if (!host_is_little_endian()) invalid(ctx, "scene state files are little-endian; host is not");
    std::vector<int64_t> steps(sc->K);
    GSC_TRY(hipMemcpyAsync(steps.data(), sc->d_step, 8 * (size_t)sc->K, hipMemcpyDeviceToHost,
                           ctx->stream));
    GSC_TRY(hipStreamSynchronize(ctx->stream));
    std::string hdr = kStateMagic;
    for (int l = 0; l < sc->K; ++l) {
      char buf[96];
      std::snprintf(buf, sizeof buf, "%s{\"n\":%lld,\"step\":%lld}", l ? "," : "", (long long)sc->n[l],
                    (long long)steps[l]);
      hdr += buf;
    }
    hdr += "]}\n";
    File out;
    out.f = std::fopen(path, "wb");
    if (!out.f) invalid(ctx, std::string("cannot open ") + path + " for writing");
    if (std::fwrite(hdr.data(), 1, hdr.size(), out.f) != hdr.size()) invalid(ctx, "write failed");
    std::vector<float> host;
    for (int l = 0; l < sc->K; ++l) {
      const size_t cnt = 14 * (size_t)sc->n[l];
      if (cnt == 0) continue;
      host.resize(cnt);
      for (float* dev : {sc->params[l], sc->m[l], sc->v[l]}) {
        GSC_TRY(hipMemcpyAsync(host.data(), dev, 4 * cnt, hipMemcpyDeviceToHost, ctx->stream));
        GSC_TRY(hipStreamSynchronize(ctx->stream));
        if (std::fwrite(host.data(), 4, cnt, out.f) != cnt) invalid(ctx, "write failed");
      }
    }
    if (std::fclose(out.f) != 0) { out.f = nullptr; invalid(ctx, "write failed"); }
    out.f = nullptr;
    return GSC_OK;
  });
}

gsc_status gsc_scene_load(gsc_ctx* ctx, gsc_scene* sc, const char* path) {
  return guarded(ctx, [&]() -> gsc_status {
    if (!sc || !path) invalid(ctx, "NULL scene or path");
    if (!host_is_little_endian()) invalid(ctx, "scene state files are little-endian; host is not");
    File in;
    in.f = std::fopen(path, "rb");
    if (!in.f) invalid(ctx, std::string("cannot open ") + path);
    std::string line;
    for (int c; (c = std::fgetc(in.f)) != '\n';) {
      if (c == EOF) invalid(ctx, "scene state file ends inside its header");
      line.push_back((char)c);
      if (line.size() > (1u << 16)) invalid(ctx, "scene state header too long");
    }
    const auto lv = parse_state_header(ctx, line);
    if ((int)lv.size() != sc->K) invalid(ctx, "scene state file holds a different number of levels");
    size_t payload = 0;
    for (int l = 0; l < sc->K; ++l) {
      if (lv[l].first != sc->n[l]) invalid(ctx, "scene state file holds different level sizes");
      payload += 3 * 14 * 4 * (size_t)sc->n[l];
    }
    const long start = std::ftell(in.f);
    if (start < 0 || std::fseek(in.f, 0, SEEK_END) != 0) invalid(ctx, "cannot size scene state file");
    const long end = std::ftell(in.f);
    if (end < 0 || (size_t)(end - start) != payload) invalid(ctx, "scene state file has the wrong length");
    if (std::fseek(in.f, start, SEEK_SET) != 0) invalid(ctx, "cannot read scene state file");
    // Everything is validated; only now is the device touched.
    std::vector<float> host;
    for (int l = 0; l < sc->K; ++l) {
      const size_t cnt = 14 * (size_t)sc->n[l];
      if (cnt == 0) continue;
      host.resize(cnt);
      for (float* dev : {sc->params[l], sc->m[l], sc->v[l]}) {
        if (std::fread(host.data(), 4, cnt, in.f) != cnt) invalid(ctx, "read failed");
        GSC_TRY(hipMemcpyAsync(dev, host.data(), 4 * cnt, hipMemcpyHostToDevice, ctx->stream));
        GSC_TRY(hipStreamSynchronize(ctx->stream));
      }
    }
    std::vector<int64_t> steps(sc->K);
    for (int l = 0; l < sc->K; ++l) steps[l] = lv[l].second;
    GSC_TRY(hipMemcpyAsync(sc->d_step, steps.data(), 8 * (size_t)sc->K, hipMemcpyHostToDevice,
                           ctx->stream));
    GSC_TRY(hipStreamSynchronize(ctx->stream));
    return GSC_OK;
  });
}

size_t gsc_scene_footprint_bytes(const gsc_scene* sc) {
  if (!sc) return 0;
  size_t b = cells_bytes(sc->nx, sc->ny, sc->nz);
  for (int l = 0; l < sc->K; ++l) b += 3 * 14 * 4 * (size_t)sc->n[l];
  return b;
}

size_t gsc_frame_footprint_bytes(const gsc_scene* sc, int32_t w, int32_t h, uint64_t instance_estimate) {
  if (!sc || w < 1 || h < 1) return 0;
  int64_t G = 0;
  for (int l = 0; l < sc->K; ++l) G += sc->n[l];
  const size_t P = (size_t)w * h;
  const size_t K = (size_t)sc->K;
  const int tw = 1 << kTileShift, th = 1 << kTileShift;   // the smaller frame tiles (more of them)
  const size_t tiles = K * (size_t)((w + tw - 1) / tw) * ((h + th - 1) / th);
  size_t b = 0;
  b += (size_t)G * (48 + 4 + 8 + 4 + 4 * 4 + 8 + 4 * kGrad2dStride + 14 * 4);  // per Gaussian
  b += 4 * (size_t)instance_estimate;                              // instance ids
  b += tiles * (8 + 16 + 4) + 4 * tiles * (size_t)((G / (int64_t)K + kChunk - 1) / kChunk);
  b += P * K * (12 * 3 + 4 + 4 + 4) + P * (20 + 12);              // images, targets, dL, T, ids
  return b;
}

gsc_status gsc_render_frame(gsc_ctx* ctx, gsc_scene* scene, const gsc_frame_request* req,
                            float* image, gsc_frame_stats* stats) {
  return guarded(ctx, [&]() -> gsc_status {
    gsc_scene* const scenes[1] = {scene};
    float* const images[1] = {image};
    if (!req) invalid(ctx, "request is NULL");
    bool retry = false;
    gsc_status st = render_batch(ctx, scenes, req, images, 1, stats, &retry);
    if (st == GSC_OK && retry) st = render_batch(ctx, scenes, req, images, 1, stats, &retry);
    return (st == GSC_OK && retry) ? GSC_E_CAPACITY : st;
  });
}

gsc_status gsc_render_frames(gsc_ctx* ctx, gsc_scene* const* scenes, const gsc_frame_request* reqs,
                             float* const* images, int32_t n, gsc_frame_stats* stats) {
  return guarded(ctx, [&]() -> gsc_status {
    bool retry = false;
    gsc_status st = render_batch(ctx, scenes, reqs, images, n, stats, &retry);
    if (st == GSC_OK && retry) st = render_batch(ctx, scenes, reqs, images, n, stats, &retry);
    return (st == GSC_OK && retry) ? GSC_E_CAPACITY : st;
  });
}

}  // extern "C"

namespace {

// ---- cache initialisation (Method: "Cache Initialization", Eq. 2) ------------------------------
constexpr int kInitMaxAttempts = 4096;

void check_init_volume(gsc_ctx* ctx, const gsc_volume* vol) {
  if (!vol || !vol->density) invalid(ctx, "volume or density is NULL");
  if (vol->nx < 1 || vol->ny < 1 || vol->nz < 1) invalid(ctx, "volume dimensions must be >= 1");
  if (!(vol->density_max > 0.0f) || !std::isfinite(vol->density_max)) invalid(ctx, "density_max must be positive");
  if (vol->tf_points < 2 || vol->tf_points > kMaxTf) invalid(ctx, "tf_points must be in [2, 64]");
  if (!vol->tf_rgba) invalid(ctx, "tf_rgba is NULL");
  for (int i = 0; i < 4 * vol->tf_points; ++i)
    if (!std::isfinite(vol->tf_rgba[i])) invalid(ctx, "transfer function not finite");
  if (!(max_alpha(vol->tf_rgba, vol->tf_points) > 0.0f))
    invalid(ctx, "transfer function opacity is zero everywhere (no majorant)");
}

void run_init_points(gsc_ctx* ctx, const gsc_volume* vol, int64_t n, uint64_t seed, float* pos,
                     float* albedo) {
  gsc_camera cam{};
  gsc_trace_params tp{};
  tp.seed = seed;
  TraceDesc d = make_trace_desc(vol->density, nullptr, vol->nx, vol->ny, vol->nz, vol->density_max,
                                vol->tf_rgba, vol->tf_points, nullptr, 0, nullptr, 0, cam, tp);
  need(ctx, ctx->trace_tab, ctx->alloc, sizeof(TraceDesc) + sizeof(int64_t), "trace descriptor");
  upload(ctx, ctx->trace_tab.p, &d, sizeof(TraceDesc));
  need(ctx, ctx->ini_tries, ctx->alloc, 4 * (size_t)n, "init attempts");
  need(ctx, ctx->ini_count, ctx->alloc, 8, "init failure count");
  hipStream_t st = ctx->stream;
  GSC_TRY(launch_init_points(st, ctx->trace_tab.as<TraceDesc>(), n, kInitMaxAttempts, pos, albedo,
                             ctx->ini_tries.as<int32_t>()));
  GSC_TRY(hipMemsetAsync(ctx->ini_count.p, 0, 8, st));
  GSC_TRY(launch_count_failed(st, ctx->ini_tries.as<int32_t>(), n,
                              ctx->ini_count.as<unsigned long long>()));
  const uint64_t failed = read_u64(ctx, ctx->ini_count.as<uint64_t>());
  if (failed) {
    char buf[200];
    snprintf(buf, sizeof(buf), "%llu of %lld points found no interaction in %d rays (is the volume "
             "transparent under its transfer function?)", (unsigned long long)failed, (long long)n,
             kInitMaxAttempts);
    ctx->err = buf;
    throw Fail{GSC_E_INVALID_ARG};
  }
}

void run_knn_mean3(gsc_ctx* ctx, const float* pos, int64_t n, float* mean3) {
  const int G = init_grid_side(n);
  const int64_t cells = (int64_t)G * G * G;
  const Alloc& a = ctx->alloc;
  need(ctx, ctx->ini_key, a, 4 * (size_t)n, "grid keys");
  need(ctx, ctx->ini_id, a, 4 * (size_t)n, "grid ids");
  need(ctx, ctx->ini_key_tmp, a, 4 * (size_t)n, "grid keys (sort)");
  need(ctx, ctx->ini_id_tmp, a, 4 * (size_t)n, "grid ids (sort)");
  need(ctx, ctx->ini_start, a, 4 * (size_t)cells, "cell starts");
  need(ctx, ctx->ini_end, a, 4 * (size_t)cells, "cell ends");
  need(ctx, ctx->ini_spos, a, 16 * (size_t)n, "sorted points");
  const int64_t seg_n[1] = {n}, seg_off[1] = {0};
  const int nb = sort_count_blocks(seg_n, 1);
  const size_t tab = sort_table_bytes(nb, 1);
  std::vector<char> host(tab, 0);
  sort_fill_table(host.data(), seg_n, seg_off, 1);
  need(ctx, ctx->ini_sort_tab, a, tab, "sort table");
  upload(ctx, ctx->ini_sort_tab.p, host.data(), tab);
  need(ctx, ctx->ini_hist, a, 4 * sort_hist_words(std::max(nb, 1), 1), "sort histograms");
  hipStream_t st = ctx->stream;
  GSC_TRY(launch_grid_keys(st, pos, n, G, ctx->ini_key.as<uint32_t>(), ctx->ini_id.as<uint32_t>()));
  GSC_TRY(launch_segmented_sort(st, ctx->ini_sort_tab.p, nb, 1, ctx->ini_key.as<uint32_t>(),
                                ctx->ini_id.as<uint32_t>(), ctx->ini_key_tmp.as<uint32_t>(),
                                ctx->ini_id_tmp.as<uint32_t>(), ctx->ini_hist.as<uint32_t>()));
  GSC_TRY(hipMemsetAsync(ctx->ini_start.p, 0, 4 * (size_t)cells, st));
  GSC_TRY(hipMemsetAsync(ctx->ini_end.p, 0, 4 * (size_t)cells, st));
  GSC_TRY(launch_cell_ranges(st, ctx->ini_key.as<uint32_t>(), ctx->ini_id.as<uint32_t>(), pos, n,
                             ctx->ini_start.as<uint32_t>(), ctx->ini_end.as<uint32_t>(),
                             ctx->ini_spos.as<float4>()));
  GSC_TRY(launch_knn3(st, ctx->ini_spos.as<float4>(), ctx->ini_id.as<uint32_t>(), n, G,
                      ctx->ini_start.as<uint32_t>(), ctx->ini_end.as<uint32_t>(), mean3));
}

}  // namespace

extern "C" {

gsc_status gsc_init_points(gsc_ctx* ctx, const gsc_volume* vol, int64_t n, uint64_t seed, float* pos,
                           float* albedo) {
  return guarded(ctx, [&]() -> gsc_status {
    check_init_volume(ctx, vol);
    if (n < 1 || n > ((int64_t)1 << 31)) invalid(ctx, "n must be in [1, 2^31]");
    if (!pos || !albedo) invalid(ctx, "pos / albedo is NULL");
    run_init_points(ctx, vol, n, seed, pos, albedo);
    return GSC_OK;
  });
}

gsc_status gsc_knn_mean3(gsc_ctx* ctx, const float* pos, int64_t n, float* mean3) {
  return guarded(ctx, [&]() -> gsc_status {
    if (n < 4 || n > ((int64_t)1 << 31)) invalid(ctx, "n must be in [4, 2^31]");
    if (!pos || !mean3) invalid(ctx, "pos / mean3 is NULL");
    run_knn_mean3(ctx, pos, n, mean3);
    return GSC_OK;
  });
}

gsc_status gsc_cache_init(gsc_ctx* ctx, const gsc_volume* vol, int64_t n, int32_t K, uint64_t seed,
                          const gsc_level_buffers* levels) {
  return guarded(ctx, [&]() -> gsc_status {
    check_init_volume(ctx, vol);
    if (K < 1 || K > 8) invalid(ctx, "K must be in [1, 8]");
    if (n > ((int64_t)1 << 31)) invalid(ctx, "n must be <= 2^31");
    if ((n >> (K - 1)) < 4) invalid(ctx, "every level needs at least 4 points (n >> (K - 1) >= 4)");
    if (!levels) invalid(ctx, "levels is NULL");
    for (int l = 0; l < K; ++l) {
      const gsc_level_buffers& g = levels[l];
      if (g.n != (n >> l)) invalid(ctx, "levels[l].n must be n >> l");
      if (!g.pos || !g.rot || !g.log_scale || !g.rgb || !g.opacity_logit) invalid(ctx, "level pointer is NULL");
    }
    const Alloc& a = ctx->alloc;
    need(ctx, ctx->ini_pos, a, 12 * (size_t)n, "init points");
    need(ctx, ctx->ini_alb, a, 12 * (size_t)n, "init albedo");
    need(ctx, ctx->ini_mean3, a, 4 * (size_t)n, "init neighbour distances");
    need(ctx, ctx->ini_partial, a, 8 * init_partial_doubles(), "init moments");
    run_init_points(ctx, vol, n, seed, ctx->ini_pos.as<float>(), ctx->ini_alb.as<float>());
    const float logit = (float)std::log(0.1 / 0.9);
    for (int l = 0; l < K; ++l) {
      const int64_t nl = n >> l;   // level l: the first n / 2^l points
      run_knn_mean3(ctx, ctx->ini_pos.as<float>(), nl, ctx->ini_mean3.as<float>());
      const gsc_level_buffers& g = levels[l];
      GSC_TRY(launch_init_level(ctx->stream, ctx->ini_mean3.as<float>(), nl, ctx->ini_pos.as<float>(),
                                ctx->ini_alb.as<float>(), logit, ctx->ini_partial.as<double>(),
                                g.pos, g.rot, g.log_scale, g.rgb, g.opacity_logit));
    }
    return GSC_OK;
  });
}

gsc_status gsc_ctx_profile(gsc_ctx* ctx, int32_t on) {
  return guarded(ctx, [&]() -> gsc_status {
    prof_resolve(ctx);
    ctx->prof_on = on != 0;
    if (on) {
      for (int i = 0; i < 16; ++i) { ctx->prof_ms[i] = 0.0; ctx->prof_n[i] = 0; }
      ctx->acc_instances = 0;
      ctx->acc_frames = 0;
      need(ctx, ctx->d_stats, ctx->alloc, kStatWords * 8, "splat counters");
      GSC_TRY(hipMemsetAsync(ctx->d_stats.p, 0, kStatWords * 8, ctx->stream));
    }
    return GSC_OK;
  });
}

gsc_status gsc_ctx_profile_read(gsc_ctx* ctx, int32_t index, char* name, size_t name_len,
                                double* total_ms, int64_t* launches) {
  return guarded(ctx, [&]() -> gsc_status {
    if (index < 0 || index >= kProfCount || !name || name_len < 2 || !total_ms || !launches)
      invalid(ctx, "bad profile query");
    prof_resolve(ctx);
    std::snprintf(name, name_len, "%s", kProfNames[index]);
    *total_ms = ctx->prof_ms[index];
    *launches = ctx->prof_n[index];
    return GSC_OK;
  });
}

gsc_status gsc_ctx_counters(gsc_ctx* ctx, gsc_counters* out) {
  return guarded(ctx, [&]() -> gsc_status {
    if (!out) invalid(ctx, "NULL argument");
    uint64_t d[kStatWords] = {};
    if (ctx->d_stats.p) {
      GSC_TRY(hipMemcpyAsync(ctx->host_u64, ctx->d_stats.p, sizeof(d), hipMemcpyDeviceToHost, ctx->stream));
      GSC_TRY(hipStreamSynchronize(ctx->stream));
      std::memcpy(d, ctx->host_u64, sizeof(d));
    }
    out->instances = ctx->acc_instances;
    out->binnings = ctx->acc_frames;
    out->frame_retries = ctx->acc_retries;
    out->evaluations = d[0];
    out->blended = d[1];
    out->contributors = d[2];
    out->tile_entries = d[3];
    out->fwd_tested = d[4];
    out->fwd_slots = d[5];
    out->bwd_tested = d[6];
    out->bwd_blended = d[7];
    out->bwd_slots = d[8];
    out->bwd_entries = d[9];
    out->bwd_atomics = d[10];
    out->bwd_records = d[11];
    return GSC_OK;
  });
}

gsc_status gsc_copy(gsc_ctx* ctx, void* dst, const void* src, size_t bytes) {
  return guarded(ctx, [&]() -> gsc_status {
    if (bytes == 0) return GSC_OK;
    if (!dst || !src) invalid(ctx, "NULL pointer");
    GSC_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, ctx->stream));
    return GSC_OK;
  });
}


gsc_status gsc_probe_gather(gsc_ctx* ctx, const void* cells, uint64_t n_cells, uint32_t threads,
                            int32_t per_thread, float* out, double* ms) {
  return guarded(ctx, [&]() -> gsc_status {
    if (!cells || !out || !ms) invalid(ctx, "NULL argument");
    if (n_cells == 0) invalid(ctx, "n_cells must be >= 1");
    check_probe_threads(ctx, threads, per_thread);
    if (per_thread % 8 != 0) invalid(ctx, "per_thread must be a multiple of 8");
    return timed_probe(ctx, ms, [&]() {
      return launch_probe_gather(ctx->stream, (const float4*)cells, n_cells, threads, per_thread, out);
    });
  });
}

gsc_status gsc_probe_atomics(gsc_ctx* ctx, float* buf, uint64_t n, uint32_t threads,
                             int32_t per_thread, double* ms) {
  return guarded(ctx, [&]() -> gsc_status {
    if (!buf || !ms) invalid(ctx, "NULL argument");
    if (n == 0) invalid(ctx, "n must be >= 1");
    check_probe_threads(ctx, threads, per_thread);
    return timed_probe(ctx, ms, [&]() {
      return launch_probe_atomic(ctx->stream, buf, n, threads, per_thread);
    });
  });
}

gsc_status gsc_probe_valu(gsc_ctx* ctx, float* out, uint32_t threads, int32_t iters, int32_t mode,
                          double* ms) {
  return guarded(ctx, [&]() -> gsc_status {
    if (!out || !ms) invalid(ctx, "NULL argument");
    if (mode != 0 && mode != 1) invalid(ctx, "mode must be 0 (fma) or 1 (exp)");
    check_probe_threads(ctx, threads, iters);
    return timed_probe(ctx, ms, [&]() { return launch_probe_valu(ctx->stream, out, threads, iters, mode); });
  });
}

gsc_status gsc_debug_selftest(gsc_ctx* ctx) {
#ifdef GSC_DEBUG
  return guarded(ctx, [&]() -> gsc_status {
    GSC_TRY(launch_debug_selftest(ctx->stream));
    return GSC_OK;
  });
#else
  if (!ctx) return GSC_E_INVALID_ARG;
  ctx->err = "not a debug build (GSC_DEBUG)";
  return GSC_E_UNSUPPORTED;
#endif
}

gsc_status gsc_ctx_synchronize(gsc_ctx* ctx) {
  return guarded(ctx, [&]() -> gsc_status {
    GSC_TRY(hipStreamSynchronize(ctx->stream));
    return GSC_OK;
  });
}

size_t gsc_abi_struct_size(int32_t which) {
  switch (which) {
    case 0: return sizeof(gsc_camera);
    case 1: return sizeof(gsc_gaussians);
    case 2: return sizeof(gsc_grads);
    case 3: return sizeof(gsc_volume);
    case 4: return sizeof(gsc_trace_params);
    case 5: return sizeof(gsc_path_record);
    case 6: return sizeof(gsc_frame_stats);
    case 7: return sizeof(gsc_binning_info);
    case 8: return sizeof(gsc_adam_hparams);
    case 9: return sizeof(gsc_frame_request);
    case 10: return sizeof(gsc_allocator);
    case 11: return sizeof(gsc_counters);
    case 12: return sizeof(gsc_level_buffers);
    default: return 0;
  }
}

}  // extern "C"
