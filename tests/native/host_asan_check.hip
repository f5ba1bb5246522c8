// host_asan_check.hip -- drives the C ABI of libgsc through its host code paths, built with
// AddressSanitizer on the host side only (the device code is built as in the library), so that a
// heap overflow, use after free or stack overflow in the runtime's host code (argument checks,
// tables, staging buffers, checkpoint files, the allocator hook, object lifetimes) stops the run
// with a report.  Exit status 0 and the line "host asan check ok" when every call behaved.
//
// The scene is small and synthetic: a 16^3 density field in the unit cube, a 4-point transfer
// function, one point light (then a sphere light), two cache levels from gsc_cache_init, and a
// 64x48 camera looking at the cube.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <unistd.h>
#include <string>
#include <vector>

#include "../../include/gsc.h"

namespace {

int g_failures = 0;

#define CHECK(cond)                                                                  \
  do {                                                                               \
    if (!(cond)) {                                                                   \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);        \
      ++g_failures;                                                                  \
    }                                                                                \
  } while (0)

#define OK(call)                                                                     \
  do {                                                                               \
    const gsc_status st_ = (call);                                                   \
    if (st_ != GSC_OK) {                                                             \
      std::fprintf(stderr, "line %d: %s -> %d\n", __LINE__, #call, (int)st_);        \
      ++g_failures;                                                                  \
    }                                                                                \
  } while (0)

template <typename T>
T* dalloc(size_t n) {
  void* p = nullptr;
  if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) {
    std::fprintf(stderr, "hipMalloc of %zu bytes failed\n", n * sizeof(T));
    std::exit(2);
  }
  return static_cast<T*>(p);
}

// Counting allocator hook: every block the library takes through it must come back.
struct Pool {
  long live = 0;
  long calls = 0;
};

void* pool_alloc(size_t bytes, void* user) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) return nullptr;
  static_cast<Pool*>(user)->live++;
  static_cast<Pool*>(user)->calls++;
  return p;
}

void pool_release(void* p, void* user) {
  if (!p) return;
  (void)hipFree(p);
  static_cast<Pool*>(user)->live--;
}

gsc_camera make_camera(int w, int h, float dz) {
  gsc_camera c;
  std::memset(&c, 0, sizeof(c));
  c.R[0] = c.R[4] = c.R[8] = 1.0f;            // axes aligned: x right, y down, z forward
  c.t[0] = -0.5f;
  c.t[1] = -0.5f;
  c.t[2] = dz;                                // the cube's centre at depth dz + 0.5
  c.fx = c.fy = 1.2f * (float)w;
  c.cx = 0.5f * (float)w;
  c.cy = 0.5f * (float)h;
  c.full_w = w;
  c.full_h = h;
  c.x0 = 0;
  c.y0 = 0;
  c.w = w;
  c.h = h;
  c.znear = 0.2f;
  return c;
}

gsc_frame_request make_request(const gsc_camera& cam, uint32_t frame, int K) {
  gsc_frame_request r;
  std::memset(&r, 0, sizeof(r));
  r.cam = cam;
  r.trace.seed = 0x1234abcdull;
  r.trace.frame = frame;
  r.trace.spp = 1;
  r.trace.max_bounces = 3;
  r.trace.num_levels = (uint32_t)K;
  r.trace.C = 0.5f;
  r.trace.C_inf = 0;
  r.trace.eps = 0.0f;
  r.trace.strategy = GSC_STRATEGY_NEE;
  r.loss = 1;
  r.train = 1;
  r.viewport_frames = frame + 1;
  const double lr[5] = {1e-3, 1e-3, 5e-3, 1e-2, 5e-2};
  for (int i = 0; i < 5; ++i) r.lr[i] = lr[i];
  r.beta1 = 0.9;
  r.beta2 = 0.999;
  r.eps = 1e-15;
  r.weight_decay = 1e-2;
  return r;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc > 1 && std::strcmp(argv[1], "--planted-overflow") == 0) {
    // Shows the instrumentation is live, before any HIP call (runs without a GPU): one write
    // past the end of a heap block, which AddressSanitizer must report.
    std::vector<int> v(8);
    int* volatile p = v.data();
    p[8] = 1;
    std::printf("planted overflow not reported\n");
    return 0;
  }
  const int N = 16, K = 2;
  const int64_t n0 = 1024;
  // Density field and optics (HOST arrays for the TF and lights, as the ABI takes them).
  std::vector<float> dens((size_t)N * N * N);
  for (int z = 0; z < N; ++z)
    for (int y = 0; y < N; ++y)
      for (int x = 0; x < N; ++x)
        dens[((size_t)z * N + y) * N + x] =
            0.5f + 0.4f * std::sin(0.7f * x) * std::cos(0.5f * y) * std::sin(0.3f * z + 1.0f);
  float* d_dens = dalloc<float>(dens.size());
  (void)hipMemcpy(d_dens, dens.data(), dens.size() * sizeof(float), hipMemcpyHostToDevice);
  const float tf[16] = {0.9f, 0.8f, 0.7f, 0.0f,  0.8f, 0.6f, 0.5f, 2.0f,
                        0.6f, 0.7f, 0.9f, 6.0f,  0.9f, 0.9f, 0.9f, 10.0f};
  const float light[6] = {2.0f, -1.0f, -1.5f, 8.0f, 8.0f, 8.0f};
  gsc_volume vol;
  std::memset(&vol, 0, sizeof(vol));
  vol.density = d_dens;
  vol.nx = vol.ny = vol.nz = N;
  vol.density_max = 0.9f;
  vol.tf_rgba = tf;
  vol.tf_points = 4;
  vol.lights = light;
  vol.n_lights = 1;

  Pool pool;
  gsc_allocator alloc = {pool_alloc, pool_release, &pool};
  gsc_ctx* ctx = nullptr;
  OK(gsc_ctx_create(0, nullptr, &alloc, &ctx));
  if (!ctx) return 1;

  // Cache initialisation into caller-owned level buffers.
  std::vector<gsc_level_buffers> lb(K);
  std::vector<gsc_gaussians> lv(K);
  std::vector<float*> owned;
  for (int l = 0; l < K; ++l) {
    const int64_t n = n0 >> l;
    lb[l].pos = dalloc<float>(3 * n);
    lb[l].rot = dalloc<float>(4 * n);
    lb[l].log_scale = dalloc<float>(3 * n);
    lb[l].rgb = dalloc<float>(3 * n);
    lb[l].opacity_logit = dalloc<float>(n);
    lb[l].n = n;
    owned.insert(owned.end(), {lb[l].pos, lb[l].rot, lb[l].log_scale, lb[l].rgb, lb[l].opacity_logit});
    lv[l] = {lb[l].pos, lb[l].rot, lb[l].log_scale, lb[l].rgb, lb[l].opacity_logit, n};
  }
  OK(gsc_cache_init(ctx, &vol, n0, K, 7, lb.data()));
  OK(gsc_ctx_synchronize(ctx));

  gsc_scene* scene = nullptr;
  gsc_scene* scene2 = nullptr;
  OK(gsc_scene_create(ctx, &vol, lv.data(), K, &scene));
  OK(gsc_scene_create(ctx, &vol, lv.data(), K, &scene2));
  CHECK(gsc_scene_footprint_bytes(scene) > 0);

  const gsc_camera cam = make_camera(64, 48, 1.5f);
  float* image = dalloc<float>(64 * 48 * 3);
  gsc_frame_stats st;
  uint32_t frame = 0;
  // Frames under each tiling and with the profile and work counters on.
  OK(gsc_ctx_profile(ctx, 1));
  OK(gsc_ctx_set_work_counters(ctx, 1));
  for (int tile : {0, 16, 32}) {
    OK(gsc_ctx_set_frame_tiles(ctx, tile));
    for (int i = 0; i < 3; ++i) {
      const gsc_frame_request req = make_request(cam, frame++, K);
      OK(gsc_render_frame(ctx, scene, &req, image, &st));
      CHECK(std::isfinite(st.loss) && st.instances > 0 && st.adam_skipped == 0);
    }
  }
  OK(gsc_ctx_set_work_counters(ctx, 0));
  for (int i = 0;; ++i) {
    char name[64];
    double ms = 0.0;
    int64_t launches = 0;
    const gsc_status s = gsc_ctx_profile_read(ctx, i, name, sizeof(name), &ms, &launches);
    if (s != GSC_OK) break;
    CHECK(std::strlen(name) < sizeof(name));
  }
  OK(gsc_ctx_profile(ctx, 0));
  gsc_counters cnt;
  OK(gsc_ctx_counters(ctx, &cnt));

  // A camera twice as close: more instances than the previous frame sized for (the retry path).
  {
    const gsc_camera nearcam = make_camera(64, 48, 0.4f);
    const gsc_frame_request req = make_request(nearcam, frame++, K);
    OK(gsc_render_frame(ctx, scene, &req, image, &st));
  }
  // Deterministic adjoint, a render-only frame, and a batch over two scenes with a cropped view.
  OK(gsc_ctx_set_deterministic(ctx, 1));
  {
    gsc_frame_request req = make_request(cam, frame++, K);
    OK(gsc_render_frame(ctx, scene, &req, image, nullptr));
    req.train = 0;
    OK(gsc_render_frame(ctx, scene, &req, image, &st));
  }
  OK(gsc_ctx_set_deterministic(ctx, 0));
  {
    gsc_camera crop = cam;
    crop.x0 = 8;
    crop.y0 = 4;
    crop.w = 40;
    crop.h = 30;
    float* image2 = dalloc<float>(40 * 30 * 3);
    gsc_scene* scenes[2] = {scene, scene2};
    gsc_frame_request reqs[2] = {make_request(cam, frame, K), make_request(crop, frame, K)};
    float* images[2] = {image, image2};
    gsc_frame_stats sts[2];
    OK(gsc_render_frames(ctx, scenes, reqs, images, 2, sts));
    ++frame;
    (void)hipFree(image2);
  }

  // The separate hot-path calls on the scene's current levels.
  {
    std::vector<gsc_gaussians> cur(K);
    for (int l = 0; l < K; ++l) OK(gsc_scene_level(scene, l, &cur[l]));
    OK(gsc_ctx_set_frame_binning(ctx, 1));
    gsc_binning* bin = nullptr;
    OK(gsc_project_bin(ctx, cur.data(), K, &cam, 0, &bin));
    gsc_binning_info info;
    OK(gsc_binning_view(ctx, bin, &info));
    CHECK(info.num_levels == K && info.n_instances > 0);
    uint64_t* keys = dalloc<uint64_t>(info.n_instances);
    OK(gsc_binning_keys(ctx, bin, keys));
    const size_t px = (size_t)cam.w * cam.h;
    float* imgs = dalloc<float>(K * px * 3);
    float* T = dalloc<float>(K * px);
    int32_t* last = dalloc<int32_t>(K * px);
    float* dimg = dalloc<float>(K * px * 3);
    (void)hipMemset(dimg, 0, K * px * 3 * sizeof(float));
    OK(gsc_splat_forward(ctx, bin, imgs, T, last));
    std::vector<gsc_grads> gr(K);
    for (int l = 0; l < K; ++l) {
      const int64_t n = cur[l].n;
      gr[l] = {dalloc<float>(3 * n), dalloc<float>(4 * n), dalloc<float>(3 * n),
               dalloc<float>(3 * n), dalloc<float>(n)};
    }
    OK(gsc_splat_backward(ctx, bin, cur.data(), K, &cam, T, last, dimg, gr.data()));
    OK(gsc_splat_backward_noalloc(ctx, bin, cur.data(), K, &cam, T, last, dimg, gr.data()));
    // A capacity hint far too small: GSC_E_CAPACITY and the count needed.
    gsc_binning* small = nullptr;
    CHECK(gsc_project_bin(ctx, cur.data(), K, &cam, 1, &small) == GSC_E_CAPACITY);
    CHECK(gsc_ctx_required_capacity(ctx) == info.n_instances);
    gsc_binning_release(ctx, bin);
    OK(gsc_ctx_set_frame_binning(ctx, 0));
    for (auto& g : gr) {
      for (float* p : {g.pos, g.rot, g.log_scale, g.rgb, g.opacity_logit}) (void)hipFree(p);
    }
    for (void* p : {(void*)keys, (void*)imgs, (void*)T, (void*)last, (void*)dimg}) (void)hipFree(p);
  }

  // Tracer alone, with path records and several samples per pixel.
  {
    gsc_trace_params tp = make_request(cam, frame, K).trace;
    tp.spp = 3;
    const size_t px = (size_t)cam.w * cam.h;
    float* targets = dalloc<float>(K * px * 3);
    gsc_path_record* rec = dalloc<gsc_path_record>(3 * px);
    OK(gsc_trace_targets(ctx, &vol, &cam, &tp, targets, rec, &st));
    (void)hipFree(targets);
    (void)hipFree(rec);
  }

  // Checkpoint round trip, optics change, state copy.
  {
    char path[] = "/tmp/gsc_asan_ckptXXXXXX";
    const int fd = mkstemp(path);
    CHECK(fd >= 0);
    if (fd >= 0) close(fd);
    OK(gsc_scene_save(ctx, scene, path));
    OK(gsc_scene_load(ctx, scene2, path));
    std::remove(path);
    CHECK(gsc_scene_load(ctx, scene2, "/tmp/gsc_asan_no_such_file") != GSC_OK);
    const float sphere[7] = {1.6f, 0.5f, 0.5f, 0.1f, 20.0f, 20.0f, 20.0f};
    OK(gsc_scene_set_optics(ctx, scene, tf, 4, nullptr, 0, sphere, 1));
    OK(gsc_scene_copy_state(ctx, scene2, scene));
    const gsc_frame_request req = make_request(cam, frame++, K);
    OK(gsc_render_frame(ctx, scene, &req, image, &st));
  }

  // Argument errors: each is refused before anything is enqueued, with a message.
  {
    const gsc_frame_request req = make_request(cam, frame, K);
    CHECK(gsc_render_frame(ctx, nullptr, &req, image, nullptr) == GSC_E_INVALID_ARG);
    CHECK(gsc_render_frame(ctx, scene, nullptr, image, nullptr) == GSC_E_INVALID_ARG);
    gsc_frame_request bad = req;
    bad.trace.num_levels = 3;
    CHECK(gsc_render_frame(ctx, scene, &bad, image, nullptr) == GSC_E_INVALID_ARG);
    bad = req;
    bad.cam.w = 0;
    CHECK(gsc_render_frame(ctx, scene, &bad, image, nullptr) == GSC_E_INVALID_ARG);
    CHECK(gsc_ctx_set_frame_tiles(ctx, 24) == GSC_E_INVALID_ARG);
    CHECK(gsc_cache_init(ctx, &vol, n0 + 1, K, 7, lb.data()) == GSC_E_INVALID_ARG);
    gsc_volume badvol = vol;
    badvol.tf_points = 1;
    gsc_scene* none = nullptr;
    CHECK(gsc_scene_create(ctx, &badvol, lv.data(), K, &none) == GSC_E_INVALID_ARG);
    const char* msg = gsc_ctx_last_error(ctx);
    CHECK(msg != nullptr && std::strlen(msg) > 0);
    for (int which = 0; which < 16; ++which) (void)gsc_abi_struct_size(which);
  }

  OK(gsc_ctx_trim(ctx));
  gsc_scene_destroy(ctx, scene2);
  gsc_scene_destroy(ctx, scene);
  gsc_ctx_destroy(ctx);
  CHECK(pool.live == 0 && pool.calls > 0);
  for (float* p : owned) (void)hipFree(p);
  (void)hipFree(image);
  (void)hipFree(d_dens);
  if (g_failures) {
    std::fprintf(stderr, "%d check(s) failed\n", g_failures);
    return 1;
  }
  std::printf("host asan check ok (%ld allocator calls)\n", pool.calls);
  return 0;
}
