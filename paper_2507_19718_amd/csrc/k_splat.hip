// k_splat.hip -- front-to-back alpha blending of the binned Gaussians (the cache images) and
// its adjoint (3D Gaussian splatting's tile rasteriser, adapted by GSCache to render each cache
// level; Method: "A Path Space Radiance Cache", "Cache Training").
//
// One 256-lane workgroup per 16x16 tile of one segment, one lane per pixel.  The tile's list
// is consumed in batches of 256 records staged in LDS (48 B each); every lane then walks the
// batch with broadcast LDS reads.  The forward stops when every pixel of the tile is saturated.
// The adjoint walks the same lists back to front from each pixel's last contributor, recovers
// the transmittance before each Gaussian by dividing the stored final transmittance by
// (1 - alpha), reduces each Gaussian's nine screen-space gradients across the wavefront with
// cross-lane shuffles and across the workgroup in LDS, and issues at most nine float atomics per
// (tile, Gaussian).
#include "gsc_dev.h"

namespace gsc {

namespace {

constexpr int kSplatThreads = kTile * kTile;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTmin = 1e-4f;

struct TileCtx {
  int64_t start, end;
  int64_t g_off, pix_off;
  float fi, fj;
  int64_t pix;           // pixel index within the segment image
  bool inside;
};

__device__ __forceinline__ TileCtx tile_setup(const Seg* __restrict__ segs,
                                              const int64_t* __restrict__ seg_tstart, int S,
                                              const DevCam* __restrict__ cams,
                                              const uint64_t* __restrict__ ranges, int64_t t,
                                              int* seg_out) {
  const int s = find_segment(seg_tstart, S, t);
  *seg_out = s;
  const Seg& sg = segs[s];
  const DevCam& cam = cams[sg.cam];
  const int64_t lt = t - sg.tile_base;
  const int tx = (int)(lt % sg.TX), ty = (int)(lt / sg.TX);
  const int lx = threadIdx.x & (kTile - 1), ly = threadIdx.x >> 4;
  const int px = tx * kTile + lx, py = ty * kTile + ly;
  TileCtx c;
  c.start = (int64_t)ranges[2 * t];
  c.end = (int64_t)ranges[2 * t + 1];
  c.g_off = sg.g_off;
  c.pix_off = sg.pix_off;
  c.inside = (px < cam.w) && (py < cam.h);
  c.pix = (int64_t)py * cam.w + px;
  c.fi = (float)(cam.x0 + px);
  c.fj = (float)(cam.y0 + py);
  return c;
}

__global__ void __launch_bounds__(kSplatThreads) splat_forward_kernel(
    const Seg* __restrict__ segs, const int64_t* __restrict__ seg_tstart, int S,
    const DevCam* __restrict__ cams, const uint64_t* __restrict__ ranges,
    const uint32_t* __restrict__ values, const SplatRec* __restrict__ rec,
    float* __restrict__ images, float* __restrict__ final_T, int32_t* __restrict__ last_id,
    uint32_t* __restrict__ n_contrib) {
  __shared__ float4 sh0[kSplatThreads], sh1[kSplatThreads], sh2[kSplatThreads];
  const int64_t t = blockIdx.x;
  int s;
  const TileCtx tc = tile_setup(segs, seg_tstart, S, cams, ranges, t, &s);
  const int tid = threadIdx.x;
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  int32_t last = -1;
  uint32_t nc = 0u;
  bool done = !tc.inside;
  for (int64_t bs = tc.start; bs < tc.end; bs += kSplatThreads) {
    if (__syncthreads_and(done)) break;
    const int64_t idx = bs + tid;
    if (idx < tc.end) {
      const SplatRec r = rec[tc.g_off + values[idx]];
      sh0[tid] = r.q0;
      sh1[tid] = r.q1;
      sh2[tid] = r.q2;
    }
    __syncthreads();
    const int n = (int)((tc.end - bs) < kSplatThreads ? (tc.end - bs) : kSplatThreads);
    if (!done) {
      for (int k = 0; k < n; ++k) {
        const float4 q2 = sh2[k];
        const uint32_t wx = __float_as_uint(q2.y), wy = __float_as_uint(q2.z);
        const float fx0 = (float)(wx & 0xffffu), fx1 = (float)(wx >> 16);
        const float fy0 = (float)(wy & 0xffffu), fy1 = (float)(wy >> 16);
        if (tc.fi < fx0 || tc.fi > fx1 || tc.fj < fy0 || tc.fj > fy1) continue;
        const float4 q0 = sh0[k];
        const float4 q1 = sh1[k];
        const float dx = q0.x - tc.fi, dy = q0.y - tc.fj;
        const float power = -0.5f * ((q0.z * dx) * dx + (q1.x * dy) * dy) - (q0.w * dx) * dy;
        if (power > 0.0f) continue;
        const float alpha = fminf(kAlphaMax, q1.y * __expf(power));
        if (alpha < kAlphaMin) continue;
        const float Tn = T * (1.0f - alpha);
        if (Tn < kTmin) { done = true; break; }
        const float w = alpha * T;
        C0 = C0 + q1.z * w;
        C1 = C1 + q1.w * w;
        C2 = C2 + q2.x * w;
        T = Tn;
        last = (int32_t)__float_as_uint(q2.w);
        nc = (uint32_t)(bs - tc.start + k + 1);
      }
    }
    __syncthreads();
  }
  if (tc.inside) {
    const int64_t p = tc.pix_off + tc.pix;
    images[3 * p + 0] = C0;
    images[3 * p + 1] = C1;
    images[3 * p + 2] = C2;
    final_T[p] = T;
    last_id[p] = last;
    n_contrib[p] = nc;
  }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void __launch_bounds__(kSplatThreads) splat_backward_kernel(
    const Seg* __restrict__ segs, const int64_t* __restrict__ seg_tstart, int S,
    const DevCam* __restrict__ cams, const uint64_t* __restrict__ ranges,
    const uint32_t* __restrict__ values, const SplatRec* __restrict__ rec,
    const float* __restrict__ final_T, const uint32_t* __restrict__ n_contrib,
    const float* __restrict__ dL_dimages, float* __restrict__ grad2d, int64_t G) {
  __shared__ float4 sh0[kSplatThreads], sh1[kSplatThreads], sh2[kSplatThreads];
  __shared__ float shg[9][kSplatThreads];
  __shared__ uint32_t sh_max;
  const int64_t t = blockIdx.x;
  int s;
  const TileCtx tc = tile_setup(segs, seg_tstart, S, cams, ranges, t, &s);
  const int tid = threadIdx.x;
  const int lane = __lane_id();
  float T = 1.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
  uint32_t nc = 0u;
  if (tc.inside) {
    const int64_t p = tc.pix_off + tc.pix;
    T = final_T[p];
    nc = n_contrib[p];
    g0 = dL_dimages[3 * p + 0];
    g1 = dL_dimages[3 * p + 1];
    g2 = dL_dimages[3 * p + 2];
  }
  if (tid == 0) sh_max = 0u;
  __syncthreads();
  if (nc) atomicMax(&sh_max, nc);
  __syncthreads();
  const int64_t stop = tc.start + (int64_t)sh_max;
  float B0 = 0.0f, B1 = 0.0f, B2 = 0.0f;       // colour accumulated behind
  for (int64_t be = stop; be > tc.start; be -= kSplatThreads) {
    const int64_t bs = (be - kSplatThreads) > tc.start ? (be - kSplatThreads) : tc.start;
    const int n = (int)(be - bs);
    if (tid < n) {
      const SplatRec r = rec[tc.g_off + values[bs + tid]];
      sh0[tid] = r.q0;
      sh1[tid] = r.q1;
      sh2[tid] = r.q2;
    }
#pragma unroll
    for (int v = 0; v < 9; ++v) shg[v][tid] = 0.0f;
    __syncthreads();
    for (int k = n - 1; k >= 0; --k) {
      const int64_t rel = bs + k - tc.start;
      bool hit = tc.inside && rel < (int64_t)nc;
      const float4 q0 = sh0[k];
      const float4 q1 = sh1[k];
      const float4 q2 = sh2[k];
      float dx = 0.0f, dy = 0.0f, e = 0.0f, oe = 0.0f, alpha = 0.0f;
      if (hit) {
        const uint32_t wx = __float_as_uint(q2.y), wy = __float_as_uint(q2.z);
        hit = !(tc.fi < (float)(wx & 0xffffu) || tc.fi > (float)(wx >> 16) ||
                tc.fj < (float)(wy & 0xffffu) || tc.fj > (float)(wy >> 16));
      }
      if (hit) {
        dx = q0.x - tc.fi;
        dy = q0.y - tc.fj;
        const float power = -0.5f * ((q0.z * dx) * dx + (q1.x * dy) * dy) - (q0.w * dx) * dy;
        hit = !(power > 0.0f);
        if (hit) {
          e = __expf(power);
          oe = q1.y * e;
          alpha = fminf(kAlphaMax, oe);
          hit = !(alpha < kAlphaMin);
        }
      }
      float gu = 0.0f, gv = 0.0f, gA = 0.0f, gB = 0.0f, gC = 0.0f, go = 0.0f;
      float gr = 0.0f, gg = 0.0f, gb = 0.0f;
      if (hit) {
        T = T / (1.0f - alpha);
        const float w = alpha * T;
        gr = w * g0;
        gg = w * g1;
        gb = w * g2;
        const float dalpha = T * (((q1.z - B0) * g0 + (q1.w - B1) * g1) + (q2.x - B2) * g2);
        B0 = alpha * q1.z + (1.0f - alpha) * B0;
        B1 = alpha * q1.w + (1.0f - alpha) * B1;
        B2 = alpha * q2.x + (1.0f - alpha) * B2;
        if (!(oe > kAlphaMax)) {
          const float dpow = dalpha * alpha;
          go = dalpha * e;
          gA = -0.5f * dx * dx * dpow;
          gC = -0.5f * dy * dy * dpow;
          gB = -dx * dy * dpow;
          gu = (-q0.z * dx - q0.w * dy) * dpow;
          gv = (-q1.x * dy - q0.w * dx) * dpow;
        }
      }
      if (__ballot(hit) != 0ull) {
        gu = wave_sum(gu); gv = wave_sum(gv); gA = wave_sum(gA);
        gB = wave_sum(gB); gC = wave_sum(gC); go = wave_sum(go);
        gr = wave_sum(gr); gg = wave_sum(gg); gb = wave_sum(gb);
        if (lane == 0) {
          atomicAdd(&shg[0][k], gu); atomicAdd(&shg[1][k], gv); atomicAdd(&shg[2][k], gA);
          atomicAdd(&shg[3][k], gB); atomicAdd(&shg[4][k], gC); atomicAdd(&shg[5][k], go);
          atomicAdd(&shg[6][k], gr); atomicAdd(&shg[7][k], gg); atomicAdd(&shg[8][k], gb);
        }
      }
    }
    __syncthreads();
    if (tid < n) {
      const int64_t gi = tc.g_off + (int64_t)__float_as_uint(sh2[tid].w);
#pragma unroll
      for (int v = 0; v < 9; ++v) {
        const float val = shg[v][tid];
        if (val != 0.0f) unsafeAtomicAdd(&grad2d[(int64_t)v * G + gi], val);
      }
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_splat_forward(hipStream_t st, const Seg* segs, const int64_t* seg_tstart, int S,
                                const DevCam* cams, int64_t n_tiles, const uint64_t* ranges,
                                const uint32_t* values, const SplatRec* rec, float* images,
                                float* final_T, int32_t* last_id, uint32_t* n_contrib) {
  if (n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(splat_forward_kernel, dim3((unsigned)n_tiles), dim3(kSplatThreads), 0, st,
                     segs, seg_tstart, S, cams, ranges, values, rec, images, final_T, last_id,
                     n_contrib);
  return hipGetLastError();
}

hipError_t launch_splat_backward(hipStream_t st, const Seg* segs, const int64_t* seg_tstart, int S,
                                 const DevCam* cams, int64_t n_tiles, const uint64_t* ranges,
                                 const uint32_t* values, const SplatRec* rec, const float* final_T,
                                 const uint32_t* n_contrib, const float* dL_dimages,
                                 float* grad2d, int64_t G, int deterministic) {
  (void)deterministic;
  if (n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(splat_backward_kernel, dim3((unsigned)n_tiles), dim3(kSplatThreads), 0, st,
                     segs, seg_tstart, S, cams, ranges, values, rec, final_T, n_contrib,
                     dL_dimages, grad2d, G);
  return hipGetLastError();
}

}  // namespace gsc
