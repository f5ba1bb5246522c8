// k_splat.hip -- front-to-back alpha blending of the binned Gaussians (the cache images) and
// its adjoint (3D Gaussian splatting's tile rasteriser, adapted by GSCache to render each cache
// level; Method: "A Path Space Radiance Cache", "Cache Training").
//
// One 64-lane wavefront per 16x16 tile; lane l owns the four pixels (l & 15, (l >> 4) + 4k),
// k = 0..3.  The tile's list is consumed 64 entries at a time: lane j loads entry j's 48-byte
// record into registers, then the wave walks the entries in list order and broadcasts each
// record to scalar registers (v_readlane), so every lane evaluates its four pixels against it
// with scalar operands -- no LDS traffic and no workgroup barriers.  An entry whose alpha >=
// 1/255 ellipse provably misses every pixel of the tile (a conservative test of the quadratic
// form over the tile rectangle) is skipped by the whole wave; such an entry is skipped by every
// pixel anyway, so results do not change.
//
// The adjoint walks the same lists back to front from each pixel's last contributor, recovers
// the transmittance before each Gaussian by dividing the stored final transmittance by
// (1 - alpha), sums each Gaussian's nine screen-space gradients over the lane's four pixels,
// reduces them across the wavefront with DPP row shifts and row broadcasts, and issues nine
// float atomics per (tile, Gaussian) from the lane that loaded the entry.
#include "gsc_dev.h"

namespace gsc {

namespace {

constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTmin = 1e-4f;
constexpr int kPx = 4;

struct Tile {
  int64_t start, end;
  int64_t g_off, pix_off;
  int W;                     // render window width
  float fi;                  // this lane's pixel column (full-frame)
  float fj[kPx];             // this lane's four pixel rows
  int64_t pix[kPx];          // pixel index within the segment image
  bool inside[kPx];
  float ti0, ti1, tj0, tj1;  // the tile's pixel rectangle inside the render window
};

__device__ __forceinline__ Tile tile_setup(const Seg* __restrict__ segs,
                                           const int64_t* __restrict__ seg_tstart, int S,
                                           const DevCam* __restrict__ cams,
                                           const uint64_t* __restrict__ ranges, int64_t t) {
  const int s = find_segment(seg_tstart, S, t);
  const Seg& sg = segs[s];
  const DevCam& cam = cams[sg.cam];
  const int64_t lt = t - sg.tile_base;
  const int tx = (int)(lt % sg.TX), ty = (int)(lt / sg.TX);
  const int lane = __lane_id();
  const int px = tx * kTile + (lane & 15);
  Tile c;
  c.start = (int64_t)ranges[2 * t];
  c.end = (int64_t)ranges[2 * t + 1];
  c.g_off = sg.g_off;
  c.pix_off = sg.pix_off;
  c.W = cam.w;
  c.fi = (float)(cam.x0 + px);
#pragma unroll
  for (int k = 0; k < kPx; ++k) {
    const int py = ty * kTile + (lane >> 4) + 4 * k;
    c.inside[k] = (px < cam.w) && (py < cam.h);
    c.pix[k] = (int64_t)py * cam.w + px;
    c.fj[k] = (float)(cam.y0 + py);
  }
  c.ti0 = (float)(cam.x0 + tx * kTile);
  c.ti1 = (float)(cam.x0 + min(tx * kTile + kTile, cam.w) - 1);
  c.tj0 = (float)(cam.y0 + ty * kTile);
  c.tj1 = (float)(cam.y0 + min(ty * kTile + kTile, cam.h) - 1);
  return c;
}

// Conservative test: can o exp(-Q(u - i, v - j) / 2) reach 1/255 at some pixel (i, j) of the
// tile inside the Gaussian's integer window?  Q is the conic's quadratic form; its minimum over
// a rectangle not containing the centre lies on the boundary.
__device__ __forceinline__ bool may_touch(const float4& q0, const float4& q1, const float4& q2,
                                          const Tile& tc) {
  const uint32_t wx = __float_as_uint(q2.y), wy = __float_as_uint(q2.z);
  const float i0 = fmaxf(tc.ti0, (float)(wx & 0xffffu)), i1 = fminf(tc.ti1, (float)(wx >> 16));
  const float j0 = fmaxf(tc.tj0, (float)(wy & 0xffffu)), j1 = fminf(tc.tj1, (float)(wy >> 16));
  if (i0 > i1 || j0 > j1) return false;
  const float A = q0.z, B = q0.w, C = q1.x;
  const float x0 = q0.x - i1, x1 = q0.x - i0;   // dx = u - i over the rectangle
  const float y0 = q0.y - j1, y1 = q0.y - j0;
  float qmin;
  if (x0 <= 0.0f && x1 >= 0.0f && y0 <= 0.0f && y1 >= 0.0f) {
    qmin = 0.0f;
  } else {
    auto q = [&](float x, float y) { return A * x * x + 2.0f * B * x * y + C * y * y; };
    const float ya = fminf(fmaxf(-B * x0 / C, y0), y1), yb = fminf(fmaxf(-B * x1 / C, y0), y1);
    const float xa = fminf(fmaxf(-B * y0 / A, x0), x1), xb = fminf(fmaxf(-B * y1 / A, x0), x1);
    qmin = fminf(fminf(q(x0, ya), q(x1, yb)), fminf(q(xa, y0), q(xb, y1)));
  }
  // 1e-3 relative slack keeps the test conservative against rounding.
  return q1.y * __expf(-0.5f * qmin) >= kAlphaMin * 0.999f;
}

__device__ __forceinline__ float rl(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

__device__ __forceinline__ uint32_t rlu(float v, int k) {
  return (uint32_t)__builtin_amdgcn_readlane(__float_as_int(v), k);
}

__global__ void __launch_bounds__(64) splat_forward_kernel(
    const Seg* __restrict__ segs, const int64_t* __restrict__ seg_tstart, int S,
    const DevCam* __restrict__ cams, const uint64_t* __restrict__ ranges,
    const uint32_t* __restrict__ values, const SplatRec* __restrict__ rec,
    float* __restrict__ images, float* __restrict__ final_T, int32_t* __restrict__ last_id,
    uint32_t* __restrict__ n_contrib, unsigned long long* __restrict__ evals) {
  const int64_t t = blockIdx.x;
  const Tile tc = tile_setup(segs, seg_tstart, S, cams, ranges, t);
  const int lane = __lane_id();
  float T[kPx], C0[kPx], C1[kPx], C2[kPx];
  uint32_t nc[kPx], stop[kPx];
  bool done[kPx];
#pragma unroll
  for (int k = 0; k < kPx; ++k) {
    T[k] = 1.0f; C0[k] = 0.0f; C1[k] = 0.0f; C2[k] = 0.0f;
    nc[k] = 0u; stop[k] = 0u;
    done[k] = !tc.inside[k];
  }
  const uint32_t len = (uint32_t)(tc.end - tc.start);
  for (int64_t bs = tc.start; bs < tc.end; bs += 64) {
    const bool all = done[0] && done[1] && done[2] && done[3];
    if (__ballot(!all) == 0ull) break;
    const int64_t idx = bs + lane;
    float4 q0 = make_float4(0, 0, 0, 0), q1 = q0, q2 = q0;
    bool keep = false;
    if (idx < tc.end) {
      const SplatRec r = rec[tc.g_off + values[idx]];
      q0 = r.q0; q1 = r.q1; q2 = r.q2;
      keep = may_touch(q0, q1, q2, tc);
    }
    uint64_t mask = __ballot(keep);
    const uint32_t rel0 = (uint32_t)(bs - tc.start);
    while (mask) {
      if (__ballot(!(done[0] && done[1] && done[2] && done[3])) == 0ull) break;
      const int k = __builtin_ctzll(mask);
      mask &= mask - 1ull;
      const float u = rl(q0.x, k), v = rl(q0.y, k), A = rl(q0.z, k), B = rl(q0.w, k);
      const float Cc = rl(q1.x, k), o = rl(q1.y, k);
      const uint32_t wx = rlu(q2.y, k), wy = rlu(q2.z, k);
      const float fx0 = (float)(wx & 0xffffu), fx1 = (float)(wx >> 16);
      const float fy0 = (float)(wy & 0xffffu), fy1 = (float)(wy >> 16);
      const float cr = rl(q1.z, k), cg = rl(q1.w, k), cb = rl(q2.x, k);
      const bool colin = !(tc.fi < fx0 || tc.fi > fx1);
      const float dx = u - tc.fi;
      const float adx = (A * dx) * dx;
      const float bdx = B * dx;
      const uint32_t pos = rel0 + (uint32_t)k + 1u;
#pragma unroll
      for (int p = 0; p < kPx; ++p) {
        if (done[p] || !colin || tc.fj[p] < fy0 || tc.fj[p] > fy1) continue;
        const float dy = v - tc.fj[p];
        const float power = -0.5f * (adx + (Cc * dy) * dy) - bdx * dy;
        if (power > 0.0f) continue;
        const float alpha = fminf(kAlphaMax, o * __expf(power));
        if (alpha < kAlphaMin) continue;
        const float Tn = T[p] * (1.0f - alpha);
        if (Tn < kTmin) { done[p] = true; stop[p] = pos; continue; }
        const float w = alpha * T[p];
        C0[p] = C0[p] + cr * w;
        C1[p] = C1[p] + cg * w;
        C2[p] = C2[p] + cb * w;
        T[p] = Tn;
        nc[p] = pos;
      }
    }
  }
  uint64_t ev = 0;
#pragma unroll
  for (int p = 0; p < kPx; ++p) {
    if (!tc.inside[p]) continue;
    const int64_t q = tc.pix_off + tc.pix[p];
    images[3 * q + 0] = C0[p];
    images[3 * q + 1] = C1[p];
    images[3 * q + 2] = C2[p];
    final_T[q] = T[p];
    last_id[q] = nc[p] ? (int32_t)values[tc.start + nc[p] - 1u] : -1;
    n_contrib[q] = nc[p];
    ev += done[p] ? stop[p] : len;
  }
  if (evals) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ev += __shfl_xor(ev, off, 64);
    if (lane == 0 && ev) atomicAdd(evals, (unsigned long long)ev);
  }
}

// Sum over the 64 lanes; the total lands in lane 63 (row shifts within 16-lane rows, then row
// broadcasts across rows).
__device__ __forceinline__ float wave_total(float v) {
  float t = v;
  t = t + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, true));
  t = t + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, true));
  t = t + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x113, 0xf, 0xf, true));
  t = t + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(t), 0x114, 0xf, 0xe, false));
  t = t + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(t), 0x118, 0xf, 0xc, false));
  t = t + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(t), 0x142, 0xa, 0xf, false));
  t = t + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(t), 0x143, 0xc, 0xf, false));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t), 63));
}

__global__ void __launch_bounds__(64) splat_backward_kernel(
    const Seg* __restrict__ segs, const int64_t* __restrict__ seg_tstart, int S,
    const DevCam* __restrict__ cams, const uint64_t* __restrict__ ranges,
    const uint32_t* __restrict__ values, const SplatRec* __restrict__ rec,
    const float* __restrict__ final_T, const uint32_t* __restrict__ n_contrib,
    const float* __restrict__ dL_dimages, float* __restrict__ grad2d, int64_t G) {
  const int64_t t = blockIdx.x;
  const Tile tc = tile_setup(segs, seg_tstart, S, cams, ranges, t);
  const int lane = __lane_id();
  float T[kPx], g0[kPx], g1[kPx], g2[kPx], B0[kPx], B1[kPx], B2[kPx];
  uint32_t nc[kPx];
  uint32_t mx = 0u;
#pragma unroll
  for (int p = 0; p < kPx; ++p) {
    T[p] = 1.0f; g0[p] = 0.0f; g1[p] = 0.0f; g2[p] = 0.0f;
    B0[p] = 0.0f; B1[p] = 0.0f; B2[p] = 0.0f;
    nc[p] = 0u;
    if (tc.inside[p]) {
      const int64_t q = tc.pix_off + tc.pix[p];
      T[p] = final_T[q];
      nc[p] = n_contrib[q];
      g0[p] = dL_dimages[3 * q + 0];
      g1[p] = dL_dimages[3 * q + 1];
      g2[p] = dL_dimages[3 * q + 2];
    }
    mx = max(mx, nc[p]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, off, 64));
  const int64_t stop = tc.start + (int64_t)mx;
  for (int64_t be = stop; be > tc.start; be -= 64) {
    const int64_t bs = (be - 64) > tc.start ? (be - 64) : tc.start;
    const int n = (int)(be - bs);
    float4 q0 = make_float4(0, 0, 0, 0), q1 = q0, q2 = q0;
    bool keep = false;
    uint32_t my_id = 0u;
    if (lane < n) {
      my_id = values[bs + lane];
      const SplatRec r = rec[tc.g_off + my_id];
      q0 = r.q0; q1 = r.q1; q2 = r.q2;
      keep = may_touch(q0, q1, q2, tc);
    }
    float acc[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) acc[a] = 0.0f;
    uint64_t mask = __ballot(keep);
    const uint32_t rel0 = (uint32_t)(bs - tc.start);
    while (mask) {
      const int k = 63 - __builtin_clzll(mask);          // back to front
      mask &= ~(1ull << k);
      const float u = rl(q0.x, k), v = rl(q0.y, k), A = rl(q0.z, k), B = rl(q0.w, k);
      const float Cc = rl(q1.x, k), o = rl(q1.y, k);
      const uint32_t wx = rlu(q2.y, k), wy = rlu(q2.z, k);
      const float fx0 = (float)(wx & 0xffffu), fx1 = (float)(wx >> 16);
      const float fy0 = (float)(wy & 0xffffu), fy1 = (float)(wy >> 16);
      const float cr = rl(q1.z, k), cg = rl(q1.w, k), cb = rl(q2.x, k);
      const bool colin = !(tc.fi < fx0 || tc.fi > fx1);
      const float dx = u - tc.fi;
      const float adx = (A * dx) * dx;
      const float bdx = B * dx;
      const uint32_t rel = rel0 + (uint32_t)k;
      float su = 0.0f, sv = 0.0f, sA = 0.0f, sB = 0.0f, sC = 0.0f, so = 0.0f;
      float sr = 0.0f, sg = 0.0f, sb = 0.0f;
      bool any = false;
#pragma unroll
      for (int p = 0; p < kPx; ++p) {
        if (!(rel < nc[p]) || !colin || tc.fj[p] < fy0 || tc.fj[p] > fy1) continue;
        const float dy = v - tc.fj[p];
        const float power = -0.5f * (adx + (Cc * dy) * dy) - bdx * dy;
        if (power > 0.0f) continue;
        const float e = __expf(power);
        const float oe = o * e;
        const float alpha = fminf(kAlphaMax, oe);
        if (alpha < kAlphaMin) continue;
        any = true;
        T[p] = T[p] / (1.0f - alpha);
        const float w = alpha * T[p];
        sr += w * g0[p];
        sg += w * g1[p];
        sb += w * g2[p];
        const float dalpha = T[p] * (((cr - B0[p]) * g0[p] + (cg - B1[p]) * g1[p]) + (cb - B2[p]) * g2[p]);
        B0[p] = alpha * cr + (1.0f - alpha) * B0[p];
        B1[p] = alpha * cg + (1.0f - alpha) * B1[p];
        B2[p] = alpha * cb + (1.0f - alpha) * B2[p];
        if (!(oe > kAlphaMax)) {
          const float dpow = dalpha * alpha;
          so += dalpha * e;
          sA += -0.5f * dx * dx * dpow;
          sC += -0.5f * dy * dy * dpow;
          sB += -dx * dy * dpow;
          su += (-A * dx - B * dy) * dpow;
          sv += (-Cc * dy - B * dx) * dpow;
        }
      }
      if (__ballot(any) == 0ull) continue;
      const float tu = wave_total(su), tv = wave_total(sv), tA = wave_total(sA);
      const float tB = wave_total(sB), tC = wave_total(sC), to = wave_total(so);
      const float tr = wave_total(sr), tg = wave_total(sg), tb = wave_total(sb);
      if (lane == k) {
        acc[0] = tu; acc[1] = tv; acc[2] = tA; acc[3] = tB; acc[4] = tC;
        acc[5] = to; acc[6] = tr; acc[7] = tg; acc[8] = tb;
      }
    }
    if (lane < n) {
      const int64_t gi = tc.g_off + (int64_t)my_id;
#pragma unroll
      for (int a = 0; a < 9; ++a)
        if (acc[a] != 0.0f) unsafeAtomicAdd(&grad2d[(int64_t)a * G + gi], acc[a]);
    }
  }
}

}  // namespace

hipError_t launch_splat_forward(hipStream_t st, const Seg* segs, const int64_t* seg_tstart, int S,
                                const DevCam* cams, int64_t n_tiles, const uint64_t* ranges,
                                const uint32_t* values, const SplatRec* rec, float* images,
                                float* final_T, int32_t* last_id, uint32_t* n_contrib,
                                unsigned long long* evals) {
  if (n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(splat_forward_kernel, dim3((unsigned)n_tiles), dim3(64), 0, st, segs,
                     seg_tstart, S, cams, ranges, values, rec, images, final_T, last_id, n_contrib,
                     evals);
  return hipGetLastError();
}

hipError_t launch_splat_backward(hipStream_t st, const Seg* segs, const int64_t* seg_tstart, int S,
                                 const DevCam* cams, int64_t n_tiles, const uint64_t* ranges,
                                 const uint32_t* values, const SplatRec* rec, const float* final_T,
                                 const uint32_t* n_contrib, const float* dL_dimages,
                                 float* grad2d, int64_t G, int deterministic) {
  (void)deterministic;
  if (n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(splat_backward_kernel, dim3((unsigned)n_tiles), dim3(64), 0, st, segs,
                     seg_tstart, S, cams, ranges, values, rec, final_T, n_contrib, dL_dimages,
                     grad2d, G);
  return hipGetLastError();
}

}  // namespace gsc
