// k_splat.hip -- front-to-back alpha blending of the binned Gaussians (the cache images) and
// its adjoint (3D Gaussian splatting's tile rasteriser, adapted by GSCache to render each cache
// level; Method: "A Path Space Radiance Cache", "Cache Training").
//
// One 64-lane wavefront per tile of 16 x 4 kS pixels (kS = 4: the 16x16 tiles of
// gsc_project_bin; kS = 8: the 16x32 tiles frames bin).  Lane l owns the kS pixels
// (l & 15, (l >> 4) + 4 p), p < kS, so slot p of the wave is the tile's 16x4 row band
// 4p..4p+3.  The tile's list is consumed 64 entries at a time: lane j loads entry j's 48-byte
// record into registers, then the wave walks the entries in list order and every lane fetches
// the current entry's record from lane k with ds_bpermute, so the record reaches the vector
// unit in vector registers (on gfx950 an instruction that reads a scalar register issues at half
// the rate of one that reads only vector registers and literals).  The Gaussian's integer pixel
// window becomes, on the scalar unit, one 64-bit lane mask per slot; a slot with no live pixel
// inside the window is skipped by a scalar branch and the others run branch-free (predicated
// selects).  An entry whose alpha >= 1/255 ellipse provably misses every pixel of the tile (a
// conservative test of the quadratic form over the tile rectangle) is skipped by the whole wave;
// such an entry is skipped by every pixel anyway, so results do not change.
//
// The adjoint walks the same lists back to front from each pixel's last contributor, recovers
// the transmittance before each Gaussian as T / (1 - alpha), sums each Gaussian's nine
// screen-space gradients over the lane's kS pixels, reduces them within each 16-lane row group
// with DPP row shifts, parks the four group sums in LDS, and once per batch of 64 entries the
// lane that loaded an entry adds its groups and issues the nine float atomics of that
// (tile, Gaussian).
#include "gsc_dev.h"

namespace gsc {

namespace {

constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTmin = 1e-4f;
constexpr int kPartStride = 10;   // floats per entry of the adjoint's LDS sums

template <int kS>
struct Tile {
  int64_t start, end;
  int64_t g_off, pix_off;
  float fi;                  // this lane's pixel column (full-frame)
  float fj[kS];              // this lane's pixel rows (full-frame)
  int px, py0;               // this lane's column and first row in the render window
  int cw, ch;                // render window size
  int xbase, ybase;          // full-frame coordinates of the tile's first pixel
  float ti0, ti1, tj0, tj1;  // the tile's pixel rectangle inside the render window
#ifdef GSC_DEBUG
  int64_t n;                 // the level's Gaussians (for the list-entry checks)
#endif
  __device__ bool inside(int p) const { return px < cw && py0 + 4 * p < ch; }
  __device__ int64_t pix(int p) const { return (int64_t)(py0 + 4 * p) * cw + px; }
};

// A wavefront covers the 16 x 4 kS block `part` (kW across, kH down, row-major) of tile t, a
// tile of 16 kW x 4 kS kH pixels; the block's rectangle is what may_touch tests.
template <int kS, int kW = 1, int kH = 1>
__device__ __forceinline__ Tile<kS> tile_setup(const Seg* __restrict__ segs,
                                               const int64_t* __restrict__ seg_tstart, int S,
                                               const DevCam* __restrict__ cams,
                                               const uint64_t* __restrict__ ranges, int64_t t,
                                               int part = 0) {
  static_assert(kS == 4 || kS == 8, "four or eight slots per lane");
  const int s = find_segment(seg_tstart, S, t);
  const Seg& sg = segs[s];
  const DevCam& cam = cams[sg.cam];
  const int64_t lt = t - sg.tile_base;
  const int tx = (int)(lt % sg.TX), ty = (int)(lt / sg.TX);
  const int lane = __lane_id();
  const int ox = tx * (16 * kW) + 16 * (part % kW);
  const int oy = ty * (4 * kS * kH) + (4 * kS) * (part / kW);
  Tile<kS> c;
  c.start = (int64_t)ranges[2 * t];
  c.end = (int64_t)ranges[2 * t + 1];
  c.g_off = sg.g_off;
  c.pix_off = sg.pix_off;
  c.px = ox + (lane & 15);
  c.py0 = oy + (lane >> 4);
  c.cw = cam.w;
  c.ch = cam.h;
  c.fi = (float)(cam.x0 + c.px);
#pragma unroll
  for (int k = 0; k < kS; ++k) c.fj[k] = (float)(cam.y0 + c.py0 + 4 * k);
  c.xbase = cam.x0 + ox;
  c.ybase = cam.y0 + oy;
  c.ti0 = (float)(cam.x0 + ox);
  c.ti1 = (float)(cam.x0 + min(ox + 16, cam.w) - 1);
  c.tj0 = (float)(cam.y0 + oy);
  c.tj1 = (float)(cam.y0 + min(oy + 4 * kS, cam.h) - 1);
#ifdef GSC_DEBUG
  c.n = sg.n;
#endif
  return c;
}

// Conservative test: can o exp(-Q(u - i, v - j) / 2) reach 1/255 at some pixel (i, j) of the
// tile inside the Gaussian's integer window?  Q is the conic's quadratic form; its minimum over
// a rectangle not containing the centre lies on the boundary.
template <int kS>
__device__ __forceinline__ bool may_touch(const float4& q0, const float4& q1, const float4& q2,
                                          const Tile<kS>& tc) {
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

__device__ __forceinline__ uint32_t rlu(float v, int k) {
  return (uint32_t)__builtin_amdgcn_readlane(__float_as_int(v), k);
}


// Lane masks of the tile's pixels inside a Gaussian's integer window (packed full-frame bounds
// wx = px0 | px1 << 16, wy = py0 | py1 << 16), one per slot.  Uniform arithmetic: it runs on
// the scalar unit.
template <int kS>
__device__ __forceinline__ void window_masks(uint32_t wx, uint32_t wy, int xbase, int ybase,
                                             uint64_t m[kS]) {
  const int lo = max((int)(wx & 0xffffu) - xbase, 0);
  const int hi = min((int)(wx >> 16) - xbase, 15);
  const uint32_t c16 = (lo <= hi) ? ((2u << hi) - (1u << lo)) : 0u;
  const uint32_t c32 = c16 | (c16 << 16);
  const uint64_t c64 = ((uint64_t)c32 << 32) | (uint64_t)c32;
  const int ylo = (int)(wy & 0xffffu) - ybase, yhi = (int)(wy >> 16) - ybase;
  if (ylo <= 0 && yhi >= 4 * kS - 1) {   // the window spans every row of the block (most entries)
#pragma unroll
    for (int p = 0; p < kS; ++p) m[p] = c64;
    return;
  }
#pragma unroll
  for (int p = 0; p < kS; ++p) {
    const int glo = max(ylo - 4 * p, 0), ghi = min(yhi - 4 * p, 3);
    m[p] = (glo <= ghi) ? (c64 & (~0ull >> (48 - 16 * ghi)) & (~0ull << (16 * glo))) : 0ull;
  }
}

// Per batch lane (one list entry): the window's columns among the block's 16 (bits 0-15) and
// bit 16 set when the window spans every row of the block, so that an entry's masks mostly
// come from one lane read and a few scalar operations.
template <int kS>
__device__ __forceinline__ uint32_t window_pack(uint32_t wx, uint32_t wy, int xbase, int ybase) {
  const int lo = max((int)(wx & 0xffffu) - xbase, 0);
  const int hi = min((int)(wx >> 16) - xbase, 15);
  const uint32_t c16 = (lo <= hi) ? ((2u << hi) - (1u << lo)) : 0u;
  const int ylo = (int)(wy & 0xffffu) - ybase, yhi = (int)(wy >> 16) - ybase;
  return c16 | ((ylo <= 0 && yhi >= 4 * kS - 1) ? 0x10000u : 0u);
}

// An entry's slot masks from its packed window (and, when the window does not span every row,
// its full bounds).
template <int kS>
__device__ __forceinline__ void entry_masks(uint32_t pk, float q2y, float q2z, int k, int xbase,
                                            int ybase, uint64_t m[kS]) {
  if (pk & 0x10000u) {
    const uint32_t c32 = (pk & 0xffffu) * 0x10001u;
    const uint64_t c64 = ((uint64_t)c32 << 32) | (uint64_t)c32;
#pragma unroll
    for (int p = 0; p < kS; ++p) m[p] = c64;
  } else {
    window_masks<kS>(rlu(q2y, k), rlu(q2z, k), xbase, ybase, m);
  }
}

__device__ __forceinline__ bool lane_in(uint64_t mask) {
  return __builtin_amdgcn_inverse_ballot_w64(mask);
}

// Work counters (stats words, all sums over the launch): the forward always adds [2] each
// pixel's walk length and [3] entries its wavefront evaluated after the cull; with kCount also
// [0] list positions each pixel examined, [1] blended pairs, [4] (pixel, entry) pairs tested
// (lanes live in an evaluated slot) and [5] slot evaluations.  The adjoint with kCount
// adds [6] pairs tested, [7] pairs blended, [8] slot evaluations, [9] entries walked after the
// cull and [10] float atomics issued.
enum { kStEval = 0, kStBlend, kStContrib, kStEntries, kStFwdTested, kStFwdSlots, kStBwdTested,
       kStBwdBlend, kStBwdSlots, kStBwdEntries, kStBwdAtomics, kStBwdRecords, kStWords };

// Workgroup b takes block b % (kW kH) of tile order[b / (kW kH)] (one independent wavefront
// per block).
template <bool kCount, int kS, int kW, int kH>
__global__ void __launch_bounds__(64) splat_forward_kernel(
    const Seg* __restrict__ segs, const int64_t* __restrict__ seg_tstart, int S,
    const DevCam* __restrict__ cams, const uint64_t* __restrict__ ranges,
    const uint32_t* __restrict__ values, const SplatRec* __restrict__ rec,
    float* __restrict__ images, float* __restrict__ final_T, int32_t* __restrict__ last_id,
    uint32_t* __restrict__ n_contrib, unsigned long long* __restrict__ stats,
    const uint32_t* __restrict__ order, uint32_t* __restrict__ tile_work,
    const uint64_t* __restrict__ n_inst, uint64_t capacity) {
  // A binning whose instances did not fit its capacity left incomplete lists: do nothing (the
  // frame is run again with a larger capacity).
  if (*n_inst > capacity) return;
  const int64_t b = (int64_t)blockIdx.x / (kW * kH);
  const int64_t t = order ? (int64_t)order[b] : b;
  const Tile<kS> tc = tile_setup<kS, kW, kH>(segs, seg_tstart, S, cams, ranges, t,
                                              (int)(blockIdx.x % (kW * kH)));
  const int lane = __lane_id();
  // The batch's records, one per lane.  Each entry's values reach every lane as LDS reads at one
  // address (broadcasts): three loads instead of nine lane-to-lane permutes (ds_bpermute), and
  // broadcasting through v_readlane into scalar registers measured slower still.
  __shared__ float4 srec[3][64];
  float T[kS], C0[kS], C1[kS], C2[kS];
  uint32_t nc[kS], stop[kS];
  uint64_t done[kS];                     // lanes finished (terminated, or outside the image)
  uint32_t n_blend = 0u, n_entries = 0u;
  uint64_t n_tested = 0u, n_slots = 0u;
#pragma unroll
  for (int p = 0; p < kS; ++p) {
    T[p] = 1.0f; C0[p] = 0.0f; C1[p] = 0.0f; C2[p] = 0.0f;
    nc[p] = 0u; stop[p] = 0u;
    done[p] = __ballot(!tc.inside(p));
  }
  auto all_done = [&]() {
    uint64_t d = ~0ull;
#pragma unroll
    for (int p = 0; p < kS; ++p) d &= done[p];
    return d == ~0ull;
  };
  const uint32_t len = (uint32_t)(tc.end - tc.start);
  for (int64_t bs = tc.start; bs < tc.end; bs += 64) {
    if (all_done()) break;
    const int64_t idx = bs + lane;
    float4 q0 = make_float4(0, 0, 0, 0), q1 = q0, q2 = q0;
    bool keep = false;
    if (idx < tc.end && GSC_DCHECK((uint64_t)idx < capacity && (int64_t)values[idx] < tc.n,
                                   kDbgListEntry)) {
      const SplatRec r = rec[tc.g_off + values[idx]];
      q0 = r.q0; q1 = r.q1; q2 = r.q2;
      keep = may_touch(q0, q1, q2, tc);
    }
    srec[0][lane] = q0; srec[1][lane] = q1; srec[2][lane] = q2;
    const uint32_t wpk = window_pack<kS>(__float_as_uint(q2.y), __float_as_uint(q2.z), tc.xbase, tc.ybase);
    uint64_t mask = __ballot(keep);
    const uint32_t rel0 = (uint32_t)(bs - tc.start);
    while (mask) {
      if (all_done()) break;
      const int k = __builtin_ctzll(mask);
      mask &= mask - 1ull;
      ++n_entries;
      // Entry k's record from LDS, read at one address by every lane (a broadcast): three
      // loads instead of nine lane-to-lane permutes.
      const float4 e0 = srec[0][k], e1 = srec[1][k];
      const float cb = srec[2][k].x;
      const float u = e0.x, v = e0.y, A = e0.z, B = e0.w;
      const float Cc = e1.x, o = e1.y, cr = e1.z, cg = e1.w;
      uint64_t win[kS];
      entry_masks<kS>(__builtin_amdgcn_readlane(wpk, k), q2.y, q2.z, k, tc.xbase, tc.ybase, win);
      const float dx = u - tc.fi;
      // power = -(A dx^2 + C dy^2) / 2 - B dx dy, with the halving applied to A dx^2 and C
      // beforehand: scaling by -1/2 is exact, so every rounding, and the result, are unchanged.
      const float adxh = -0.5f * ((A * dx) * dx);
      const float Ch = -0.5f * Cc;
      const float bdx = B * dx;
      uint32_t pos = rel0 + (uint32_t)k + 1u;
      // Held in a vector register once per entry (the slots' selects would otherwise each copy
      // it from its scalar register).
      asm volatile("" : "+v"(pos));
#pragma unroll
      for (int p = 0; p < kS; ++p) {
        const uint64_t act = win[p] & ~done[p];
        if (act == 0ull) continue;
        if (kCount) { n_tested += (uint64_t)__popcll(act); ++n_slots; }
        const float dy = v - tc.fj[p];
        const float power = (adxh + (Ch * dy) * dy) - bdx * dy;
        const float alpha = fminf(kAlphaMax, o * __expf(power));
        // Lane masks on the scalar unit: ballots of single compares cost no vector work.
        const uint64_t okm = act & __builtin_amdgcn_ballot_w64(!(power > 0.0f)) &
                             __builtin_amdgcn_ballot_w64(!(alpha < kAlphaMin));
        const float Tn = T[p] * (1.0f - alpha);
        const uint64_t finm = okm & __builtin_amdgcn_ballot_w64(Tn < kTmin);
        const uint64_t blm = okm & ~finm;
        const bool bl = lane_in(blm);
        const float w = bl ? alpha * T[p] : 0.0f;
        C0[p] = fmaf(cr, w, C0[p]);
        C1[p] = fmaf(cg, w, C1[p]);
        C2[p] = fmaf(cb, w, C2[p]);
        T[p] = bl ? Tn : T[p];
        nc[p] = bl ? pos : nc[p];
        done[p] |= finm;
        if (kCount) {
          stop[p] = lane_in(finm) ? pos : stop[p];
          n_blend += (uint32_t)__popcll(blm);
        }
      }
    }
  }
  // The tile's work estimate for the adjoint's schedule (with several blocks per tile summed
  // into a zeroed array).
  if (tile_work && lane == 0) {
    if (kW * kH == 1) tile_work[t] = n_entries;
    else atomicAdd(&tile_work[t], n_entries);
  }
  uint64_t ev = 0, ncs = 0;
#pragma unroll
  for (int p = 0; p < kS; ++p) {
    if (!tc.inside(p)) continue;
    const int64_t q = tc.pix_off + tc.pix(p);
    images[3 * q + 0] = C0[p];
    images[3 * q + 1] = C1[p];
    images[3 * q + 2] = C2[p];
    final_T[q] = T[p];
    last_id[q] = nc[p] ? (int32_t)values[tc.start + nc[p] - 1u] : -1;
    n_contrib[q] = nc[p];
    if (kCount) ev += stop[p] ? stop[p] : len;
    ncs += nc[p];
  }
  if (stats) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      ev += __shfl_xor(ev, off, 64);
      ncs += __shfl_xor(ncs, off, 64);
    }
    if (lane == 0) {
      atomicAdd(&stats[kStContrib], (unsigned long long)ncs);
      atomicAdd(&stats[kStEntries], (unsigned long long)n_entries);
      if (kCount) {
        atomicAdd(&stats[kStEval], (unsigned long long)ev);
        atomicAdd(&stats[kStBlend], (unsigned long long)n_blend);
        atomicAdd(&stats[kStFwdTested], (unsigned long long)n_tested);
        atomicAdd(&stats[kStFwdSlots], (unsigned long long)n_slots);
      }
    }
  }
}

// The adjoint's ways of accumulating the per-(tile, Gaussian) partials: float atomics into grad2d;
// or, deterministically, a first pass that finds the largest |partial| of each gradient component
// of each Gaussian and a second that adds round(partial * scale) as 64-bit integers, with
// scale = 2^(40 - e) for a largest |partial| in [2^e, 2^(e+1)).  Every rounded partial is below
// 2^41 and a Gaussian has at most one partial per tile (at most 2^20 tiles in an image), so the
// integer sum stays below 2^61; each partial is kept to 2^-41 of the Gaussian's largest.
enum { kAdjointAtomic = 0, kAdjointMax = 1, kAdjointFixed = 2 };

__device__ __forceinline__ double fixed_scale(uint32_t max_bits) {
  const float m = __uint_as_float(max_bits);
  return m > 0.0f ? ldexp(1.0, 40 - ilogbf(m)) : 0.0;
}

// gmax, gfix: [9][G]; grad2d: [G][kGrad2dStride].
__global__ void __launch_bounds__(256) fixed_to_float_kernel(const uint32_t* __restrict__ gmax,
                                                             const unsigned long long* __restrict__ gfix,
                                                             int64_t G, float* __restrict__ grad2d) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= 9 * G) return;
  const double sc = fixed_scale(gmax[i]);
  const int64_t a = i / G, g = i - a * G;
  grad2d[g * kGrad2dStride + a] = sc > 0.0 ? (float)((double)(long long)gfix[i] / sc) : 0.0f;
}

// Workgroup b walks block b % kW (16 x 4 kS, the tile's blocks side by side) of tile
// order[b / kW], one independent wavefront per block.
template <bool kCount, int kS, int kW>
__global__ void __launch_bounds__(64) splat_backward_kernel(
    const Seg* __restrict__ segs, const int64_t* __restrict__ seg_tstart, int S,
    const DevCam* __restrict__ cams, const uint64_t* __restrict__ ranges,
    const uint32_t* __restrict__ values, const SplatRec* __restrict__ rec,
    const float* __restrict__ final_T, const uint32_t* __restrict__ n_contrib,
    const float* __restrict__ dL_dimages, float* __restrict__ grad2d, int64_t G,
    const uint32_t* __restrict__ order, int mode, uint32_t* __restrict__ gmax,
    unsigned long long* __restrict__ gfix, unsigned long long* __restrict__ stats,
    const uint64_t* __restrict__ n_inst, uint64_t capacity) {
  if (*n_inst > capacity) return;               // incomplete lists (see the forward)
  __shared__ float part[64][kPartStride];       // [entry][component]: the wave's sums
  // One entry's per-lane values by component; rows padded to 68 floats so that the sixteen-float
  // reads of the nine components start in different banks.
  __shared__ __align__(16) float red[9][68];
  __shared__ uint32_t sent[64], sid[64];        // entries with partials: batch position, id
  __shared__ float4 srec[3][64];                // the batch's records, one per lane
  const int64_t b = (int64_t)blockIdx.x / kW;
  const int64_t t = order ? (int64_t)order[b] : b;
  const Tile<kS> tc = tile_setup<kS, kW, 1>(segs, seg_tstart, S, cams, ranges, t,
                                             (int)(blockIdx.x % kW));
  const int lane = __lane_id();
  // BG: the colour blended behind the current Gaussian (from the entries already walked), dotted
  // with the pixel's image gradient g; it is all the adjoint needs of that colour.
  float T[kS], g0[kS], g1[kS], g2[kS], BG[kS];
  uint32_t nc[kS];
  uint32_t mx = 0u;
#pragma unroll
  for (int p = 0; p < kS; ++p) {
    T[p] = 1.0f; g0[p] = 0.0f; g1[p] = 0.0f; g2[p] = 0.0f;
    BG[p] = 0.0f;
    nc[p] = 0u;
    if (tc.inside(p)) {
      const int64_t q = tc.pix_off + tc.pix(p);
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
  uint64_t n_tested = 0u, n_blended = 0u, n_slots = 0u, n_entries = 0u, n_records = 0u;
  uint32_t n_atomics = 0u;
  for (int64_t be = stop; be > tc.start; be -= 64) {
    const int64_t bs = (be - 64) > tc.start ? (be - 64) : tc.start;
    const int n = (int)(be - bs);
    float4 q0 = make_float4(0, 0, 0, 0), q1 = q0, q2 = q0;
    bool keep = false;
    uint32_t my_id = 0u;
    if (lane < n && GSC_DCHECK((uint64_t)(bs + lane) < capacity &&
                               (int64_t)values[bs + lane] < tc.n, kDbgListEntry)) {
      my_id = values[bs + lane];
      const SplatRec r = rec[tc.g_off + my_id];
      q0 = r.q0; q1 = r.q1; q2 = r.q2;
      keep = may_touch(q0, q1, q2, tc);
    }
    srec[0][lane] = q0; srec[1][lane] = q1; srec[2][lane] = q2;
    const uint32_t wpk = window_pack<kS>(__float_as_uint(q2.y), __float_as_uint(q2.z), tc.xbase, tc.ybase);
    uint64_t mask = __ballot(keep);
    uint64_t has = 0ull;                       // entries whose row sums are parked in LDS
    const uint32_t rel0 = (uint32_t)(bs - tc.start);
    while (mask) {
      const int k = 63 - __builtin_clzll(mask);          // back to front
      mask &= ~(1ull << k);
      if (kCount) ++n_entries;
      // Entry k's record from LDS, read at one address by every lane (a broadcast): three
      // loads instead of nine lane-to-lane permutes.
      const float4 e0 = srec[0][k], e1 = srec[1][k];
      const float cb = srec[2][k].x;
      const float u = e0.x, v = e0.y, A = e0.z, B = e0.w;
      const float Cc = e1.x, o = e1.y, cr = e1.z, cg = e1.w;
      uint64_t win[kS];
      entry_masks<kS>(__builtin_amdgcn_readlane(wpk, k), q2.y, q2.z, k, tc.xbase, tc.ybase, win);
      const float dx = u - tc.fi;
      // The halving of the quadratic form applied beforehand (exact; see the forward).
      const float adxh = -0.5f * ((A * dx) * dx);
      const float Ch = -0.5f * Cc;
      const float bdx = B * dx;
      const uint32_t rel = rel0 + (uint32_t)k;
      // Per lane, the moments of dL/dpower over its pixels (all in one column, so dx is
      // common): m0 = sum dpow, m1 = sum dpow dy, m2 = sum dpow dy^2; the conic, mean and
      // opacity gradients are linear in them.
      float m0 = 0.0f, m1 = 0.0f, m2 = 0.0f;
      float sr = 0.0f, sg = 0.0f, sb = 0.0f;
      uint64_t any = 0ull;
#pragma unroll
      for (int p = 0; p < kS; ++p) {
        const uint64_t act = win[p] & __builtin_amdgcn_ballot_w64(rel < nc[p]);
        if (act == 0ull) continue;
        const float dy = v - tc.fj[p];
        const float power = (adxh + (Ch * dy) * dy) - bdx * dy;
        const float e = __expf(power);
        const float oe = o * e;
        const float alpha = fminf(kAlphaMax, oe);
        const uint64_t okm = act & __builtin_amdgcn_ballot_w64(!(power > 0.0f)) &
                             __builtin_amdgcn_ballot_w64(!(alpha < kAlphaMin));
        if (kCount) {
          n_tested += (uint64_t)__popcll(act);
          n_blended += (uint64_t)__popcll(okm);
          ++n_slots;
        }
        any |= okm;
        const bool ok = lane_in(okm);
        const float az = ok ? alpha : 0.0f;
        T[p] = ok ? T[p] * __builtin_amdgcn_rcpf(1.0f - alpha) : T[p];
        const float w = az * T[p];
        sr = fmaf(w, g0[p], sr);
        sg = fmaf(w, g1[p], sg);
        sb = fmaf(w, g2[p], sb);
        // dL/dalpha = T (c - background) . g; the background moves towards c by alpha.
        const float cgp = fmaf(cr, g0[p], fmaf(cg, g1[p], cb * g2[p]));
        const float dd = cgp - BG[p];
        BG[p] = fmaf(az, dd, BG[p]);
        // dL/dpower = alpha dL/dalpha = (alpha T) dd where alpha is not clamped (it then depends
        // on power and opacity; dL/do = dL/dpower / o).
        const float dpow = !(oe > kAlphaMax) ? w * dd : 0.0f;
        const float tdy = dpow * dy;
        m0 += dpow;
        m1 += tdy;
        m2 = fmaf(tdy, dy, m2);
      }
      if (any == 0ull) continue;
      has |= 1ull << k;
      // power = -(A dx^2 + C dy^2) / 2 - B dx dy with dx = u - i, dy = v - j, and dL/do from
      // alpha = o e^power (the unclamped pairs only, as dpow).
      const float so = m0 * __builtin_amdgcn_rcpf(o);
      const float sA = ((-0.5f * dx) * dx) * m0;
      const float sC = -0.5f * m2;
      const float sB = -dx * m1;
      const float su = fmaf(-B, m1, (-A * dx) * m0);
      const float sv = fmaf(-Cc, m1, (-B * dx) * m0);
      // The wave's nine sums through LDS (a transpose instead of per-row DPP steps): every lane
      // parks its nine values by component; lane 16 r + a then adds the sixteen values of
      // component a in row r (lanes with a >= 9 add a copy of component 8 and are ignored),
      // and two shuffles add the four rows.  A single wave runs the workgroup and its LDS
      // accesses complete in order, so no barrier is needed.
      red[0][lane] = su; red[1][lane] = sv; red[2][lane] = sA;
      red[3][lane] = sB; red[4][lane] = sC; red[5][lane] = so;
      red[6][lane] = sr; red[7][lane] = sg; red[8][lane] = sb;
      {
        const int ra = (lane & 15) < 9 ? (lane & 15) : 8;
        const float4* q = reinterpret_cast<const float4*>(&red[ra][lane & 48]);
        const float4 x0 = q[0], x1 = q[1], x2 = q[2], x3 = q[3];
        float t = ((x0.x + x0.y) + (x0.z + x0.w)) + ((x1.x + x1.y) + (x1.z + x1.w)) +
                  (((x2.x + x2.y) + (x2.z + x2.w)) + ((x3.x + x3.y) + (x3.z + x3.w)));
        t += __shfl_xor(t, 32, 64);
        t += __shfl_xor(t, 16, 64);
        if (lane < 9) part[k][lane] = t;
      }
    }
    if (has == 0ull) continue;
    // The entries with partials, in order, then their nine sums: lane 9 j + a adds component a
    // of the (j0 + j)-th of them, seven entries per instruction, so the nine atomics of an entry
    // go out together and land in one 64-byte record.
    if ((has >> lane) & 1ull) {
      const int r = __popcll(has & ((1ull << lane) - 1ull));
      sent[r] = (uint32_t)lane;
      sid[r] = my_id;
    }
    __syncthreads();
    const int E = __popcll(has);
    if (kCount) n_records += (uint64_t)E;
    const int jl = lane / 9, a = lane - 9 * jl;
    for (int j0 = 0; j0 < E; j0 += 7) {
      const int j = j0 + jl;
      if (lane < 63 && j < E) {
        const uint32_t k = sent[j];
        const float acc = part[k][a];
        const int64_t gi = tc.g_off + (int64_t)sid[j];
        if (mode == kAdjointAtomic) {
          if (acc != 0.0f) {
            unsafeAtomicAdd(&grad2d[gi * kGrad2dStride + a], acc);
            if (kCount) ++n_atomics;
          }
        } else if (mode == kAdjointMax) {
          if (acc != 0.0f) atomicMax(&gmax[(int64_t)a * G + gi], __float_as_uint(fabsf(acc)));
        } else {
          // Integer sums do not depend on the order in which the atomics land.
          const int64_t at = (int64_t)a * G + gi;
          const long long qv = llrint((double)acc * fixed_scale(gmax[at]));
          if (qv) atomicAdd(&gfix[at], (unsigned long long)qv);
        }
      }
    }
    __syncthreads();
  }
  if (kCount) {
    uint64_t na = n_atomics;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) na += __shfl_xor(na, off, 64);
    if (lane == 0) {
      atomicAdd(&stats[kStBwdTested], (unsigned long long)n_tested);
      atomicAdd(&stats[kStBwdBlend], (unsigned long long)n_blended);
      atomicAdd(&stats[kStBwdSlots], (unsigned long long)n_slots);
      atomicAdd(&stats[kStBwdEntries], (unsigned long long)n_entries);
      atomicAdd(&stats[kStBwdAtomics], (unsigned long long)na);
      atomicAdd(&stats[kStBwdRecords], (unsigned long long)n_records);
    }
  }
}

// Heaviest-first tile schedule, by a bucket sort in one workgroup: a tile's work estimate (the
// list length, or the entries the forward processed) falls into one of 256 buckets of width
// 2^(1/8) in log scale; order[] lists the tiles bucket by bucket, heaviest first.  The order
// within a bucket is whatever the LDS atomics give: it only schedules, no result depends on it.
constexpr int kOrderThreads = 1024;

__device__ __forceinline__ int work_bucket(uint32_t w) {
  if (w == 0u) return 0;
  const int lg = 31 - __builtin_clz(w);                             // floor(log2 w)
  const int frac = lg >= 3 ? (int)((w >> (lg - 3)) & 7u) : (int)((w << (3 - lg)) & 7u);
  return min(255, 1 + 8 * lg + frac);
}

__global__ void __launch_bounds__(kOrderThreads) tile_order_kernel(const uint64_t* __restrict__ ranges,
                                                                   const uint32_t* __restrict__ work,
                                                                   int64_t n_tiles,
                                                                   uint32_t* __restrict__ order) {
  __shared__ uint32_t cnt[256];
  const int tid = threadIdx.x;
  for (int i = tid; i < 256; i += kOrderThreads) cnt[i] = 0u;
  __syncthreads();
  auto bucket = [&](int64_t t) -> int {
    const uint64_t w = work ? (uint64_t)work[t] : ranges[2 * t + 1] - ranges[2 * t];
    return 255 - work_bucket((uint32_t)(w > 0xffffffffull ? 0xffffffffull : w));
  };
  for (int64_t t = tid; t < n_tiles; t += kOrderThreads) atomicAdd(&cnt[bucket(t)], 1u);
  __syncthreads();
  if (tid < 64) {                                   // exclusive scan of the 256 counts, 4 per lane
    uint32_t c[4], s = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) { c[j] = cnt[4 * tid + j]; s += c[j]; }
    uint32_t incl = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t u = (uint32_t)__shfl_up((int)incl, off, 64);
      if (tid >= off) incl += u;
    }
    uint32_t run = incl - s;
#pragma unroll
    for (int j = 0; j < 4; ++j) { cnt[4 * tid + j] = run; run += c[j]; }
  }
  __syncthreads();
  for (int64_t t = tid; t < n_tiles; t += kOrderThreads)
    order[atomicAdd(&cnt[bucket(t)], 1u)] = (uint32_t)t;
}

template <int kS, int kW, int kH>
void splat_forward_dispatch(hipStream_t st, const Seg* segs, const int64_t* seg_tstart, int S,
                            const DevCam* cams, int64_t n_tiles, const uint64_t* ranges,
                            const uint32_t* values, const SplatRec* rec, float* images,
                            float* final_T, int32_t* last_id, uint32_t* n_contrib,
                            unsigned long long* stats, const uint32_t* order, uint32_t* tile_work,
                            bool count, const uint64_t* n_inst, uint64_t capacity) {
  const dim3 grid((unsigned)(n_tiles * kW * kH)), block(64);
  if (count && stats)
    hipLaunchKernelGGL((splat_forward_kernel<true, kS, kW, kH>), grid, block, 0, st, segs,
                       seg_tstart, S, cams, ranges, values, rec, images, final_T, last_id,
                       n_contrib, stats, order, tile_work, n_inst, capacity);
  else
    hipLaunchKernelGGL((splat_forward_kernel<false, kS, kW, kH>), grid, block, 0, st, segs,
                       seg_tstart, S, cams, ranges, values, rec, images, final_T, last_id,
                       n_contrib, stats, order, tile_work, n_inst, capacity);
}

template <int kS, int kW>
void splat_backward_dispatch(hipStream_t st, const Seg* segs, const int64_t* seg_tstart, int S,
                             const DevCam* cams, int64_t n_tiles, const uint64_t* ranges,
                             const uint32_t* values, const SplatRec* rec, const float* final_T,
                             const uint32_t* n_contrib, const float* dL_dimages, float* grad2d,
                             int64_t G, const uint32_t* order, uint32_t* gmax,
                             unsigned long long* gfix, unsigned long long* stats, bool count,
                             const uint64_t* n_inst, uint64_t capacity) {
  const dim3 grid((unsigned)(n_tiles * kW)), block(64);
  if (!gmax) {
    if (count && stats)
      hipLaunchKernelGGL((splat_backward_kernel<true, kS, kW>), grid, block, 0, st, segs, seg_tstart,
                         S, cams, ranges, values, rec, final_T, n_contrib, dL_dimages, grad2d, G,
                         order, (int)kAdjointAtomic, gmax, gfix, stats, n_inst, capacity);
    else
      hipLaunchKernelGGL((splat_backward_kernel<false, kS, kW>), grid, block, 0, st, segs,
                         seg_tstart, S, cams, ranges, values, rec, final_T, n_contrib, dL_dimages,
                         grad2d, G, order, (int)kAdjointAtomic, gmax, gfix, stats, n_inst, capacity);
    return;
  }
  // Deterministic: gmax [9][G] and gfix [9][G] must be zero on entry.  The first pass counts
  // the work when asked (the second walks the same pairs).
  if (count && stats)
    hipLaunchKernelGGL((splat_backward_kernel<true, kS, kW>), grid, block, 0, st, segs, seg_tstart,
                       S, cams, ranges, values, rec, final_T, n_contrib, dL_dimages, grad2d, G,
                       order, (int)kAdjointMax, gmax, gfix, stats, n_inst, capacity);
  else
    hipLaunchKernelGGL((splat_backward_kernel<false, kS, kW>), grid, block, 0, st, segs, seg_tstart,
                       S, cams, ranges, values, rec, final_T, n_contrib, dL_dimages, grad2d, G,
                       order, (int)kAdjointMax, gmax, gfix, stats, n_inst, capacity);
  hipLaunchKernelGGL((splat_backward_kernel<false, kS, kW>), grid, block, 0, st, segs, seg_tstart, S,
                     cams, ranges, values, rec, final_T, n_contrib, dL_dimages, grad2d, G, order,
                     (int)kAdjointFixed, gmax, gfix, stats, n_inst, capacity);
  if (G > 0)
    hipLaunchKernelGGL(fixed_to_float_kernel, dim3((unsigned)((9 * G + 255) / 256)), dim3(256), 0,
                       st, gmax, gfix, G, grad2d);
}

}  // namespace

// Tiles of 2^tsx x 2^tsy pixels: 16x16 (4, 4) or 32x32 (5, 5); any other shape is rejected.
hipError_t launch_splat_forward(hipStream_t st, const Seg* segs, const int64_t* seg_tstart, int S,
                                const DevCam* cams, int64_t n_tiles, const uint64_t* ranges,
                                const uint32_t* values, const SplatRec* rec, float* images,
                                float* final_T, int32_t* last_id, uint32_t* n_contrib,
                                unsigned long long* stats, const uint32_t* order,
                                uint32_t* tile_work, bool count, int tsx, int tsy,
                                const uint64_t* n_inst, uint64_t capacity) {
  if (n_tiles == 0) return hipSuccess;
  if (tsx == 5 && tsy == 5)        // four independent 16x16 wavefronts per tile
    splat_forward_dispatch<4, 2, 2>(st, segs, seg_tstart, S, cams, n_tiles, ranges, values, rec,
                                    images, final_T, last_id, n_contrib, stats, order, tile_work,
                                    count, n_inst, capacity);
  else if (tsx == 4 && tsy == 4)
    splat_forward_dispatch<4, 1, 1>(st, segs, seg_tstart, S, cams, n_tiles, ranges, values, rec,
                                    images, final_T, last_id, n_contrib, stats, order, tile_work,
                                    count, n_inst, capacity);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_splat_backward(hipStream_t st, const Seg* segs, const int64_t* seg_tstart, int S,
                                 const DevCam* cams, int64_t n_tiles, const uint64_t* ranges,
                                 const uint32_t* values, const SplatRec* rec, const float* final_T,
                                 const uint32_t* n_contrib, const float* dL_dimages,
                                 float* grad2d, int64_t G, const uint32_t* order, uint32_t* gmax,
                                 unsigned long long* gfix, unsigned long long* stats, bool count,
                                 int tsx, int tsy, const uint64_t* n_inst, uint64_t capacity) {
  if (n_tiles == 0) return hipSuccess;
  if (tsx == 5 && tsy == 5)        // two independent 16x32 wavefronts of eight slots per tile
    splat_backward_dispatch<8, 2>(st, segs, seg_tstart, S, cams, n_tiles, ranges, values, rec,
                                  final_T, n_contrib, dL_dimages, grad2d, G, order, gmax, gfix,
                                  stats, count, n_inst, capacity);
  else if (tsx == 4 && tsy == 4)
    splat_backward_dispatch<4, 1>(st, segs, seg_tstart, S, cams, n_tiles, ranges, values, rec,
                                  final_T, n_contrib, dL_dimages, grad2d, G, order, gmax, gfix,
                                  stats, count, n_inst, capacity);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_tile_order(hipStream_t st, const uint64_t* ranges, const uint32_t* work,
                             int64_t n_tiles, uint32_t* order) {
  if (n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(tile_order_kernel, dim3(1), dim3(kOrderThreads), 0, st, ranges, work, n_tiles,
                     order);
  return hipGetLastError();
}

GSC_DEBUG_FLAGS_READER(debug_flags_splat)

}  // namespace gsc
