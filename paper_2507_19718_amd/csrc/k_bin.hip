// k_bin.hip -- tile binning of depth-ordered Gaussians.
//
// The instance list of 3D Gaussian splatting is every (tile, Gaussian) pair sorted by the
// 64-bit key (tile << 32) | bits(depth), ties by id.  Here the depth digits are sorted once per
// Gaussian (k_sort.hip), and the tile digit is applied in a single stable counting pass whose
// histogram is computed from the Gaussians' tile rectangles, so no key or per-instance
// temporary is ever written: every instance costs one 4-byte id store.
//
//   count  : one workgroup per (segment, chunk of kChunk depth-ordered Gaussians, band of tile
//            rows).  The number of the chunk's rectangles covering each tile is a 2D prefix sum
//            of a difference array: each rectangle adds +1/-1 at its four corners (LDS
//            atomics), then the band is summed down its columns and along its rows.
//   scan   : per tile, an exclusive scan over chunks; then a scan over all tiles gives each
//            tile's [start, end) and the instance total.
//   place  : one workgroup per (segment, chunk, 16x16-tile region), one 16x4 block of tiles
//            per wavefront and one tile per lane; the wave walks the chunk's rectangles in depth
//            order and every covered lane appends the id to its tile's run, so within a tile
//            ids come out in (depth, id) order (details at the kernel).
//
// Optional list cut (frames): front-to-back blending stops at a pixel once its transmittance
// would fall below 1e-4, so the entries of a tile's list behind the point where every pixel of
// the tile has surely stopped are never read.  Each Gaussian carries a saturation core (the
// tiles where it multiplies every unterminated pixel's transmittance by at most 1 - o/2, see the
// projection) and its weight -ln(1 - o/2); the count pass also sums the weights per
// (chunk, tile), and the scan keeps, per tile, the chunks up to the first one at which the
// running weight reaches -ln(0.5e-4): from there on every pixel of the tile has stopped, with a
// factor 2 to spare for rounding.  Placement skips the later chunks, so the cut lists give the
// same splat forward and backward results as the full ones.
#include "gsc_dev.h"

namespace gsc {

namespace {

struct BinWork {          // per segment, for the workgroup -> work item maps
  int64_t region_base;    // global index of this segment's first 16x16-tile region
  int64_t count_start;    // first counting workgroup of this segment
  int64_t g_off;
  int64_t n;
  int64_t tile_base;
  int64_t ct_off;         // offset of this segment's [chunk][tile] counts
  int32_t TX, TY;         // tiles
  int32_t n_chunks;
  int32_t band_rows;      // tile rows per counting workgroup
  int32_t n_bands;
};

// Difference-array words per counting workgroup (48 KB of LDS): a band holds
// floor(kDiffWords / TX) tile rows.
constexpr int kDiffWords = 12288;

// -ln(0.5e-4) in the 2^-16 units of the saturation weights.
constexpr uint32_t kCutWeight = 649035u;

__global__ void __launch_bounds__(256) gather_rect_kernel(const int64_t* __restrict__ seg_gstart,
                                                          int S, int64_t G,
                                                          const uint32_t* __restrict__ sorted_ids,
                                                          const uint64_t* __restrict__ rect,
                                                          uint64_t* __restrict__ rect_sorted,
                                                          const uint64_t* __restrict__ core,
                                                          uint64_t* __restrict__ core_sorted) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G) return;
  const int s = find_segment(seg_gstart, S, i);
  const int64_t src = seg_gstart[s] + sorted_ids[i];
  rect_sorted[i] = rect[src];
  if (core) core_sorted[i] = core[src];
}

// Inclusive prefix sum over the 64 lanes by DPP: row shifts of 1, 2, 4 and 8 lanes (zero fill)
// scan each 16-lane row, then lane 15 of rows 0 and 2 is added to rows 1 and 3, and lane 31 to
// rows 2 and 3.  Every lane of the wavefront must be active.
__device__ __forceinline__ int wave_inclusive_scan(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
  return v;
}

// 2D prefix sum in place of a band's difference array D[R][TX] (down the columns, then along
// the rows, one wavefront per row).  Ends with a barrier.
__device__ __forceinline__ void band_prefix_sum(int32_t* D, int R, int TX) {
  for (int x = threadIdx.x; x < TX; x += 256) {
    int run = 0, y = 0;
    for (; y + 8 <= R; y += 8) {             // eight loads in flight, then the running sums
      int t[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) t[j] = D[(y + j) * TX + x];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        run += t[j];
        D[(y + j) * TX + x] = run;
      }
    }
    for (; y < R; ++y) {
      run += D[y * TX + x];
      D[y * TX + x] = run;
    }
  }
  __syncthreads();
  const int lane = __lane_id();
  for (int y = threadIdx.x >> 6; y < R; y += 4) {
    int carry = 0;
    for (int xb = 0; xb < TX; xb += 64) {
      const int x = xb + lane;
      const int v = wave_inclusive_scan((x < TX) ? D[y * TX + x] : 0);
      if (x < TX) D[y * TX + x] = carry + v;
      carry += __builtin_amdgcn_readlane(v, 63);
    }
  }
  __syncthreads();
}

// Adds w at the corners of the rectangle's part inside the band (rows b0 .. b0 + R - 1).
__device__ __forceinline__ void band_rect_add(int32_t* D, uint64_t r, int w, int b0, int R, int TX) {
  const int tx0 = (int)(r & 0xffffu), tx1 = (int)((r >> 16) & 0xffffu);
  const int ty0 = (int)((r >> 32) & 0xffffu), ty1 = (int)(r >> 48);
  if (tx0 > tx1) return;                         // culled (empty rectangle)
  const int y0 = max(ty0, b0) - b0, y1 = min(ty1, b0 + R - 1) - b0;
  if (y0 > y1) return;                           // outside the band
  const bool right = tx1 + 1 < TX, below = y1 + 1 < R;
  atomicAdd(&D[y0 * TX + tx0], w);
  if (right) atomicAdd(&D[y0 * TX + tx1 + 1], -w);
  if (below) {
    atomicAdd(&D[(y1 + 1) * TX + tx0], -w);
    if (right) atomicAdd(&D[(y1 + 1) * TX + tx1 + 1], w);
  }
}

// One workgroup per (segment, chunk, band of tile rows): counts[chunk][tile] = the number of the
// chunk's tile rectangles that contain the tile, for every tile of the band; with wsum, also
// wsum[chunk][tile] = the sum of the weights of the chunk's saturation cores that contain it.
__global__ void __launch_bounds__(256) bin_count_kernel(const BinWork* __restrict__ work,
                                                        const int64_t* __restrict__ block_start,
                                                        int S, int64_t total_blocks,
                                                        const uint64_t* __restrict__ rect_sorted,
                                                        uint32_t* __restrict__ counts,
                                                        const uint64_t* __restrict__ core_sorted,
                                                        uint32_t* __restrict__ wsum) {
  __shared__ int32_t D[kDiffWords];
  const int64_t blk = blockIdx.x;
  if (blk >= total_blocks) return;
  const int s = find_segment(block_start, S, blk);
  const BinWork W = work[s];
  const int64_t l = blk - W.count_start;
  const int band = (int)(l % W.n_bands);
  const int c = (int)(l / W.n_bands);
  const int TX = W.TX;
  const int b0 = band * W.band_rows;
  const int R = min(W.band_rows, W.TY - b0);
  const int words = R * TX;
  const int64_t g0 = (int64_t)c * kChunk;
  const int cnt_g = (int)((W.n - g0) < kChunk ? (W.n - g0) : kChunk);
  const int64_t out_off = W.ct_off + (int64_t)c * ((int64_t)TX * W.TY) + (int64_t)b0 * TX;
  for (int k = threadIdx.x; k < words; k += 256) D[k] = 0;
  __syncthreads();
  const uint64_t* rs = rect_sorted + W.g_off + g0;
  for (int k = threadIdx.x; k < cnt_g; k += 256) band_rect_add(D, rs[k], 1, b0, R, TX);
  __syncthreads();
  band_prefix_sum(D, R, TX);
  for (int k = threadIdx.x; k < words; k += 256) {
    counts[out_off + k] = (uint32_t)D[k];
    D[k] = 0;
  }
  if (!wsum) return;
  __syncthreads();
  const uint64_t* cs = core_sorted + W.g_off + g0;
  for (int k = threadIdx.x; k < cnt_g; k += 256) {
    const uint64_t c = cs[k];
    const int w = (int)(c >> 48);
    if (!w) continue;
    const uint64_t r = (c & 0x7ffull) | (((c >> 11) & 0x7ffull) << 16) |
                       (((c >> 22) & 0x7ffull) << 32) | (((c >> 33) & 0x7ffull) << 48);
    band_rect_add(D, r, w, b0, R, TX);
  }
  __syncthreads();
  band_prefix_sum(D, R, TX);
  for (int k = threadIdx.x; k < words; k += 256) wsum[out_off + k] = (uint32_t)D[k];
}

// Placement.  One workgroup per (segment, group of kPlaceChunks consecutive chunks, 16x16-tile
// region); wavefront w owns the region's 16x4 block of tiles in rows 4w..4w+3, lane t the
// block's tile (t & 15, t >> 4).  Chunk by chunk, the depth-ordered rectangles and ids are
// staged in LDS; each wave scans them 64 at a time and compacts, in order, the Gaussians whose
// rectangle overlaps its block into a small LDS queue; whenever 64 are queued it places them as
// a batch, lanes now holding Gaussians: for every tile of the batch's bounding box, the lanes
// whose rectangle covers it (a ballot) write their ids to consecutive positions of the tile's
// run (rank = number of covering lanes below), one coalesced store per tile, and the tile's
// cursor (kept in VGPR lane t) advances by their count.  A tile's runs for consecutive chunks
// are adjacent in the output, so the cursors and the queue carry over from one chunk of the
// group to the next.  Within a tile ids come out in (depth, id) order, and every store writes a
// contiguous stretch of the run.
constexpr int kRegion = 16;      // tiles per region side
constexpr int kQueue = 128;      // compaction queue entries per wave (a ring)
constexpr int kPlaceChunks = 1;  // chunks per placement workgroup
static_assert(kPlaceChunks == 1, "the list cut decides a tile's liveness once per workgroup");

__device__ __forceinline__ uint32_t lane_rank(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Places n <= 64 queued Gaussians (lane i holds entry i) into the runs of the wave's live tiles
// (bit t of `live_t`: tile (ox + (t & 15), oy + (t >> 4)), whose cursor lane t holds), all
// inside [bx0, bx1] x [by0, by1].
__device__ __forceinline__ void place_batch(uint32_t* __restrict__ values, uint64_t capacity,
                                            uint64_t& cur, int lane, int n, uint64_t r, uint32_t id,
                                            int ox, int oy, uint64_t live_t, int bx0, int by0,
                                            int bx1, int by1) {
  const bool live = lane < n;
  const uint32_t xr = (uint32_t)r, yr = (uint32_t)(r >> 32);
  const int tx0 = (int)(xr & 0xffffu), tx1 = (int)(xr >> 16);
  const int ty0 = (int)(yr & 0xffffu), ty1 = (int)(yr >> 16);
  // Bounding box of the batch inside the block (wave-uniform).
  int x0 = live ? max(tx0, bx0) : 0x7fff, x1 = live ? min(tx1, bx1) : -1;
  int y0 = live ? max(ty0, by0) : 0x7fff, y1 = live ? min(ty1, by1) : -1;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    x0 = min(x0, __shfl_xor(x0, off, 64));
    x1 = max(x1, __shfl_xor(x1, off, 64));
    y0 = min(y0, __shfl_xor(y0, off, 64));
    y1 = max(y1, __shfl_xor(y1, off, 64));
  }
  x0 = __builtin_amdgcn_readfirstlane(x0);
  x1 = __builtin_amdgcn_readfirstlane(x1);
  y0 = __builtin_amdgcn_readfirstlane(y0);
  y1 = __builtin_amdgcn_readfirstlane(y1);
  for (int ty = y0; ty <= y1; ++ty) {
    const bool rowin = live && ty0 <= ty && ty <= ty1;
    for (int tx = x0; tx <= x1; ++tx) {
      const bool cov = rowin && tx0 <= tx && tx <= tx1;
      const int t = (tx - ox) + 16 * (ty - oy);
      if (!((live_t >> t) & 1ull)) continue;
      const uint64_t m = __ballot(cov);
      if (m == 0ull) continue;
      const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)cur, t);
      const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(cur >> 32), t);
      const uint64_t base = ((uint64_t)hi << 32) | lo;
      const uint64_t at = base + lane_rank(m);
      if (cov && GSC_DCHECK(at < capacity, kDbgInstanceStore)) values[at] = id;
      cur = (lane == t) ? base + (uint64_t)__popcll(m) : cur;
    }
  }
}

__global__ void __launch_bounds__(256) bin_place_kernel(const BinWork* __restrict__ work,
                                                        const int64_t* __restrict__ seg_rbase,
                                                        int S, int64_t n_regions,
                                                        const uint64_t* __restrict__ region_start,
                                                        const uint64_t* __restrict__ n_blocks,
                                                        const uint32_t* __restrict__ sorted_ids,
                                                        const uint64_t* __restrict__ rect_sorted,
                                                        const uint32_t* __restrict__ counts,
                                                        const uint64_t* __restrict__ tile_start,
                                                        const uint64_t* __restrict__ n_instances,
                                                        uint64_t capacity,
                                                        uint32_t* __restrict__ values,
                                                        const int32_t* __restrict__ cut) {
  __shared__ uint64_t sh_rect[kChunk];
  __shared__ uint32_t sh_id[kChunk];
  __shared__ uint64_t q_rect[4][kQueue];
  __shared__ uint32_t q_id[4][kQueue];
  // Workgroups are packed region by region, each region's chunks [0, region_n) consecutively:
  // consecutive workgroups (which the dispatcher spreads over the XCDs round-robin) take
  // different depth slices of the same region, so every XCD gets a share of the heavily
  // covered central regions, and chunks no tile of a region needs get no workgroup.
  const uint64_t blk = blockIdx.x;
  if (blk >= *n_blocks) return;
  if (*n_instances > capacity) return;
  const int lane = __lane_id();
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // uniform per wave
  const int64_t g = find_segment(region_start, (int)n_regions, blk);
  const int s = find_segment(seg_rbase, S, g);
  const BinWork W = work[s];
  const int RX = (W.TX + kRegion - 1) / kRegion;
  const int region = (int)(g - W.region_base);
  const int rx = region % RX, ry = region / RX;
  const int c0 = (int)(blk - region_start[g]);
  const int c1 = c0 + 1;
  const int ox = rx * kRegion, oy = ry * kRegion + 4 * wave;   // the wave's block origin
  int bx0 = ox, by0 = oy;
  int bx1 = min(bx0 + kRegion, W.TX) - 1, by1 = min(by0 + 4, W.TY) - 1;
  // Lane t's tile cursor: where the tile's run continues (first, chunk c0's run).  With a list
  // cut, only the tiles whose lists still take chunk c0 are live.
  uint64_t cur = 0ull;
  bool tile_live = false;
  {
    const int col = bx0 + (lane & 15), row = by0 + (lane >> 4);
    if (by0 < W.TY && col <= bx1 && row <= by1) {
      const int64_t tl = (int64_t)row * W.TX + col;
      cur = tile_start[W.tile_base + tl] +
            counts[W.ct_off + (int64_t)c0 * ((int64_t)W.TX * W.TY) + tl];
      tile_live = !cut || c0 <= cut[W.tile_base + tl];
    }
  }
  const uint64_t live_tiles = __ballot(tile_live);
  const bool wave_live = live_tiles != 0ull;
  if (!__syncthreads_or(wave_live)) return;    // every tile of the region is cut here
  if (wave_live && cut) {
    // Shrink the block to the bounding box of its live tiles (lane t = tile (t & 15, t >> 4)).
    int lx0 = tile_live ? (lane & 15) : 16, lx1 = tile_live ? (lane & 15) : -1;
    int ly0 = tile_live ? (lane >> 4) : 4, ly1 = tile_live ? (lane >> 4) : -1;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      lx0 = min(lx0, __shfl_xor(lx0, off, 64));
      lx1 = max(lx1, __shfl_xor(lx1, off, 64));
      ly0 = min(ly0, __shfl_xor(ly0, off, 64));
      ly1 = max(ly1, __shfl_xor(ly1, off, 64));
    }
    bx0 = ox + __builtin_amdgcn_readfirstlane(lx0);
    bx1 = ox + __builtin_amdgcn_readfirstlane(lx1);
    by0 = oy + __builtin_amdgcn_readfirstlane(ly0);
    by1 = oy + __builtin_amdgcn_readfirstlane(ly1);
  }
  uint64_t* qr = q_rect[wave];
  uint32_t* qi = q_id[wave];
  int head = 0, tail = 0;                 // queue: entries [head, tail), modulo kQueue
  for (int c = c0; c < c1; ++c) {
    const int64_t g0 = (int64_t)c * kChunk;
    const int cnt_g = (int)((W.n - g0) < kChunk ? (W.n - g0) : kChunk);
    const uint64_t* rs = rect_sorted + W.g_off + g0;
    const uint32_t* ids = sorted_ids + W.g_off + g0;
    __syncthreads();                       // the previous chunk is consumed
    for (int k = threadIdx.x; k < cnt_g; k += 256) {
      sh_rect[k] = rs[k];
      sh_id[k] = ids[k];
    }
    __syncthreads();
    if (!wave_live) continue;
    for (int j = 0; j < cnt_g; j += 64) {
      const int k = j + lane;
      uint64_t r = 0x0000000100000001ull;   // empty rectangle
      uint32_t id = 0u;
      if (k < cnt_g) {
        r = sh_rect[k];
        id = sh_id[k];
      }
      const uint32_t xr = (uint32_t)r, yr = (uint32_t)(r >> 32);
      const int tx0 = (int)(xr & 0xffffu), tx1 = (int)(xr >> 16);
      const int ty0 = (int)(yr & 0xffffu), ty1 = (int)(yr >> 16);
      const bool hit = (tx0 <= tx1) && (tx0 <= bx1) && (tx1 >= bx0) && (ty0 <= by1) && (ty1 >= by0);
      const uint64_t m = __ballot(hit);
      if (hit) {
        const int slot = (tail + (int)lane_rank(m)) & (kQueue - 1);
        qr[slot] = r;
        qi[slot] = id;
      }
      tail += __popcll(m);
      (void)GSC_DCHECK(tail - head <= kQueue, kDbgPlaceQueue);
      while (tail - head >= 64) {
        __builtin_amdgcn_wave_barrier();
        const uint64_t qrr = qr[(head + lane) & (kQueue - 1)];
        const uint32_t qid = qi[(head + lane) & (kQueue - 1)];
        head += 64;
        place_batch(values, capacity, cur, lane, 64, qrr, qid, ox, oy, live_tiles, bx0, by0, bx1,
                    by1);
      }
    }
  }
  if (wave_live && tail > head) {          // the last, partial batch
    const int n = tail - head;
    __builtin_amdgcn_wave_barrier();
    uint64_t qrr = 0x0000000100000001ull;
    uint32_t qid = 0u;
    if (lane < n) {
      qrr = qr[(head + lane) & (kQueue - 1)];
      qid = qi[(head + lane) & (kQueue - 1)];
    }
    place_batch(values, capacity, cur, lane, n, qrr, qid, ox, oy, live_tiles, bx0, by0, bx1, by1);
  }
}

// Per tile: exclusive scan over chunks (in place) and the tile total.  With wsum, chunks after
// the one at which the running saturation weight reaches kCutWeight add nothing.  cut[tile] is
// the last kept chunk that has entries for the tile (-1: none), so placement can skip the rest.
//
// A workgroup takes 64 consecutive tiles (lane = tile, so every load and store is coalesced
// over tiles) and splits each tile's chunks into kScanParts contiguous parts, one per wave, so
// the launch has enough waves to hide the loads.  Three passes over the parts, with the parts'
// sums combined in LDS between them: (A) saturation weights, whose prefix over the parts tells
// each part the weight before it and so where the cut falls; (B) the counts of the chunks up to
// the cut, whose prefix gives each part its starting offset; (C) the exclusive scan written in
// place.  The result equals the sequential scan over the chunks.
constexpr int kScanParts = 16;

__global__ void __launch_bounds__(64 * kScanParts) chunk_scan_kernel(
    const BinWork* __restrict__ work, const int64_t* __restrict__ seg_tstart, int S,
    int64_t n_tiles, uint32_t* __restrict__ counts, uint32_t* __restrict__ tile_total,
    const uint32_t* __restrict__ wsum, int32_t* __restrict__ cut, int32_t* __restrict__ region_n) {
  __shared__ uint32_t sh_w[kScanParts][64];   // weight, then count, sums of each part
  __shared__ int32_t sh_nz[kScanParts][64];   // each part's last kept chunk with entries
  const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
  const int64_t t = (int64_t)blockIdx.x * 64 + lane;
  const bool live = t < n_tiles;
  BinWork W{};
  int64_t lt = 0, T = 1;
  int c0 = 0, c1 = 0;
  if (live) {
    W = work[find_segment(seg_tstart, S, t)];
    lt = t - W.tile_base;
    T = (int64_t)W.TX * W.TY;
    const int q = (W.n_chunks + kScanParts - 1) / kScanParts;
    c0 = min(part * q, W.n_chunks);
    c1 = min(c0 + q, W.n_chunks);
  }
  uint32_t* col = counts + W.ct_off + lt;            // chunk c at col[c * T]
  const uint32_t* wcol = wsum ? wsum + W.ct_off + lt : nullptr;
  constexpr int kAhead = 8;
  // (A) the part's saturation weight.
  uint32_t wpart = 0u;
  if (wcol) {
    for (int cb = c0; cb < c1; cb += kAhead) {
      uint32_t ws[kAhead];
#pragma unroll
      for (int j = 0; j < kAhead; ++j) ws[j] = (cb + j < c1) ? wcol[(int64_t)(cb + j) * T] : 0u;
#pragma unroll
      for (int j = 0; j < kAhead; ++j) wpart += ws[j];
    }
  }
  sh_w[part][lane] = wpart;
  __syncthreads();
  uint32_t weight = 0u;                      // the weight of the chunks before this part
  for (int p = 0; p < part; ++p) weight += sh_w[p][lane];
  __syncthreads();
  // (B) the counts of the part's chunks up to the cut, and its last kept chunk with entries.
  // `last` is the cut chunk once the running weight reaches kCutWeight (inclusive).
  int last = (wcol && weight >= kCutWeight) ? c0 - 1 : W.n_chunks - 1;
  uint32_t cpart = 0u;
  int last_nz = -1;
  {
    uint32_t wr = weight;
    for (int cb = c0; cb < c1 && cb <= last; cb += kAhead) {
      uint32_t v[kAhead], ws[kAhead];
#pragma unroll
      for (int j = 0; j < kAhead; ++j) {
        const bool in = cb + j < c1;
        v[j] = in ? col[(int64_t)(cb + j) * T] : 0u;
        ws[j] = (in && wcol) ? wcol[(int64_t)(cb + j) * T] : 0u;
      }
#pragma unroll
      for (int j = 0; j < kAhead; ++j) {
        const int c = cb + j;
        if (c >= c1 || c > last) break;
        cpart += v[j];
        if (v[j]) last_nz = c;
        wr += ws[j];
        if (wcol && wr >= kCutWeight) last = c;
      }
    }
  }
  sh_w[part][lane] = cpart;
  sh_nz[part][lane] = last_nz;
  __syncthreads();
  uint32_t run = 0u, total = 0u;
  int nz = -1;
  for (int p = 0; p < kScanParts; ++p) {
    const uint32_t x = sh_w[p][lane];
    if (p < part) run += x;
    total += x;
    nz = max(nz, sh_nz[p][lane]);
  }
  // (C) the exclusive scan, in place; chunks after the cut keep the offset of the tile's end.
  for (int cb = c0; cb < c1; cb += kAhead) {
    uint32_t v[kAhead];
#pragma unroll
    for (int j = 0; j < kAhead; ++j) v[j] = (cb + j < c1 && cb + j <= last) ? col[(int64_t)(cb + j) * T] : 0u;
#pragma unroll
    for (int j = 0; j < kAhead; ++j) {
      const int c = cb + j;
      if (c >= c1) break;
      col[(int64_t)c * T] = run;
      run += v[j];
    }
  }
  if (!live || part != 0) return;
  tile_total[t] = total;
  cut[t] = nz;
  // The region's chunk count for placement: 1 + the largest cut of its tiles (zeroed before).
  const int RX = (W.TX + kRegion - 1) / kRegion;
  const int tx = (int)(lt % W.TX), ty = (int)(lt / W.TX);
  if (nz >= 0)
    atomicMax(&region_n[W.region_base + (int64_t)(ty / kRegion) * RX + tx / kRegion], nz + 1);
}

// Exclusive scan of u32 into u64, three phases over blocks of 1024 items.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanBlock = kScanThreads * kScanItems;

__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* tmp, uint64_t* total) {
  const int tid = threadIdx.x;
  tmp[tid] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const uint64_t a = (tid >= off) ? tmp[tid - off] : 0ull;
    __syncthreads();
    tmp[tid] += a;
    __syncthreads();
  }
  const uint64_t incl = tmp[tid];
  *total = tmp[kScanThreads - 1];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(kScanThreads) scan_reduce_kernel(const uint32_t* __restrict__ in,
                                                                   int64_t n,
                                                                   uint64_t* __restrict__ partial) {
  __shared__ uint64_t tmp[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  uint64_t s = 0ull;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
    if (i < n) s += in[i];
  }
  uint64_t total;
  block_exclusive_scan(s, tmp, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Single workgroup: region_start[g] = sum of region_n over the regions before g, total to *sum.
__global__ void __launch_bounds__(kScanThreads) region_scan_kernel(const int32_t* __restrict__ region_n,
                                                                   int64_t n,
                                                                   uint64_t* __restrict__ region_start,
                                                                   uint64_t* __restrict__ sum) {
  __shared__ uint64_t tmp[kScanThreads];
  uint64_t carry = 0ull;
  for (int64_t base = 0; base < n; base += kScanThreads) {
    const int64_t i = base + threadIdx.x;
    const uint64_t v = (i < n) ? (uint64_t)region_n[i] : 0ull;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan(v, tmp, &total);
    if (i < n) region_start[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) *sum = carry;
}

// Single workgroup: exclusive scan of the block partials (any count), total to *sum.
__global__ void __launch_bounds__(kScanThreads) scan_partials_kernel(uint64_t* __restrict__ partial,
                                                                     int64_t nb,
                                                                     uint64_t* __restrict__ sum) {
  __shared__ uint64_t tmp[kScanThreads];
  uint64_t carry = 0ull;
  for (int64_t base = 0; base < nb; base += kScanThreads) {
    const int64_t i = base + threadIdx.x;
    const uint64_t v = (i < nb) ? partial[i] : 0ull;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan(v, tmp, &total);
    if (i < nb) partial[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) *sum = carry;
}

__global__ void __launch_bounds__(kScanThreads) scan_down_kernel(const uint32_t* __restrict__ in,
                                                                 int64_t n,
                                                                 const uint64_t* __restrict__ partial,
                                                                 uint64_t* __restrict__ out,
                                                                 uint64_t* __restrict__ ranges) {
  __shared__ uint64_t tmp[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  uint32_t v[kScanItems];
  uint64_t s = 0ull;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
    v[k] = (i < n) ? in[i] : 0u;
    s += v[k];
  }
  uint64_t total;
  uint64_t run = partial[blockIdx.x] + block_exclusive_scan(s, tmp, &total);
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
    if (i < n) {
      out[i] = run;
      ranges[2 * i] = v[k] ? run : 0ull;
      ranges[2 * i + 1] = v[k] ? run + v[k] : 0ull;
    }
    run += v[k];
  }
}

// 64-bit keys of the binned instances, for inspection: (global tile << 32) | bits(depth).
__global__ void __launch_bounds__(256) keys_kernel(const int64_t* __restrict__ seg_tstart, int S,
                                                   const int64_t* __restrict__ seg_goff,
                                                   int64_t n_tiles, const uint64_t* __restrict__ tile_start,
                                                   const uint64_t* __restrict__ n_instances,
                                                   const uint32_t* __restrict__ values,
                                                   const uint32_t* __restrict__ depth_key,
                                                   uint64_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)*n_instances) return;
  // Last tile whose start <= i (empty tiles share their successor's start).
  int64_t lo = 0, hi = n_tiles - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (tile_start[mid] <= (uint64_t)i) lo = mid; else hi = mid - 1;
  }
  const int s = find_segment(seg_tstart, S, lo);
  keys[i] = ((uint64_t)lo << 32) | (uint64_t)depth_key[seg_goff[s] + values[i]];
}

__global__ void __launch_bounds__(256) view_kernel(int64_t G, const SplatRec* __restrict__ rec,
                                                   const uint32_t* __restrict__ tiles,
                                                   int32_t* __restrict__ window,
                                                   float* __restrict__ screen) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G) return;
  const SplatRec r = rec[i];
  const uint32_t wx = __float_as_uint(r.q2.y), wy = __float_as_uint(r.q2.z);
  const bool live = tiles[i] != 0u;
  window[4 * i + 0] = live ? (int32_t)(wx & 0xffffu) : 0;
  window[4 * i + 1] = live ? (int32_t)(wx >> 16) : 0;
  window[4 * i + 2] = live ? (int32_t)(wy & 0xffffu) : 0;
  window[4 * i + 3] = live ? (int32_t)(wy >> 16) : 0;
  screen[6 * i + 0] = r.q0.x;
  screen[6 * i + 1] = r.q0.y;
  screen[6 * i + 2] = r.q0.z;
  screen[6 * i + 3] = r.q0.w;
  screen[6 * i + 4] = r.q1.x;
  screen[6 * i + 5] = r.q1.y;
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

size_t bin_work_bytes(int S) { return sizeof(BinWork) * (size_t)S + 2 * sizeof(int64_t) * (size_t)S; }

// Host: fills [BinWork x S][int64 first region x S][int64 count start x S]; returns the
// placement workgroup count when every region visits every chunk (an upper bound), the counting
// workgroup count, the [chunk][tile] count total and the region count.
int64_t bin_fill_work(void* host, const Seg* segs, int S, int64_t* total_chunk_tiles,
                      int64_t* total_count_blocks, int64_t* total_regions) {
  BinWork* W = (BinWork*)host;
  int64_t* ws = (int64_t*)(W + S);
  int64_t* cs = ws + S;
  int64_t waves = 0, ct = 0, cblk = 0, regions = 0;
  for (int s = 0; s < S; ++s) {
    const Seg& g = segs[s];
    W[s].region_base = regions;
    W[s].count_start = cblk;
    W[s].g_off = g.g_off;
    W[s].n = g.n;
    W[s].tile_base = g.tile_base;
    W[s].ct_off = ct;
    W[s].TX = g.TX;
    W[s].TY = g.TY;
    W[s].n_chunks = (int32_t)((g.n + kChunk - 1) / kChunk);
    W[s].band_rows = std::max(1, std::min(g.TY, kDiffWords / std::max(g.TX, 1)));
    W[s].n_bands = (g.TY + W[s].band_rows - 1) / W[s].band_rows;
    ws[s] = regions;
    cs[s] = cblk;
    const int64_t nreg = (int64_t)((g.TY + kRegion - 1) / kRegion) * ((g.TX + kRegion - 1) / kRegion);
    regions += nreg;
    waves += (int64_t)W[s].n_chunks * nreg;
    cblk += (int64_t)W[s].n_chunks * W[s].n_bands;
    ct += (int64_t)W[s].n_chunks * g.TX * g.TY;
  }
  *total_chunk_tiles = ct;
  *total_count_blocks = cblk;
  *total_regions = regions;
  return waves;
}

hipError_t launch_gather_rect(hipStream_t st, const int64_t* seg_gstart, int S, int64_t G,
                              const uint32_t* sorted_ids, const uint64_t* rect,
                              uint64_t* rect_sorted, const uint64_t* core, uint64_t* core_sorted) {
  if (G == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_rect_kernel, dim3(nblk(G, 256)), dim3(256), 0, st, seg_gstart, S, G,
                     sorted_ids, rect, rect_sorted, core, core_sorted);
  return hipGetLastError();
}

hipError_t launch_bin_count(hipStream_t st, const void* work_dev, int S, int64_t total_blocks,
                            const uint64_t* rect_sorted, uint32_t* counts,
                            const uint64_t* core_sorted, uint32_t* wsum) {
  if (total_blocks == 0) return hipSuccess;
  const BinWork* W = (const BinWork*)work_dev;
  const int64_t* cs = (const int64_t*)(W + S) + S;
  hipLaunchKernelGGL(bin_count_kernel, dim3((unsigned)total_blocks), dim3(256), 0, st, W, cs, S,
                     total_blocks, rect_sorted, counts, core_sorted, wsum);
  return hipGetLastError();
}

hipError_t launch_bin_scan(hipStream_t st, const void* work_dev, int S, const int64_t* seg_tstart,
                           int64_t n_tiles, uint32_t* counts, uint32_t* tile_total,
                           uint64_t* partial, uint64_t* tile_start, uint64_t* ranges,
                           uint64_t* n_instances, const uint32_t* wsum, int32_t* cut,
                           int32_t* region_n) {
  const BinWork* W = (const BinWork*)work_dev;
  if (n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(chunk_scan_kernel, dim3(nblk(n_tiles, 64)), dim3(64 * kScanParts), 0, st, W,
                     seg_tstart, S, n_tiles, counts, tile_total, wsum, cut, region_n);
  const int64_t nb = (n_tiles + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, st, tile_total,
                     n_tiles, partial);
  hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(kScanThreads), 0, st, partial, nb,
                     n_instances);
  hipLaunchKernelGGL(scan_down_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, st, tile_total,
                     n_tiles, partial, tile_start, ranges);
  return hipGetLastError();
}

size_t bin_scan_partials(int64_t n_tiles) { return (size_t)((n_tiles + kScanBlock - 1) / kScanBlock) + 1; }

hipError_t launch_bin_regions(hipStream_t st, int64_t n_regions, const int32_t* region_n,
                              uint64_t* region_start, uint64_t* n_blocks) {
  if (n_regions == 0) return hipSuccess;
  hipLaunchKernelGGL(region_scan_kernel, dim3(1), dim3(kScanThreads), 0, st, region_n, n_regions,
                     region_start, n_blocks);
  return hipGetLastError();
}

hipError_t launch_bin_place(hipStream_t st, const void* work_dev, int S, int64_t n_regions,
                            const uint64_t* region_start, const uint64_t* n_blocks,
                            int64_t grid_blocks, const uint32_t* sorted_ids,
                            const uint64_t* rect_sorted, const uint32_t* counts,
                            const uint64_t* tile_start, const uint64_t* n_instances,
                            uint64_t capacity, uint32_t* values, const int32_t* cut) {
  if (grid_blocks == 0) return hipSuccess;
  if (grid_blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const BinWork* W = (const BinWork*)work_dev;
  const int64_t* ws = (const int64_t*)(W + S);
  hipLaunchKernelGGL(bin_place_kernel, dim3((unsigned)grid_blocks), dim3(256), 0, st, W, ws, S,
                     n_regions, region_start, n_blocks, sorted_ids, rect_sorted, counts, tile_start,
                     n_instances, capacity, values, cut);
  return hipGetLastError();
}

hipError_t launch_binning_keys(hipStream_t st, const int64_t* seg_tstart, int S,
                               const int64_t* seg_goff, int64_t n_tiles, const uint64_t* tile_start,
                               const uint64_t* n_instances, uint64_t n_host,
                               const uint32_t* values, const uint32_t* depth_key, uint64_t* keys) {
  if (n_host == 0) return hipSuccess;
  hipLaunchKernelGGL(keys_kernel, dim3(nblk((int64_t)n_host, 256)), dim3(256), 0, st, seg_tstart, S,
                     seg_goff, n_tiles, tile_start, n_instances, values, depth_key, keys);
  return hipGetLastError();
}

hipError_t launch_view(hipStream_t st, int64_t G, const SplatRec* rec, const uint32_t* tiles,
                       int32_t* window, float* screen) {
  if (G == 0) return hipSuccess;
  hipLaunchKernelGGL(view_kernel, dim3(nblk(G, 256)), dim3(256), 0, st, G, rec, tiles, window,
                     screen);
  return hipGetLastError();
}

GSC_DEBUG_FLAGS_READER(debug_flags_bin)

}  // namespace gsc
