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
//   place  : one workgroup per (segment, chunk, 4 tile rows, block of 64 tile columns); the
//            chunk is staged in LDS, each wavefront owns a row and its lanes own tile columns.
//            The wave tests 64 Gaussians at a time against its row (ballot), then walks the hits
//            in depth order; each lane appends the ids covering its column at its cursor, so
//            within a tile ids come out in (depth, id) order.
#include "gsc_dev.h"

namespace gsc {

namespace {

struct BinWork {          // per segment, for the workgroup -> work item maps
  int64_t wave_start;     // first placement workgroup of this segment
  int64_t count_start;    // first counting workgroup of this segment
  int64_t g_off;
  int64_t n;
  int64_t tile_base;
  int64_t ct_off;         // offset of this segment's [chunk][tile] counts
  int32_t TX, TY, CB;     // tiles, column blocks of 64
  int32_t n_chunks;
  int32_t band_rows;      // tile rows per counting workgroup
  int32_t n_bands;
};

// Difference-array words per counting workgroup (48 KB of LDS): a band holds
// floor(kDiffWords / TX) tile rows.
constexpr int kDiffWords = 12288;

__global__ void __launch_bounds__(256) gather_rect_kernel(const int64_t* __restrict__ seg_gstart,
                                                          int S, int64_t G,
                                                          const uint32_t* __restrict__ sorted_ids,
                                                          const uint64_t* __restrict__ rect,
                                                          uint64_t* __restrict__ rect_sorted) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G) return;
  const int s = find_segment(seg_gstart, S, i);
  rect_sorted[i] = rect[seg_gstart[s] + sorted_ids[i]];
}

// One workgroup per (segment, chunk, band of tile rows): counts[chunk][tile] = the number of the
// chunk's tile rectangles that contain the tile, for every tile of the band.
__global__ void __launch_bounds__(256) bin_count_kernel(const BinWork* __restrict__ work,
                                                        const int64_t* __restrict__ block_start,
                                                        int S, int64_t total_blocks,
                                                        const uint64_t* __restrict__ rect_sorted,
                                                        uint32_t* __restrict__ counts) {
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
  for (int k = threadIdx.x; k < words; k += 256) D[k] = 0;
  __syncthreads();
  const int64_t g0 = (int64_t)c * kChunk;
  const int cnt_g = (int)((W.n - g0) < kChunk ? (W.n - g0) : kChunk);
  const uint64_t* rs = rect_sorted + W.g_off + g0;
  for (int k = threadIdx.x; k < cnt_g; k += 256) {
    const uint64_t r = rs[k];
    const int tx0 = (int)(r & 0xffffu), tx1 = (int)((r >> 16) & 0xffffu);
    const int ty0 = (int)((r >> 32) & 0xffffu), ty1 = (int)(r >> 48);
    if (tx0 > tx1) continue;                       // culled (empty rectangle)
    const int y0 = max(ty0, b0) - b0, y1 = min(ty1, b0 + R - 1) - b0;
    if (y0 > y1) continue;                         // outside the band
    const bool right = tx1 + 1 < TX, below = y1 + 1 < R;
    atomicAdd(&D[y0 * TX + tx0], 1);
    if (right) atomicAdd(&D[y0 * TX + tx1 + 1], -1);
    if (below) {
      atomicAdd(&D[(y1 + 1) * TX + tx0], -1);
      if (right) atomicAdd(&D[(y1 + 1) * TX + tx1 + 1], 1);
    }
  }
  __syncthreads();
  for (int x = threadIdx.x; x < TX; x += 256) {    // down the columns
    int run = 0;
    for (int y = 0; y < R; ++y) {
      run += D[y * TX + x];
      D[y * TX + x] = run;
    }
  }
  __syncthreads();
  const int lane = __lane_id();
  for (int y = threadIdx.x >> 6; y < R; y += 4) {  // along the rows, one wavefront per row
    int carry = 0;
    for (int xb = 0; xb < TX; xb += 64) {
      const int x = xb + lane;
      int v = (x < TX) ? D[y * TX + x] : 0;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
      }
      if (x < TX) D[y * TX + x] = carry + v;
      carry += __shfl(v, 63, 64);
    }
  }
  __syncthreads();
  uint32_t* out = counts + W.ct_off + (int64_t)c * ((int64_t)TX * W.TY) + (int64_t)b0 * TX;
  for (int k = threadIdx.x; k < words; k += 256) out[k] = (uint32_t)D[k];
}

// One workgroup per (segment, chunk, group of 4 tile rows, block of 64 tile columns); wave w
// owns row 4 g + w.  The chunk's depth-ordered rects and ids are staged in LDS once and scanned
// by all four waves.  Each lane writes its tile's run for the chunk: ids before the first
// 16-byte boundary one by one, then four at a time from registers (one 16-byte store per four
// instances), the remainder at the end.
constexpr int kRowsPerGroup = 4;

__global__ void __launch_bounds__(256) bin_place_kernel(const BinWork* __restrict__ work,
                                                        const int64_t* __restrict__ block_start,
                                                        int S, int64_t total_blocks,
                                                        const uint32_t* __restrict__ sorted_ids,
                                                        const uint64_t* __restrict__ rect_sorted,
                                                        const uint32_t* __restrict__ counts,
                                                        const uint64_t* __restrict__ tile_start,
                                                        const uint64_t* __restrict__ n_instances,
                                                        uint64_t capacity,
                                                        uint32_t* __restrict__ values) {
  __shared__ uint64_t sh_rect[kChunk];
  __shared__ uint32_t sh_id[kChunk];
  const int64_t blk = blockIdx.x;
  if (blk >= total_blocks) return;
  if (*n_instances > capacity) return;
  const int lane = __lane_id();
  const int wave = threadIdx.x >> 6;
  const int s = find_segment(block_start, S, blk);
  const BinWork W = work[s];
  int64_t l = blk - W.wave_start;
  const int cb = (int)(l % W.CB);
  l /= W.CB;
  const int RG = (W.TY + kRowsPerGroup - 1) / kRowsPerGroup;
  const int rg = (int)(l % RG);
  const int c = (int)(l / RG);
  const int64_t g0 = (int64_t)c * kChunk;
  const int cnt_g = (int)((W.n - g0) < kChunk ? (W.n - g0) : kChunk);
  const uint64_t* rs = rect_sorted + W.g_off + g0;
  const uint32_t* ids = sorted_ids + W.g_off + g0;
  for (int k = threadIdx.x; k < cnt_g; k += 256) {
    sh_rect[k] = rs[k];
    sh_id[k] = ids[k];
  }
  __syncthreads();
  const int ty = rg * kRowsPerGroup + wave;
  if (ty >= W.TY) return;
  const int cbs = cb * 64, cbe = cbs + 63;
  const int col = cbs + lane;
  const bool col_ok = col < W.TX;
  const int64_t T = (int64_t)W.TX * W.TY;
  uint64_t cursor = 0ull;
  if (col_ok)
    cursor = tile_start[W.tile_base + (int64_t)ty * W.TX + col] +
             counts[W.ct_off + (int64_t)c * T + (int64_t)ty * W.TX + col];
  const uint64_t head_end = (cursor + 3ull) & ~3ull;   // first 16-byte boundary of the run
  uint32_t q0 = 0u, q1 = 0u, q2 = 0u, q3 = 0u;          // ids of [cursor & ~3, cursor)
  for (int j = 0; j < cnt_g; j += 64) {
    const int k = j + lane;
    uint64_t r = 0x0000000100000001ull;
    uint32_t my_id = 0u;
    if (k < cnt_g) {
      r = sh_rect[k];
      my_id = sh_id[k];
    }
    const uint32_t xr = (uint32_t)r;
    const int tx0 = (int)(xr & 0xffffu), tx1 = (int)(xr >> 16);
    const int ty0 = (int)((r >> 32) & 0xffffu), ty1 = (int)(r >> 48);
    const bool hit = (ty0 <= ty) && (ty <= ty1) && (tx0 <= cbe) && (tx1 >= cbs) && (tx0 <= tx1);
    uint64_t mask = __ballot(hit);
    while (mask) {
      const int b = __builtin_ctzll(mask);
      mask &= mask - 1ull;
      const uint32_t hx = (uint32_t)__builtin_amdgcn_readlane((int)xr, b);
      const uint32_t id = (uint32_t)__builtin_amdgcn_readlane((int)my_id, b);
      const int hx0 = (int)(hx & 0xffffu), hx1 = (int)(hx >> 16);
      if (col >= hx0 && col <= hx1) {
        if (cursor < head_end) {
          values[cursor] = id;
        } else {
          const uint32_t slot = (uint32_t)cursor & 3u;
          q0 = slot == 0u ? id : q0;
          q1 = slot == 1u ? id : q1;
          q2 = slot == 2u ? id : q2;
          q3 = slot == 3u ? id : q3;
          if (slot == 3u) *(uint4*)(values + (cursor - 3ull)) = make_uint4(q0, q1, q2, q3);
        }
        ++cursor;
      }
    }
  }
  if (cursor > head_end) {   // then cursor & ~3 >= head_end: flush the partial group
    const uint64_t base = cursor & ~3ull;
    const uint32_t n = (uint32_t)cursor & 3u;
    if (n > 0u) values[base] = q0;
    if (n > 1u) values[base + 1] = q1;
    if (n > 2u) values[base + 2] = q2;
  }
}

// Per tile: exclusive scan over chunks (in place) and the tile total.
__global__ void __launch_bounds__(256) chunk_scan_kernel(const BinWork* __restrict__ work,
                                                         const int64_t* __restrict__ seg_tstart,
                                                         int S, int64_t n_tiles,
                                                         uint32_t* __restrict__ counts,
                                                         uint32_t* __restrict__ tile_total) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const int s = find_segment(seg_tstart, S, t);
  const BinWork W = work[s];
  const int64_t lt = t - W.tile_base;
  const int64_t T = (int64_t)W.TX * W.TY;
  uint32_t run = 0u;
  for (int c = 0; c < W.n_chunks; ++c) {
    const int64_t k = W.ct_off + (int64_t)c * T + lt;
    const uint32_t v = counts[k];
    counts[k] = run;
    run += v;
  }
  tile_total[t] = run;
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

// Host: fills [BinWork x S][int64 place start x S][int64 count start x S]; returns the placement
// workgroup count, the counting workgroup count and the [chunk][tile] count total.
int64_t bin_fill_work(void* host, const Seg* segs, int S, int64_t* total_chunk_tiles,
                      int64_t* total_count_blocks) {
  BinWork* W = (BinWork*)host;
  int64_t* ws = (int64_t*)(W + S);
  int64_t* cs = ws + S;
  int64_t waves = 0, ct = 0, cblk = 0;
  for (int s = 0; s < S; ++s) {
    const Seg& g = segs[s];
    W[s].wave_start = waves;
    W[s].count_start = cblk;
    W[s].g_off = g.g_off;
    W[s].n = g.n;
    W[s].tile_base = g.tile_base;
    W[s].ct_off = ct;
    W[s].TX = g.TX;
    W[s].TY = g.TY;
    W[s].CB = (g.TX + 63) / 64;
    W[s].n_chunks = (int32_t)((g.n + kChunk - 1) / kChunk);
    W[s].band_rows = std::max(1, std::min(g.TY, kDiffWords / std::max(g.TX, 1)));
    W[s].n_bands = (g.TY + W[s].band_rows - 1) / W[s].band_rows;
    ws[s] = waves;
    cs[s] = cblk;
    waves += (int64_t)W[s].n_chunks * ((g.TY + kRowsPerGroup - 1) / kRowsPerGroup) * W[s].CB;
    cblk += (int64_t)W[s].n_chunks * W[s].n_bands;
    ct += (int64_t)W[s].n_chunks * g.TX * g.TY;
  }
  *total_chunk_tiles = ct;
  *total_count_blocks = cblk;
  return waves;
}

hipError_t launch_gather_rect(hipStream_t st, const int64_t* seg_gstart, int S, int64_t G,
                              const uint32_t* sorted_ids, const uint64_t* rect,
                              uint64_t* rect_sorted) {
  if (G == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_rect_kernel, dim3(nblk(G, 256)), dim3(256), 0, st, seg_gstart, S, G,
                     sorted_ids, rect, rect_sorted);
  return hipGetLastError();
}

hipError_t launch_bin_count(hipStream_t st, const void* work_dev, int S, int64_t total_blocks,
                            const uint64_t* rect_sorted, uint32_t* counts) {
  if (total_blocks == 0) return hipSuccess;
  const BinWork* W = (const BinWork*)work_dev;
  const int64_t* cs = (const int64_t*)(W + S) + S;
  hipLaunchKernelGGL(bin_count_kernel, dim3((unsigned)total_blocks), dim3(256), 0, st, W, cs, S,
                     total_blocks, rect_sorted, counts);
  return hipGetLastError();
}

hipError_t launch_bin_scan(hipStream_t st, const void* work_dev, int S, const int64_t* seg_tstart,
                           int64_t n_tiles, uint32_t* counts, uint32_t* tile_total,
                           uint64_t* partial, uint64_t* tile_start, uint64_t* ranges,
                           uint64_t* n_instances) {
  const BinWork* W = (const BinWork*)work_dev;
  if (n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(chunk_scan_kernel, dim3(nblk(n_tiles, 256)), dim3(256), 0, st, W, seg_tstart,
                     S, n_tiles, counts, tile_total);
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

hipError_t launch_bin_place(hipStream_t st, const void* work_dev, int S, int64_t total_waves,
                            const uint32_t* sorted_ids, const uint64_t* rect_sorted,
                            const uint32_t* counts, const uint64_t* tile_start,
                            const uint64_t* n_instances, uint64_t capacity, uint32_t* values) {
  if (total_waves == 0) return hipSuccess;
  const BinWork* W = (const BinWork*)work_dev;
  const int64_t* ws = (const int64_t*)(W + S);
  hipLaunchKernelGGL(bin_place_kernel, dim3((unsigned)total_waves), dim3(256), 0, st, W, ws, S,
                     total_waves, sorted_ids, rect_sorted, counts, tile_start, n_instances,
                     capacity, values);
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

}  // namespace gsc
