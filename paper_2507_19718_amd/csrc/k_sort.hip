// k_sort.hip -- segmented least-significant-digit radix sort of 32-bit keys with 32-bit
// values, 8-bit digits, stable.  Used to order each segment's Gaussians by the bit pattern of
// their camera depth (positive floats order as unsigned integers); ties keep id order.  These
// are the four low digits of the (tile << 32 | depth) instance key, sorted once per Gaussian
// instead of once per instance; the tile digit is applied by the binning placement pass.
//
// Per pass: (1) per-block digit histograms, (2) per (segment, digit) exclusive scans over the
// segment's blocks and a per-segment scan of the digit totals, (3) stable scatter: items are
// taken in index order, 256 per round, and ranked within a 64-wide wavefront by eight ballots
// (lanes with equal digits), then across the block's four wavefronts in LDS.
#include "gsc_dev.h"

namespace gsc {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortItems = kSortThreads * kSortRounds;   // 2048 items per block

struct SortBlock {
  int64_t start;      // first item (global index)
  int64_t seg_base;   // first item of the block's segment
  int32_t count;      // items in this block
  int32_t seg;        // segment index
};

// Lanes of the wavefront whose 8-bit digit equals this lane's (valid lanes only).
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < 8; ++bit) {
    const bool set = (d >> bit) & 1u;
    const uint64_t m = __ballot(valid && set);
    peers &= set ? m : ~m;
  }
  return peers;
}

__global__ void __launch_bounds__(kSortThreads) sort_hist_kernel(const SortBlock* __restrict__ blocks,
                                                                 const uint32_t* __restrict__ keys,
                                                                 int shift, uint32_t* __restrict__ hist,
                                                                 int n_blocks) {
  __shared__ uint32_t cnt[256];
  const SortBlock B = blocks[blockIdx.x];
  const int lane = __lane_id();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t kr[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int k = r * kSortThreads + threadIdx.x;
    kr[r] = (k < B.count) ? keys[B.start + k] : 0u;
  }
  cnt[threadIdx.x] = 0u;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const bool valid = r * kSortThreads + (int)threadIdx.x < B.count;
    const uint32_t d = (kr[r] >> shift) & 0xffu;
    // One LDS atomic per distinct digit of the wavefront (keys often share their high digits).
    const uint64_t peers = digit_peers(d, valid);
    if (valid && (peers & lt_mask) == 0ull) atomicAdd(&cnt[d], (uint32_t)__popcll(peers));
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * n_blocks + blockIdx.x] = cnt[threadIdx.x];
}

// One workgroup per (segment, digit): exclusive scan of the digit's per-block counts over the
// segment's blocks (in place, digit-local offsets) and the digit total.
__global__ void __launch_bounds__(256) sort_scan_digit_kernel(const int32_t* __restrict__ seg_first_block,
                                                              uint32_t* __restrict__ hist, int n_blocks,
                                                              uint32_t* __restrict__ dtot) {
  __shared__ uint32_t tmp[256];
  const int s = blockIdx.x >> 8, d = blockIdx.x & 255;
  const int b0 = seg_first_block[s], b1 = seg_first_block[s + 1];
  uint32_t* h = hist + (int64_t)d * n_blocks;
  uint32_t carry = 0u;
  for (int base = b0; base < b1; base += 256) {
    const int b = base + (int)threadIdx.x;
    const uint32_t v = (b < b1) ? h[b] : 0u;
    tmp[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const uint32_t a = (threadIdx.x >= (unsigned)off) ? tmp[threadIdx.x - off] : 0u;
      __syncthreads();
      tmp[threadIdx.x] += a;
      __syncthreads();
    }
    if (b < b1) h[b] = carry + tmp[threadIdx.x] - v;
    carry += tmp[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) dtot[s * 256 + d] = carry;
}

// One workgroup per segment: exclusive scan of the 256 digit totals -> digit bases.
__global__ void __launch_bounds__(256) sort_scan_base_kernel(uint32_t* __restrict__ dtot) {
  __shared__ uint32_t tmp[256];
  const int s = blockIdx.x, d = threadIdx.x;
  const uint32_t v = dtot[s * 256 + d];
  tmp[d] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t a = (d >= off) ? tmp[d - off] : 0u;
    __syncthreads();
    tmp[d] += a;
    __syncthreads();
  }
  dtot[s * 256 + d] = tmp[d] - v;
}

__global__ void __launch_bounds__(kSortThreads) sort_scatter_kernel(
    const SortBlock* __restrict__ blocks, const uint32_t* __restrict__ keys_in,
    const uint32_t* __restrict__ vals_in, int shift, const uint32_t* __restrict__ hist, int n_blocks,
    const uint32_t* __restrict__ dbase, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[4][256];
  const SortBlock B = blocks[blockIdx.x];
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = __lane_id();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t kr[kSortRounds], vr[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {   // all loads issued before the first barrier
    const int k = r * kSortThreads + tid;
    kr[r] = (k < B.count) ? keys_in[B.start + k] : 0u;
    vr[r] = (k < B.count) ? vals_in[B.start + k] : 0u;
  }
  run[tid] = hist[(int64_t)tid * n_blocks + blockIdx.x] + dbase[B.seg * 256 + tid];
  for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0u;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const bool valid = r * kSortThreads + tid < B.count;
    const uint32_t key = kr[r], val = vr[r];
    const uint32_t d = (key >> shift) & 0xffu;
    const uint64_t peers = digit_peers(d, valid);
    const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
    const bool leader = valid && ((peers & lt_mask) == 0ull);
    if (leader) wcnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      keys_out[B.seg_base + pos] = key;
      vals_out[B.seg_base + pos] = val;
    }
    __syncthreads();
    run[tid] += (wcnt[0][tid] + wcnt[1][tid]) + (wcnt[2][tid] + wcnt[3][tid]);
    for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0u;
    __syncthreads();
  }
}

}  // namespace

// Host side of the sort: the block table is built from the segment sizes.
size_t sort_table_bytes(int n_blocks, int S) {
  return sizeof(SortBlock) * (size_t)n_blocks + sizeof(int32_t) * (size_t)(S + 1);
}

// Histogram scratch in 32-bit words: [256][n_blocks] counts plus [S][256] digit totals.
size_t sort_hist_words(int n_blocks, int S) { return 256 * (size_t)n_blocks + 256 * (size_t)S; }

int sort_count_blocks(const int64_t* seg_n, int S) {
  int nb = 0;
  for (int s = 0; s < S; ++s) nb += (int)((seg_n[s] + kSortItems - 1) / kSortItems);
  return nb;
}

// Fills a host staging area: [SortBlock x n_blocks][int32 first_block x (S + 1)].
void sort_fill_table(void* host, const int64_t* seg_n, const int64_t* seg_off, int S) {
  SortBlock* blk = (SortBlock*)host;
  int32_t* first = (int32_t*)(blk + sort_count_blocks(seg_n, S));
  int b = 0;
  for (int s = 0; s < S; ++s) {
    first[s] = b;
    for (int64_t k = 0; k < seg_n[s]; k += kSortItems) {
      blk[b].start = seg_off[s] + k;
      blk[b].seg_base = seg_off[s];
      blk[b].count = (int32_t)((seg_n[s] - k) < kSortItems ? (seg_n[s] - k) : kSortItems);
      blk[b].seg = s;
      ++b;
    }
  }
  first[S] = b;
}

// Sorts keys/vals of every segment in place (4 passes; the temporaries receive the odd passes).
hipError_t launch_segmented_sort(hipStream_t st, const void* table_dev, int n_blocks, int S,
                                 uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp,
                                 uint32_t* vals_tmp, uint32_t* hist) {
  if (n_blocks == 0) return hipSuccess;
  const SortBlock* blocks = (const SortBlock*)table_dev;
  const int32_t* first = (const int32_t*)(blocks + n_blocks);
  uint32_t* kin = keys; uint32_t* vin = vals;
  uint32_t* kout = keys_tmp; uint32_t* vout = vals_tmp;
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 8 * pass;
    uint32_t* dtot = hist + 256 * (size_t)n_blocks;
    hipLaunchKernelGGL(sort_hist_kernel, dim3(n_blocks), dim3(kSortThreads), 0, st, blocks, kin,
                       shift, hist, n_blocks);
    hipLaunchKernelGGL(sort_scan_digit_kernel, dim3(S * 256), dim3(256), 0, st, first, hist,
                       n_blocks, dtot);
    hipLaunchKernelGGL(sort_scan_base_kernel, dim3(S), dim3(256), 0, st, dtot);
    hipLaunchKernelGGL(sort_scatter_kernel, dim3(n_blocks), dim3(kSortThreads), 0, st, blocks,
                       kin, vin, shift, hist, n_blocks, dtot, kout, vout);
    uint32_t* t;
    t = kin; kin = kout; kout = t;
    t = vin; vin = vout; vout = t;
  }
  return hipGetLastError();
}

}  // namespace gsc
