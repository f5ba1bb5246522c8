// k_init.hip -- the rest of cache initialisation (Method: "Cache Initialization", Eq. 2): the
// mean distance of every point to its three nearest neighbours, Eq. 2's capped isotropic
// scales, and the Gaussians of each level.
//
// Neighbour search: points are binned into a uniform G^3 grid over the unit cube (G chosen for
// about two points per cell), sorted by cell (the library's segmented radix sort), and every
// point scans rings of cells of growing Chebyshev radius r around its own until its third
// nearest distance is at most r / G, the least distance of any point outside the rings scanned.
// Lanes run in cell order, so a wavefront's lanes scan overlapping cells.
#include "gsc_dev.h"

namespace gsc {

namespace {

constexpr int kInitBlock = 256;

__device__ __forceinline__ int cell_of(float x, int G) {
  const int c = (int)floorf(x * (float)G);
  return min(max(c, 0), G - 1);
}

__global__ void __launch_bounds__(kInitBlock) grid_key_kernel(const float* __restrict__ pos, int64_t n,
                                                              int G, uint32_t* __restrict__ key,
                                                              uint32_t* __restrict__ id) {
  const int64_t i = (int64_t)blockIdx.x * kInitBlock + threadIdx.x;
  if (i >= n) return;
  const int cx = cell_of(pos[3 * i], G), cy = cell_of(pos[3 * i + 1], G), cz = cell_of(pos[3 * i + 2], G);
  key[i] = (uint32_t)((cz * G + cy) * G + cx);
  id[i] = (uint32_t)i;
}

// Cell ranges [start, end) of the sorted keys (cells without points keep start = end = 0) and
// the points gathered into sorted order.
__global__ void __launch_bounds__(kInitBlock) cell_range_kernel(const uint32_t* __restrict__ key,
                                                                const uint32_t* __restrict__ id,
                                                                const float* __restrict__ pos, int64_t n,
                                                                uint32_t* __restrict__ start,
                                                                uint32_t* __restrict__ end,
                                                                float4* __restrict__ spos) {
  const int64_t j = (int64_t)blockIdx.x * kInitBlock + threadIdx.x;
  if (j >= n) return;
  const uint32_t k = key[j];
  if (j == 0 || key[j - 1] != k) start[k] = (uint32_t)j;
  if (j == n - 1 || key[j + 1] != k) end[k] = (uint32_t)(j + 1);
  const uint32_t i = id[j];
  spos[j] = make_float4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], 0.0f);
}

__device__ __forceinline__ void keep3(float d2, float& b0, float& b1, float& b2) {
  if (d2 < b2) {
    if (d2 < b1) {
      b2 = b1;
      if (d2 < b0) { b1 = b0; b0 = d2; } else { b1 = d2; }
    } else {
      b2 = d2;
    }
  }
}

// One lane per sorted point: mean of the three smallest distances to other points.
__global__ void __launch_bounds__(kInitBlock) knn3_kernel(const float4* __restrict__ spos,
                                                          const uint32_t* __restrict__ id, int64_t n,
                                                          int G, const uint32_t* __restrict__ start,
                                                          const uint32_t* __restrict__ end,
                                                          float* __restrict__ mean3) {
  const int64_t j = (int64_t)blockIdx.x * kInitBlock + threadIdx.x;
  if (j >= n) return;
  const float4 p = spos[j];
  const int cx = cell_of(p.x, G), cy = cell_of(p.y, G), cz = cell_of(p.z, G);
  const float inf = __int_as_float(0x7f800000);
  float b0 = inf, b1 = inf, b2 = inf;
  const float h = 1.0f / (float)G;
  for (int r = 0; r <= G; ++r) {
    for (int dz = -r; dz <= r; ++dz) {
      const int z = cz + dz;
      if (z < 0 || z >= G) continue;
      for (int dy = -r; dy <= r; ++dy) {
        const int y = cy + dy;
        if (y < 0 || y >= G) continue;
        const bool face = (dz == -r || dz == r || dy == -r || dy == r);
        for (int dx = -r; dx <= r; dx += (face ? 1 : 2 * r)) {   // the ring's cells only
          const int x = cx + dx;
          if (x >= 0 && x < G) {
            const uint32_t c = (uint32_t)((z * G + y) * G + x);
            for (uint32_t k = start[c]; k < end[c]; ++k) {
              if ((int64_t)k == j) continue;
              const float4 q = spos[k];
              const float ex = q.x - p.x, ey = q.y - p.y, ez = q.z - p.z;
              keep3((ex * ex + ey * ey) + ez * ez, b0, b1, b2);
            }
          }
          if (r == 0) break;
        }
      }
    }
    // Every point not yet scanned lies at least r h away.
    const float reach = (float)r * h;
    if (b2 <= reach * reach) break;
  }
  mean3[id[j]] = ((sqrtf(b0) + sqrtf(b1)) + sqrtf(b2)) / 3.0f;
}

// Sum and sum of squares of mean3 in double, per workgroup, then over workgroups.
__global__ void __launch_bounds__(kInitBlock) moments_kernel(const float* __restrict__ v, int64_t n,
                                                             double* __restrict__ partial) {
  __shared__ double s1[kInitBlock], s2[kInitBlock];
  double a = 0.0, b = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kInitBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kInitBlock) {
    const double x = (double)v[i];
    a += x;
    b += x * x;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int off = kInitBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s1[threadIdx.x] += s1[threadIdx.x + off];
      s2[threadIdx.x] += s2[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s1[0];
    partial[2 * blockIdx.x + 1] = s2[0];
  }
}

// mu and the cap mu + 2 sigma (population standard deviation) into partial[2 nb], [2 nb + 1].
__global__ void __launch_bounds__(64) moments_final_kernel(double* __restrict__ partial, int nb,
                                                           int64_t n) {
  if (threadIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int k = 0; k < nb; ++k) { a += partial[2 * k]; b += partial[2 * k + 1]; }
  const double mu = a / (double)n;
  const double var = fmax(b / (double)n - mu * mu, 0.0);
  partial[2 * nb] = mu;
  partial[2 * nb + 1] = mu + 2.0 * sqrt(var);
}

// Eq. 2 and the level's Gaussians: position, identity rotation, log of the isotropic scale
// s = min(mu + 2 sigma, mean3) / 2, albedo as colour, the initial opacity logit.
__global__ void __launch_bounds__(kInitBlock) level_kernel(const double* __restrict__ stats,
                                                           int64_t n, const float* __restrict__ pos,
                                                           const float* __restrict__ albedo,
                                                           const float* __restrict__ mean3,
                                                           float opacity_logit, float* __restrict__ gpos,
                                                           float* __restrict__ grot,
                                                           float* __restrict__ gls,
                                                           float* __restrict__ grgb,
                                                           float* __restrict__ glogit) {
  const int64_t i = (int64_t)blockIdx.x * kInitBlock + threadIdx.x;
  if (i >= n) return;
  const double cap = stats[1];
  const double s = fmin(cap, (double)mean3[i]) / 2.0;
  const float ls = (float)log(s);
  for (int k = 0; k < 3; ++k) {
    gpos[3 * i + k] = pos[3 * i + k];
    gls[3 * i + k] = ls;
    grgb[3 * i + k] = albedo[3 * i + k];
  }
  grot[4 * i + 0] = 1.0f; grot[4 * i + 1] = 0.0f; grot[4 * i + 2] = 0.0f; grot[4 * i + 3] = 0.0f;
  glogit[i] = opacity_logit;
}

// Counts the points for which no attempt found an interaction (tries == 0).
__global__ void __launch_bounds__(kInitBlock) count_failed_kernel(const int32_t* __restrict__ tries,
                                                                  int64_t n,
                                                                  unsigned long long* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kInitBlock + threadIdx.x;
  const bool bad = i < n && tries[i] == 0;
  const uint64_t m = __ballot(bad);
  if (m != 0ull && __lane_id() == 0) atomicAdd(out, (unsigned long long)__popcll(m));
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kInitBlock - 1) / kInitBlock); }

}  // namespace

int init_grid_side(int64_t n) {
  int G = (int)std::cbrt((double)n / 2.0);
  return G < 1 ? 1 : (G > 256 ? 256 : G);
}

hipError_t launch_grid_keys(hipStream_t st, const float* pos, int64_t n, int G, uint32_t* key,
                            uint32_t* id) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(grid_key_kernel, dim3(nblk(n)), dim3(kInitBlock), 0, st, pos, n, G, key, id);
  return hipGetLastError();
}

hipError_t launch_cell_ranges(hipStream_t st, const uint32_t* key, const uint32_t* id, const float* pos,
                              int64_t n, uint32_t* start, uint32_t* end, float4* spos) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cell_range_kernel, dim3(nblk(n)), dim3(kInitBlock), 0, st, key, id, pos, n, start,
                     end, spos);
  return hipGetLastError();
}

hipError_t launch_knn3(hipStream_t st, const float4* spos, const uint32_t* id, int64_t n, int G,
                       const uint32_t* start, const uint32_t* end, float* mean3) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(knn3_kernel, dim3(nblk(n)), dim3(kInitBlock), 0, st, spos, id, n, G, start, end,
                     mean3);
  return hipGetLastError();
}

// Partial-sum slots: 2 per moments workgroup plus (mu, cap).
int init_moment_blocks() { return 512; }
size_t init_partial_doubles() { return 2 * 512 + 2; }

hipError_t launch_init_level(hipStream_t st, const float* mean3, int64_t n, const float* pos,
                             const float* albedo, float opacity_logit, double* partial, float* gpos,
                             float* grot, float* gls, float* grgb, float* glogit) {
  if (n == 0) return hipSuccess;
  const int nb = init_moment_blocks();
  hipLaunchKernelGGL(moments_kernel, dim3(nb), dim3(kInitBlock), 0, st, mean3, n, partial);
  hipLaunchKernelGGL(moments_final_kernel, dim3(1), dim3(64), 0, st, partial, nb, n);
  hipLaunchKernelGGL(level_kernel, dim3(nblk(n)), dim3(kInitBlock), 0, st, partial + 2 * nb, n, pos,
                     albedo, mean3, opacity_logit, gpos, grot, gls, grgb, glogit);
  return hipGetLastError();
}

hipError_t launch_count_failed(hipStream_t st, const int32_t* tries, int64_t n,
                               unsigned long long* out) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(count_failed_kernel, dim3(nblk(n)), dim3(kInitBlock), 0, st, tries, n, out);
  return hipGetLastError();
}

}  // namespace gsc
