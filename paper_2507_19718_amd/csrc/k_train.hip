// k_train.hip -- per-pixel loss and its gradient (Eq. 4 or L2), the cached composite, and the
// AdamW step (Method: "Optimization and Hyperparameters", "Natural Path Termination",
// "Cascaded Cache Radiance Importance Sampling", Eq. 3).
#include "gsc_dev.h"

namespace gsc {

namespace {

constexpr int kLossThreads = 256;

// One lane per pixel, all K levels and three channels.  Per-block loss partials in fp64,
// summed afterwards in a fixed order.
__global__ void __launch_bounds__(kLossThreads) loss_composite_kernel(
    const float* __restrict__ images, const float* __restrict__ targets,
    const uint32_t* __restrict__ records, int spp, int K, int64_t P, int loss, float inv_k,
    float* __restrict__ dL, double* __restrict__ partials, float* __restrict__ composite) {
  __shared__ double red[kLossThreads];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (p < P) {
    for (int l = 0; l < K; ++l) {
      const int64_t base = 3 * ((int64_t)l * P + p);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float y = images[base + c], x = targets[base + c];
        const float diff = y - x;
        float g;
        if (loss == 1) {
          const float dn = fmaxf(y, 0.0f) + 0.01f;
          const float den = dn * dn;
          acc += (double)((diff * diff) / den);
          g = ((2.0f * diff) / den) * inv_k;
        } else {
          acc += (double)(diff * diff);
          g = (2.0f * diff) * inv_k;
        }
        dL[base + c] = g;
      }
    }
    if (composite) {
      // Per sample: the path's own radiance, or the cache of its length divided by beta; the
      // pixel is the mean over samples, summed in sample order.
      float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
      for (int smp = 0; smp < spp; ++smp) {
        const uint32_t* rec = records + 5 * ((int64_t)smp * P + p);
        const float L0 = __uint_as_float(rec[0]), L1 = __uint_as_float(rec[1]),
                    L2 = __uint_as_float(rec[2]), beta = __uint_as_float(rec[3]);
        const uint32_t n = rec[4] & 0xffffu, kind = rec[4] >> 16;
        float o0 = 0.0f, o1 = 0.0f, o2 = 0.0f;
        if (n >= 1u) {
          const float lum = (0.2126f * L0 + 0.7152f * L1) + 0.0722f * L2;
          const bool use_cache = (kind == (uint32_t)GSC_KIND_EARLY) || !(lum > 0.0f);
          if (use_cache) {
            const uint32_t lvl = (n < (uint32_t)K ? n : (uint32_t)K) - 1u;
            const float* cv = images + 3 * ((int64_t)lvl * P + p);
            o0 = fmaxf(cv[0], 0.0f) / beta;
            o1 = fmaxf(cv[1], 0.0f) / beta;
            o2 = fmaxf(cv[2], 0.0f) / beta;
          } else {
            o0 = L0; o1 = L1; o2 = L2;
          }
        }
        a0 = a0 + o0; a1 = a1 + o1; a2 = a2 + o2;
      }
      const float fs = (float)spp;
      composite[3 * p + 0] = a0 / fs;
      composite[3 * p + 1] = a1 / fs;
      composite[3 * p + 2] = a2 / fs;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kLossThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) loss_final_kernel(const double* __restrict__ partials, int n,
                                                         float scale, float* __restrict__ loss_out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += partials[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss_out = (float)(red[0] * (double)scale);
}

// AdamW, every operation separately rounded; skipped entirely when *guard is not finite.
__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ param, float* __restrict__ m,
                                                   float* __restrict__ v, const float* __restrict__ grad,
                                                   int64_t n, float b1, float b2, float omb1,
                                                   float omb2, float s1, float s2, float wdf,
                                                   float eps, const float* __restrict__ guard) {
  if (guard && !isfinite(*guard)) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  AdamGroup G;
  G.b1 = b1; G.b2 = b2; G.omb1 = omb1; G.omb2 = omb2; G.s1 = s1; G.s2 = s2; G.wdf = wdf; G.eps = eps;
  adamw_element(param, m, v, i, grad[i], G);
}

// s1 = lr / (1 - beta1^t) and s2 = 1 / sqrt(1 - beta2^t) in double, then rounded, with
// t = steps taken + 1 read from the device (Optimization: AdamW with bias correction).
__global__ void adam_factors_kernel(AdamGroup* __restrict__ groups, int n) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  AdamGroup& g = groups[i];
  if (g.p == nullptr || g.step == nullptr) return;
  const double t = (double)(*g.step + 1);
  g.s1 = (float)(g.lr / (1.0 - pow(g.b1d, t)));
  g.s2 = (float)(1.0 / sqrt(1.0 - pow(g.b2d, t)));
}

// One thread per segment: the level's step count advances only if its update was not skipped.
__global__ void adam_commit_kernel(const AdamGroup* __restrict__ groups, int S) {
  const int s = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (s >= S) return;
  const AdamGroup& g = groups[5 * s];
  if (g.p == nullptr || g.step == nullptr) return;
  if (g.guard && !isfinite(*g.guard)) return;
  *g.step += 1;
}

__global__ void capacity_guard_kernel(const uint64_t* __restrict__ n_inst, uint64_t capacity,
                                      float* __restrict__ losses, int n) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n && *n_inst > capacity) losses[i] = __int_as_float(0x7fc00000);
}

}  // namespace

int loss_num_partials(int64_t pixels) { return (int)((pixels + kLossThreads - 1) / kLossThreads); }

hipError_t launch_loss_composite(hipStream_t st, const float* images, const float* targets,
                                 const void* records, int spp, int K, int w, int h, int loss,
                                 float* dL_dimages, double* partials, float* loss_out,
                                 float* composite) {
  const int64_t P = (int64_t)w * h;
  if (P == 0) return hipSuccess;
  const int nb = loss_num_partials(P);
  const float kf = (float)(3.0 * (double)P);
  const float inv_k = 1.0f / kf;
  hipLaunchKernelGGL(loss_composite_kernel, dim3(nb), dim3(kLossThreads), 0, st, images, targets,
                     (const uint32_t*)records, spp, K, P, loss, inv_k, dL_dimages, partials, composite);
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, st, partials, nb, inv_k, loss_out);
  return hipGetLastError();
}

hipError_t launch_adam(hipStream_t st, float* param, float* m, float* v, const float* grad,
                       int64_t count, float b1, float b2, float omb1, float omb2, float s1,
                       float s2, float wdf, float eps, const float* guard) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, param, m,
                     v, grad, count, b1, b2, omb1, omb2, s1, s2, wdf, eps, guard);
  return hipGetLastError();
}


hipError_t launch_adam_factors(hipStream_t st, AdamGroup* groups, int n_groups) {
  if (n_groups <= 0) return hipSuccess;
  hipLaunchKernelGGL(adam_factors_kernel, dim3((unsigned)((n_groups + 63) / 64)), dim3(64), 0, st,
                     groups, n_groups);
  return hipGetLastError();
}

hipError_t launch_adam_commit(hipStream_t st, const AdamGroup* groups, int S) {
  if (S <= 0) return hipSuccess;
  hipLaunchKernelGGL(adam_commit_kernel, dim3((unsigned)((S + 63) / 64)), dim3(64), 0, st, groups, S);
  return hipGetLastError();
}

hipError_t launch_capacity_guard(hipStream_t st, const uint64_t* n_inst, uint64_t capacity,
                                 float* losses, int n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(capacity_guard_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, n_inst,
                     capacity, losses, n);
  return hipGetLastError();
}

}  // namespace gsc
