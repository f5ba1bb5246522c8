// k_probe.hip -- micro-benchmarks that measure the ceilings the hot-path kernels are held
// against: random 32-byte gathers over a working set the size of a density grid (the tracer's
// lookups), float atomic adds to random addresses of a gradient-sized array (the adjoint's
// accumulation), and the vector ALU's fp32 FMA and exp rates (the splat kernels).  Each kernel
// leaves a value in memory that depends on all of its work, so none of it can be removed.
#include "gsc_dev.h"

namespace gsc {

namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  // Integer hash (a multiply-xorshift finaliser); spreads consecutive indices over the range.
  x ^= x >> 16; x *= 0x7feb352dU;
  x ^= x >> 15; x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

// Each thread reads `per_thread` random 32-byte cells, eight loads in flight.
__global__ void __launch_bounds__(256) probe_gather_kernel(const float4* __restrict__ cells,
                                                           uint64_t n_cells, int per_thread,
                                                           float* __restrict__ out) {
  const uint32_t tid = blockIdx.x * 256u + threadIdx.x;
  float acc = 0.0f;
  for (int i = 0; i < per_thread; i += 8) {
    float4 a[8], b[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint64_t h = ((uint64_t)mix32(tid * 0x9E3779B9u + (uint32_t)(i + k)) << 32) |
                         mix32(tid ^ (uint32_t)(0x85EBCA6Bu * (i + k + 1)));
      const uint64_t c = h % n_cells;
      a[k] = cells[2 * c];
      b[k] = cells[2 * c + 1];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += (a[k].x + a[k].w) + (b[k].y + b[k].z);
  }
  out[tid] = acc;
}

// Each thread adds 1 to `per_thread` random elements of an n-float array.
__global__ void __launch_bounds__(256) probe_atomic_kernel(float* __restrict__ buf, uint64_t n,
                                                           int per_thread) {
  const uint32_t tid = blockIdx.x * 256u + threadIdx.x;
  for (int i = 0; i < per_thread; ++i) {
    const uint64_t h = ((uint64_t)mix32(tid * 0x9E3779B9u + (uint32_t)i) << 32) |
                       mix32(tid ^ (uint32_t)(0x85EBCA6Bu * (i + 1)));
    unsafeAtomicAdd(&buf[h % n], 1.0f);
  }
}

// Eight independent chains of `iters` fp32 FMAs (mode 0) or exponentials (mode 1) per thread.
__global__ void __launch_bounds__(256) probe_valu_kernel(float* __restrict__ out, int iters,
                                                         int mode, float seed) {
  const uint32_t tid = blockIdx.x * 256u + threadIdx.x;
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = seed * (float)(tid + k + 1) * 1e-9f;
  if (mode == 0) {
    const float a = 0.999f, b = 1e-3f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], a, b);
    }
  } else {
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = __expf(-x[k]);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[tid] = s;
}

// Sets the self-test bit through the debug-check path, from one lane (debug builds only).
__global__ void __launch_bounds__(64) debug_selftest_kernel() {
  if (threadIdx.x == 0) (void)GSC_DCHECK(false, kDbgSelfTest);
}

}  // namespace

hipError_t launch_debug_selftest(hipStream_t st) {
  hipLaunchKernelGGL(debug_selftest_kernel, dim3(1), dim3(64), 0, st);
  return hipGetLastError();
}

GSC_DEBUG_FLAGS_READER(debug_flags_probe)

hipError_t launch_probe_gather(hipStream_t st, const float4* cells, uint64_t n_cells,
                               uint32_t threads, int per_thread, float* out) {
  hipLaunchKernelGGL(probe_gather_kernel, dim3(threads / 256), dim3(256), 0, st, cells, n_cells,
                     per_thread, out);
  return hipGetLastError();
}

hipError_t launch_probe_atomic(hipStream_t st, float* buf, uint64_t n, uint32_t threads,
                               int per_thread) {
  hipLaunchKernelGGL(probe_atomic_kernel, dim3(threads / 256), dim3(256), 0, st, buf, n,
                     per_thread);
  return hipGetLastError();
}

hipError_t launch_probe_valu(hipStream_t st, float* out, uint32_t threads, int iters, int mode) {
  hipLaunchKernelGGL(probe_valu_kernel, dim3(threads / 256), dim3(256), 0, st, out, iters, mode,
                     1.0f);
  return hipGetLastError();
}

}  // namespace gsc
