// gsc_dev.h -- device-side building blocks of the GSCache HIP path for gfx950 (CDNA4).
//
// Everything here is evaluated in binary32 with no FMA contraction (-ffp-contract=off), with
// correctly rounded division and square root, so that the projection (and with it the tile
// binning) and the tracer follow a fixed operation order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsc_internal.h"

namespace gsc {

// Device bounds checks of a debug build (compiled with -DGSC_DEBUG).  GSC_DCHECK(cond, bit)
// guards an access whose index comes from data (a list entry, a cursor, a count) and yields
// cond; in a debug build a false cond also sets `bit` in this translation unit's flag word, the
// guarded access is skipped, and the call that ran the kernel fails (the runtime reads and
// clears the words after every call).  In other builds it is the constant true and cond is not
// compiled at all.
#ifdef GSC_DEBUG
static __device__ uint32_t g_debug_flags;
__device__ __forceinline__ bool dcheck(bool ok, uint32_t bit) {
  if (!ok) atomicOr(&g_debug_flags, bit);
  return ok;
}
#define GSC_DCHECK(cond, bit) ::gsc::dcheck((cond), (bit))
#define GSC_DEBUG_FLAGS_READER(fn)                                                          \
  uint32_t fn() {                                                                           \
    uint32_t v = 0u, z = 0u;                                                                \
    if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_debug_flags), 4) != hipSuccess) return ~0u;     \
    if (hipMemcpyToSymbol(HIP_SYMBOL(g_debug_flags), &z, 4) != hipSuccess) return ~0u;       \
    return v;                                                                               \
  }
#else
#define GSC_DCHECK(cond, bit) true
#define GSC_DEBUG_FLAGS_READER(fn) \
  uint32_t fn() { return 0u; }
#endif

// AdamW on element i of one parameter group (decoupled weight decay folded into wdf = 1 - lr wd,
// bias corrections into s1 = lr / (1 - b1^t) and s2 = 1 / sqrt(1 - b2^t)); every operation is
// separately rounded, in this order, wherever the step runs.
__device__ __forceinline__ void adamw_element(float* p, float* m, float* v, int64_t i, float g,
                                              const AdamGroup& G) {
  const float mn = G.b1 * m[i] + G.omb1 * g;
  const float vn = G.b2 * v[i] + G.omb2 * (g * g);
  float q = p[i] * G.wdf;
  const float den = sqrtf(vn) * G.s2 + G.eps;
  q = q - (G.s1 * mn) / den;
  m[i] = mn;
  v[i] = vn;
  p[i] = q;
}

// ---------------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3",
// SC'11): ten rounds of two 32x32->64-bit multiplications of counter words 0 and 2 by the
// round multipliers, the high halves xor-ed into words 1 and 3 with the round key, and the key
// advanced by the two Weyl increments between rounds.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t a = c[0], b = c[2];
    const uint32_t hi_a = __umulhi(0xD2511F53u, a), lo_a = 0xD2511F53u * a;
    const uint32_t hi_b = __umulhi(0xCD9E8D57u, b), lo_b = 0xCD9E8D57u * b;
    c[0] = hi_b ^ c[1] ^ k0;
    c[1] = lo_b;
    c[2] = hi_a ^ c[3] ^ k1;
    c[3] = lo_a;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// The random stream of one path: counter (pixel, sample, frame, block), key (lo32 seed,
// hi32 seed).  Draw k is word k mod 4 of block k / 4; the block's words are consumed in order
// by shifting them down.
struct PathStream {
  uint32_t key0, key1, pixel, sample, frame, block;
  uint32_t w0, w1, w2, w3, left;
  __device__ __forceinline__ PathStream(uint64_t seed, uint32_t pix, uint32_t smp, uint32_t frm)
      : key0((uint32_t)seed), key1((uint32_t)(seed >> 32)), pixel(pix), sample(smp), frame(frm),
        block(0), w0(0), w1(0), w2(0), w3(0), left(0) {}
  __device__ __forceinline__ uint32_t next() {
    if (left == 0) {
      uint32_t c[4] = {pixel, sample, frame, block};
      philox4x32_10(c, key0, key1);
      w0 = c[0]; w1 = c[1]; w2 = c[2]; w3 = c[3];
      ++block;
      left = 4;
    }
    const uint32_t r = w0;
    w0 = w1; w1 = w2; w2 = w3;
    --left;
    return r;
  }
  // (word >> 8) * 2^-24: exact, in [0, 1 - 2^-24].
  __device__ __forceinline__ float uniform() { return (float)(next() >> 8) * 0x1p-24f; }
};

// ---------------------------------------------------------------------------------------------
// Portable exp / log / sincos.  Cody-Waite argument reduction and truncated series with
// coefficients fl(1/k!) or fl(1/k); each operation separately rounded.
//   ln 2 = LN2_HI + LN2_LO, LN2_HI = 45426 / 2^16 (16 significant bits), LN2_LO = fl(ln2 - HI)
//   pi/2 = P1 + P2 + P3: P1 = pi/2 to 16 significant bits, P2 = the remainder to 16 bits,
//   P3 = fl(remainder - P2).
// ---------------------------------------------------------------------------------------------
constexpr float kLn2Hi = 0x1.62e4p-1f;
constexpr float kLn2Lo = 0x1.7f7d1cp-20f;
constexpr float kLog2e = 0x1.715476p+0f;
constexpr float kPio2_1 = 0x1.922p+0f;
constexpr float kPio2_2 = -0x1.2aeep-18f;
constexpr float kPio2_3 = -0x1.e973dcp-35f;
constexpr float kTwoOverPi = 0x1.45f306p-1f;
constexpr float kTwoPi = 0x1.921fb6p+2f;
constexpr float kInv4Pi = 0x1.45f306p-4f;

__device__ __forceinline__ float pow2i(int e) {   // 2^e for e in [-126, 127]
  return __int_as_float((e + 127) << 23);
}

__device__ __forceinline__ float gexp(float x) {
  if (x != x) return x;
  if (x > 88.7f) return __int_as_float(0x7f800000);
  if (x < -87.3f) return 0.0f;
  const float n = rintf(x * kLog2e);
  const float r = (x - n * kLn2Hi) - n * kLn2Lo;
  float p = (float)(1.0 / 5040.0);
  p = p * r + (float)(1.0 / 720.0);
  p = p * r + (float)(1.0 / 120.0);
  p = p * r + (float)(1.0 / 24.0);
  p = p * r + (float)(1.0 / 6.0);
  p = p * r + 0.5f;
  p = p * r + 1.0f;
  p = p * r + 1.0f;
  const int ni = (int)n;
  const int half = ni / 2;
  return (p * pow2i(ni - half)) * pow2i(half);
}

// x in [2^-24, 1] (normal numbers): x = m 2^e with m in [sqrt(1/2), sqrt(2)).
__device__ __forceinline__ float glog(float x) {
  const uint32_t bits = __float_as_uint(x);
  int e = (int)((bits >> 23) & 0xffu) - 126;               // x = f 2^e, f in [0.5, 1)
  float m = __uint_as_float((bits & 0x007fffffu) | 0x3f000000u);
  if (m < 0.70710678118654752f) { m = m * 2.0f; e -= 1; }
  const float s = (m - 1.0f) / (m + 1.0f);
  const float t = s * s;
  float p = (float)(1.0 / 9.0);
  p = p * t + (float)(1.0 / 7.0);
  p = p * t + (float)(1.0 / 5.0);
  p = p * t + (float)(1.0 / 3.0);
  p = p * t;
  const float lm = 2.0f * (s + s * p);
  const float ef = (float)e;
  return ef * kLn2Hi + (ef * kLn2Lo + lm);
}

// phi in [0, 2 pi).
__device__ __forceinline__ void gsincos(float phi, float* so, float* co) {
  const float k = rintf(phi * kTwoOverPi);
  const float r = ((phi - k * kPio2_1) - k * kPio2_2) - k * kPio2_3;
  const float r2 = r * r;
  float ps = (float)(1.0 / 362880.0);
  ps = ps * r2 + (float)(-1.0 / 5040.0);
  ps = ps * r2 + (float)(1.0 / 120.0);
  ps = ps * r2 + (float)(-1.0 / 6.0);
  const float sn = r + r * (ps * r2);
  float pc = (float)(-1.0 / 3628800.0);
  pc = pc * r2 + (float)(1.0 / 40320.0);
  pc = pc * r2 + (float)(-1.0 / 720.0);
  pc = pc * r2 + (float)(1.0 / 24.0);
  pc = pc * r2 + -0.5f;
  const float cs = 1.0f + pc * r2;
  const int q = ((int)k) & 3;
  float s = sn, c = cs;
  if (q == 1) { s = cs; c = -sn; }
  else if (q == 2) { s = -sn; c = -cs; }
  else if (q == 3) { s = -cs; c = sn; }
  *so = s;
  *co = c;
}

// ---------------------------------------------------------------------------------------------
// Projection of one Gaussian (the contract shared with the binning: each step separately
// rounded in the order written, sums left to right).
// ---------------------------------------------------------------------------------------------
struct Projected {
  float u, v, A, B, Cc, o, z;
  float radius;
  int px0, px1, py0, py1;   // full-frame inclusive window
  int tx0, tx1, ty0, ty1;   // window-local inclusive tile rect (tiles of 2^tsx x 2^tsy pixels)
  uint32_t tiles;           // 0 when culled
};

__device__ __forceinline__ Projected project_one(const float* __restrict__ pos,
                                                 const float* __restrict__ rot,
                                                 const float* __restrict__ ls, float logit,
                                                 const DevCam& cam, int tsx, int tsy) {
  Projected P;
  P.tiles = 0u;
  P.px0 = P.px1 = P.py0 = P.py1 = 0;
  P.tx0 = P.tx1 = P.ty0 = P.ty1 = 0;
  P.u = P.v = P.A = P.B = P.Cc = P.radius = 0.0f;
  // Camera transform first: it decides culling.
  const float p0 = pos[0], p1 = pos[1], p2 = pos[2];
  const float* Rc = cam.R;
  const float x = ((Rc[0] * p0 + Rc[1] * p1) + Rc[2] * p2) + cam.t[0];
  const float y = ((Rc[3] * p0 + Rc[4] * p1) + Rc[5] * p2) + cam.t[1];
  const float z = ((Rc[6] * p0 + Rc[7] * p1) + Rc[8] * p2) + cam.t[2];
  P.z = z;
  // Activations: normalised quaternion, exp scale, sigmoid opacity.
  float qw = rot[0], qx = rot[1], qy = rot[2], qz = rot[3];
  const float qn = sqrtf(((qw * qw + qx * qx) + qy * qy) + qz * qz);
  qw = qw / qn; qx = qx / qn; qy = qy / qn; qz = qz / qn;
  P.o = 1.0f / (1.0f + gexp(-logit));
  if (!(z > cam.znear) || !isfinite(x) || !isfinite(y)) return P;
  const float s0 = gexp(ls[0]), s1 = gexp(ls[1]), s2 = gexp(ls[2]);
  // M = R(q) diag(s).
  const float m00 = (1.0f - 2.0f * (qy * qy + qz * qz)) * s0;
  const float m01 = (2.0f * (qx * qy - qw * qz)) * s1;
  const float m02 = (2.0f * (qx * qz + qw * qy)) * s2;
  const float m10 = (2.0f * (qx * qy + qw * qz)) * s0;
  const float m11 = (1.0f - 2.0f * (qx * qx + qz * qz)) * s1;
  const float m12 = (2.0f * (qy * qz - qw * qx)) * s2;
  const float m20 = (2.0f * (qx * qz - qw * qy)) * s0;
  const float m21 = (2.0f * (qy * qz + qw * qx)) * s1;
  const float m22 = (1.0f - 2.0f * (qx * qx + qy * qy)) * s2;
  // Sigma3 = M M^T (symmetric).
  const float S00 = (m00 * m00 + m01 * m01) + m02 * m02;
  const float S01 = (m00 * m10 + m01 * m11) + m02 * m12;
  const float S02 = (m00 * m20 + m01 * m21) + m02 * m22;
  const float S11 = (m10 * m10 + m11 * m11) + m12 * m12;
  const float S12 = (m10 * m20 + m11 * m21) + m12 * m22;
  const float S22 = (m20 * m20 + m21 * m21) + m22 * m22;
  // EWA Jacobian with the 1.3x frustum clamp, T = J Rc.
  const float iz = 1.0f / z;
  const float limx = 1.3f * ((float)cam.full_w / (2.0f * cam.fx));
  const float limy = 1.3f * ((float)cam.full_h / (2.0f * cam.fy));
  const float txz = fminf(fmaxf(x * iz, -limx), limx);
  const float tyz = fminf(fmaxf(y * iz, -limy), limy);
  const float tx = txz * z, ty = tyz * z;
  const float iz2 = iz * iz;
  const float J00 = cam.fx * iz, J02 = -(cam.fx * tx) * iz2;
  const float J11 = cam.fy * iz, J12 = -(cam.fy * ty) * iz2;
  const float T00 = J00 * Rc[0] + J02 * Rc[6], T01 = J00 * Rc[1] + J02 * Rc[7],
              T02 = J00 * Rc[2] + J02 * Rc[8];
  const float T10 = J11 * Rc[3] + J12 * Rc[6], T11 = J11 * Rc[4] + J12 * Rc[7],
              T12 = J11 * Rc[5] + J12 * Rc[8];
  // U = T Sigma3; Sigma2 = U T^T.
  const float U00 = (T00 * S00 + T01 * S01) + T02 * S02;
  const float U01 = (T00 * S01 + T01 * S11) + T02 * S12;
  const float U02 = (T00 * S02 + T01 * S12) + T02 * S22;
  const float U10 = (T10 * S00 + T11 * S01) + T12 * S02;
  const float U11 = (T10 * S01 + T11 * S11) + T12 * S12;
  const float U12 = (T10 * S02 + T11 * S12) + T12 * S22;
  const float c00 = (U00 * T00 + U01 * T01) + U02 * T02;
  const float c01 = (U00 * T10 + U01 * T11) + U02 * T12;
  const float c11 = (U10 * T10 + U11 * T11) + U12 * T12;
  const float a = c00 + 0.3f, b = c01, c = c11 + 0.3f;
  const float det = a * c - b * b;
  if (!(det > 0.0f)) return P;
  P.A = c / det;
  P.B = (-b) / det;
  P.Cc = a / det;
  const float mid = 0.5f * (a + c);
  const float lam = mid + sqrtf(fmaxf(0.1f, mid * mid - det));
  const float r = ceilf(3.0f * sqrtf(lam));
  P.radius = r;
  P.u = cam.fx * (x * iz) + (cam.cx - 0.5f);
  P.v = cam.fy * (y * iz) + (cam.cy - 0.5f);
  const float fx0 = fmaxf((float)cam.x0, ceilf(P.u - r));
  const float fx1 = fminf((float)(cam.x0 + cam.w - 1), floorf(P.u + r));
  const float fy0 = fmaxf((float)cam.y0, ceilf(P.v - r));
  const float fy1 = fminf((float)(cam.y0 + cam.h - 1), floorf(P.v + r));
  if (!(fx0 <= fx1) || !(fy0 <= fy1)) return P;
  P.px0 = (int)fx0; P.px1 = (int)fx1; P.py0 = (int)fy0; P.py1 = (int)fy1;
  P.tx0 = (P.px0 - cam.x0) >> tsx; P.tx1 = (P.px1 - cam.x0) >> tsx;
  P.ty0 = (P.py0 - cam.y0) >> tsy; P.ty1 = (P.py1 - cam.y0) >> tsy;
  P.tiles = (uint32_t)((P.tx1 - P.tx0 + 1) * (P.ty1 - P.ty0 + 1));
  return P;
}

// Segment lookup: the last s with start[s] <= i (start ascending, start[0] == 0).
template <typename T>
__device__ __forceinline__ int find_segment(const T* __restrict__ start, int n, T i) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace gsc
