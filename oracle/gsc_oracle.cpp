// GSCache CPU oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, deliberately untiled CPU statement of what the GSCache hot path computes.
// Only the tests, the smoke check and the benchmark's CPU-baseline leg may load this library.
// It shares no code, header, constant table or helper with the HIP implementation; the two are
// written independently from the paper and from the published methods named below.
//
// Build: g++ -O2 -std=c++17 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC
// Every float expression is evaluated in binary32 in the order written (x86-64 SSE, no FMA
// contraction), which is what makes the projection and binning outputs bit-reproducible.
//
// Contents (paper sections in brackets):
//   * Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).
//   * Portable exp / log / sincos (Cody-Waite reduction + truncated series).
//   * Trilinear density lookup and 1D RGBA transfer function [Evaluation: predefined 1D TF].
//   * Delta-tracking volume path tracer with next-event estimation to point lights and to
//     spherical area lights (cone sampling, combined with the phase-sampled continuation by
//     MIS, power heuristic), or phase sampling only (the uniform baseline), ratio-tracked
//     shadow rays, the early-termination heuristic (Algorithm 1) with the cascaded survival
//     product beta (Eq. 3), and per-path-length training targets [Method: path-space radiance
//     cache, path termination heuristics, cache sampling, cache training; Evaluation: lights].
//   * Projection of 3D Gaussians to screen-space conics (the 3D Gaussian splatting
//     rasteriser the paper builds on) [Method: a path space radiance cache].
//   * Binning: every (tile, Gaussian) pair sorted by (tile, depth, id), per-tile ranges.
//   * Brute-force forward splatting per pixel: every covering Gaussian in depth order,
//     front-to-back alpha blending, no tiles.
//
// Parity status: every function here is pinned by tests under tests/ (closed forms,
// invariants, brute force, library routines); see each function's comment.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ------------------------------------------------------------------------------------------
// Philox4x32-10 (SC'11, "Parallel Random Numbers: As Easy as 1, 2, 3").
// Round: two 32x32->64 multiplications of counter words 0 and 2 by the round multipliers;
// the outputs are (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)).  The key
// is bumped by the Weyl constants between rounds.
// ------------------------------------------------------------------------------------------
struct Philox {
  static constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  static constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  static void block(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
      if (r > 0) { k0 += W0; k1 += W1; }
      uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
      uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
      uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
      uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
      c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
  }
};

// One path's stream: counter (pixel, sample, frame, block); draw k is word k%4 of block k/4.
struct PathRng {
  uint32_t key[2];
  uint32_t ctr[4];
  uint32_t buf[4];
  uint32_t k = 0;
  PathRng(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t frame) {
    key[0] = (uint32_t)seed; key[1] = (uint32_t)(seed >> 32);
    ctr[0] = pixel; ctr[1] = sample; ctr[2] = frame; ctr[3] = 0;
  }
  uint32_t next_u32() {
    if ((k & 3u) == 0) { ctr[3] = k >> 2; Philox::block(ctr, key, buf); }
    return buf[(k++) & 3u];
  }
  // u = (w >> 8) * 2^-24, exactly representable, in [0, 1 - 2^-24].
  float uniform() { return (float)(next_u32() >> 8) * (1.0f / 16777216.0f); }
};

// ------------------------------------------------------------------------------------------
// Portable transcendentals.  Every operation separately rounded in binary32.
// ------------------------------------------------------------------------------------------
// ln 2 split: the high part keeps 16 significant bits (so n*LN2_HI is exact for |n| < 2^8).
const float O_LN2_HI = 45426.0f / 65536.0f;
const float O_LN2_LO = (float)(0.69314718055994530942 - 45426.0 / 65536.0);
const float O_LOG2E = (float)1.44269504088896340736;

// exp: Cody-Waite reduction x = n ln2 + r, |r| <= ln2/2, then the degree-7 Taylor polynomial
// in Horner form with coefficients fl(1/k!), then scaling by 2^n in two exact steps.
float ora_expf_impl(float x) {
  if (x != x) return x;
  if (x > 88.7f) return std::numeric_limits<float>::infinity();
  if (x < -87.3f) return 0.0f;
  float n = std::nearbyint(x * O_LOG2E);            // round half to even (default mode)
  float r = (x - n * O_LN2_HI) - n * O_LN2_LO;
  const float c[8] = {1.0f, 1.0f, 0.5f, (float)(1.0 / 6.0), (float)(1.0 / 24.0),
                      (float)(1.0 / 120.0), (float)(1.0 / 720.0), (float)(1.0 / 5040.0)};
  float p = c[7];
  for (int k = 6; k >= 0; --k) p = p * r + c[k];
  int ni = (int)n;
  int h = ni / 2;
  float s1 = std::ldexp(1.0f, ni - h), s2 = std::ldexp(1.0f, h);
  return (p * s1) * s2;
}

// log for x in [2^-24, 1]: x = m 2^e with m in [sqrt(1/2), sqrt(2)); s = (m-1)/(m+1);
// log m = 2 atanh(s) = 2 (s + s^3/3 + ... + s^9/9); log x = e LN2_HI + (e LN2_LO + log m).
float ora_logf_impl(float x) {
  int e;
  float f = std::frexp(x, &e);                      // x = f 2^e, f in [0.5, 1)
  float m = f;
  if (f < 0.70710678118654752f) { m = f * 2.0f; e -= 1; }
  float s = (m - 1.0f) / (m + 1.0f);
  float t = s * s;
  float p = (float)(1.0 / 9.0);
  p = p * t + (float)(1.0 / 7.0);
  p = p * t + (float)(1.0 / 5.0);
  p = p * t + (float)(1.0 / 3.0);
  p = p * t;
  float lm = 2.0f * (s + s * p);
  float ef = (float)e;
  return ef * O_LN2_HI + (ef * O_LN2_LO + lm);
}

void ora_sincosf_impl(float phi, float* s_out, float* c_out);

}  // namespace

// sincos for phi in [0, 2pi): k = rint(phi / (pi/2)), r = phi - k pi/2 with a three-part
// Cody-Waite split of pi/2 (16 + 16 + 24 bits, computed once from long double pi), Taylor
// series (sin to r^9, cos to r^10), quadrant swap.
namespace {
struct PiSplit {
  float p1, p2, p3;
  PiSplit() {
    long double pio2 = 1.5707963267948966192313216916397514L;
    p1 = (float)(std::nearbyint((double)(pio2 * 32768.0L)) / 32768.0);
    long double rem = pio2 - (long double)p1;
    // p2: rem rounded to 16 significant bits
    int e;
    std::frexp((double)rem, &e);
    long double sc = std::ldexp(1.0L, 16 - e);
    p2 = (float)(std::nearbyint((double)(rem * sc)) / (double)sc);
    p3 = (float)(rem - (long double)p2);
  }
};
const PiSplit O_PI;

void ora_sincosf_impl(float phi, float* s_out, float* c_out) {
  const float TWO_OVER_PI = (float)0.63661977236758134308;
  float k = std::nearbyint(phi * TWO_OVER_PI);
  float r = ((phi - k * O_PI.p1) - k * O_PI.p2) - k * O_PI.p3;
  float r2 = r * r;
  const float s3 = (float)(-1.0 / 6.0), s5 = (float)(1.0 / 120.0), s7 = (float)(-1.0 / 5040.0),
              s9 = (float)(1.0 / 362880.0);
  const float c2 = -0.5f, c4 = (float)(1.0 / 24.0), c6 = (float)(-1.0 / 720.0),
              c8 = (float)(1.0 / 40320.0), c10 = (float)(-1.0 / 3628800.0);
  float ps = s9;
  ps = ps * r2 + s7;
  ps = ps * r2 + s5;
  ps = ps * r2 + s3;
  float sn = r + r * (ps * r2);
  float pc = c10;
  pc = pc * r2 + c8;
  pc = pc * r2 + c6;
  pc = pc * r2 + c4;
  pc = pc * r2 + c2;
  float cs = 1.0f + pc * r2;
  int q = ((int)k) & 3;
  switch (q) {
    case 0: *s_out = sn; *c_out = cs; break;
    case 1: *s_out = cs; *c_out = -sn; break;
    case 2: *s_out = -sn; *c_out = -cs; break;
    default: *s_out = -cs; *c_out = sn; break;
  }
}

// ------------------------------------------------------------------------------------------
// Volume: trilinear, cell-centred, clamp-to-edge lookup in the unit cube; 1D RGBA TF.
// ------------------------------------------------------------------------------------------
struct OVolume {
  const float* d; int nx, ny, nz; float dmax;
  const float* tf; int P;
  float majorant;   // dmax * max_i A_i
};

inline float olerp(float a, float b, float f) { return a + f * (b - a); }

float ora_density(const OVolume& V, float px, float py, float pz) {
  float gx = px * (float)V.nx - 0.5f, gy = py * (float)V.ny - 0.5f, gz = pz * (float)V.nz - 0.5f;
  float fx0 = std::floor(gx), fy0 = std::floor(gy), fz0 = std::floor(gz);
  float fx = gx - fx0, fy = gy - fy0, fz = gz - fz0;
  int ix = (int)fx0, iy = (int)fy0, iz = (int)fz0;
  int x0 = std::min(std::max(ix, 0), V.nx - 1), x1 = std::min(std::max(ix + 1, 0), V.nx - 1);
  int y0 = std::min(std::max(iy, 0), V.ny - 1), y1 = std::min(std::max(iy + 1, 0), V.ny - 1);
  int z0 = std::min(std::max(iz, 0), V.nz - 1), z1 = std::min(std::max(iz + 1, 0), V.nz - 1);
  auto at = [&](int x, int y, int z) { return V.d[((size_t)z * V.ny + y) * V.nx + x]; };
  float c00 = olerp(at(x0, y0, z0), at(x1, y0, z0), fx);
  float c10 = olerp(at(x0, y1, z0), at(x1, y1, z0), fx);
  float c01 = olerp(at(x0, y0, z1), at(x1, y0, z1), fx);
  float c11 = olerp(at(x0, y1, z1), at(x1, y1, z1), fx);
  float c0 = olerp(c00, c10, fy), c1 = olerp(c01, c11, fy);
  return olerp(c0, c1, fz);
}

void ora_tf(const OVolume& V, float d, float rgba[4]) {
  float s = d / V.dmax;
  s = std::fmin(std::fmax(s, 0.0f), 1.0f) * (float)(V.P - 1);
  float fi = std::floor(s);
  int i = std::min((int)fi, V.P - 2);
  float f = s - (float)i;
  for (int c = 0; c < 4; ++c) rgba[c] = olerp(V.tf[4 * i + c], V.tf[4 * (i + 1) + c], f);
}

// Extinction sigma_t = d * A(d); zero outside the unit cube.
float ora_sigma_t(const OVolume& V, float x, float y, float z) {
  if (!(x >= 0.0f && x <= 1.0f && y >= 0.0f && y <= 1.0f && z >= 0.0f && z <= 1.0f)) return 0.0f;
  float d = ora_density(V, x, y, z);
  float rgba[4];
  ora_tf(V, d, rgba);
  return d * rgba[3];
}

// Slab method against [0,1]^3.  Returns false on a miss.  t0 is clamped to >= 0.
bool ora_box(const float o[3], const float w[3], float* t0, float* t1) {
  float tmin = -std::numeric_limits<float>::infinity();
  float tmax = std::numeric_limits<float>::infinity();
  for (int a = 0; a < 3; ++a) {
    if (w[a] != 0.0f) {
      float inv = 1.0f / w[a];
      float ta = (0.0f - o[a]) * inv, tb = (1.0f - o[a]) * inv;
      tmin = std::fmax(tmin, std::fmin(ta, tb));
      tmax = std::fmin(tmax, std::fmax(ta, tb));
    } else if (o[a] < 0.0f || o[a] > 1.0f) {
      return false;
    }
  }
  float lo = std::fmax(tmin, 0.0f);
  if (!(tmax > lo)) return false;
  *t0 = lo; *t1 = tmax;
  return true;
}

struct OCam {
  float R[9], t[3], fx, fy, cx, cy;
  int full_w, full_h, x0, y0, w, h;
  float znear;
};

struct OTraceParams {
  uint64_t seed; uint32_t frame, spp, max_bounces, K;
  float C; int C_inf; float eps;
  int strategy;   // STRAT_NEE or STRAT_UNIFORM
};

// Light-transport estimators (Method: path termination heuristics): next-event estimation at
// every vertex combined with the phase-sampled continuation by multiple importance sampling,
// or the uniform (phase-sampling only) path tracer that the evaluation uses as a baseline.
enum { STRAT_NEE = 0, STRAT_UNIFORM = 1 };

// ------------------------------------------------------------------------------------------
// Spherical area lights (Evaluation: small spherical lights placed outside the volume).
// Seven floats per light: centre xyz, radius, emitted radiance rgb (uniform over the surface
// and over outgoing directions).  Every light lies outside the unit cube, so a point inside
// the cube sees each light under a cone and a ray from it reaches a light only after leaving
// the cube.
// ------------------------------------------------------------------------------------------
float odot(const float a[3], const float b[3]) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

// 1 - cos(theta_max) of the cone a sphere of radius r subtends from squared distance d2,
// written as sin^2 / (1 + cos) so that small cones keep their precision.
float ora_cone_one_minus(float r, float d2) {
  float s2 = (r * r) / d2;
  return s2 / (1.0f + std::sqrt(1.0f - s2));
}

// Nearest intersection of the ray o + t w (|w| = 1, o outside the sphere) with sphere s:
// the smaller root of t^2 - 2 t (w.(c-o)) + |c-o|^2 - r^2 = 0.  False when the ray misses
// or the sphere is behind the origin.
bool ora_sphere_hit(const float* s, const float o[3], const float w[3], float* t) {
  float oc[3] = {s[0] - o[0], s[1] - o[1], s[2] - o[2]};
  float b = odot(w, oc);
  float c = odot(oc, oc) - s[3] * s[3];
  float disc = b * b - c;
  if (!(b > 0.0f) || !(disc >= 0.0f)) return false;
  *t = b - std::sqrt(disc);
  return true;
}

// Orthonormal basis (b1, b2) completing the unit vector a (Duff, Burgess, Christensen, Hill,
// Kensler, Liani, Lyne: "Building an Orthonormal Basis, Revisited", JCGT 2017).
void ora_onb(const float a[3], float b1[3], float b2[3]) {
  float sg = std::copysign(1.0f, a[2]);
  float k = -1.0f / (sg + a[2]);
  float m = (a[0] * a[1]) * k;
  b1[0] = 1.0f + ((sg * a[0]) * a[0]) * k;
  b1[1] = sg * m;
  b1[2] = -(sg * a[0]);
  b2[0] = m;
  b2[1] = sg + (a[1] * a[1]) * k;
  b2[2] = -a[1];
}

// Radiance picked up by a ray (o, w) that has left the volume from vertex o: the emitted
// radiance of the nearest sphere light it hits (none: false), weighted for MIS against light
// sampling of that sphere from o.  Solid-angle pdfs: phase 1/(4 pi), light 1/(2 pi (1-cos)),
// so with the power heuristic the phase sample's weight is om^2 / (om^2 + 4), om = 1 - cos.
bool ora_escape_light(const float* sph, int ns, int strategy, const float o[3], const float w[3],
                      float le[3]) {
  int best = -1;
  float tbest = std::numeric_limits<float>::infinity();
  for (int s = 0; s < ns; ++s) {
    float th;
    if (ora_sphere_hit(sph + 7 * s, o, w, &th) && th < tbest) { tbest = th; best = s; }
  }
  if (best < 0) return false;
  const float* sp = sph + 7 * best;
  float wt = 1.0f;
  if (strategy == STRAT_NEE) {
    float oc[3] = {sp[0] - o[0], sp[1] - o[1], sp[2] - o[2]};
    float om = ora_cone_one_minus(sp[3], odot(oc, oc));
    wt = (om * om) / (om * om + 4.0f);
  }
  for (int c = 0; c < 3; ++c) le[c] = sp[4 + c] * wt;
  return true;
}

enum { KIND_ESCAPE0 = 0, KIND_ESCAPE = 1, KIND_MAXDEPTH = 2, KIND_EARLY = 3 };
const uint32_t MAX_STEPS = 1u << 20;   // per free-flight / shadow segment (never reached)

struct PathOut { float L[3]; float beta; int n; int kind; };

// One path (Method: path termination heuristics, Algorithm 1, Eq. 3; cache training).
PathOut ora_trace_path(const OVolume& V, const float* lights, int nl, const float* sph, int ns,
                       const OCam& cam, const OTraceParams& tp, int px, int py, uint32_t sample) {
  PathOut out{{0.f, 0.f, 0.f}, 1.0f, 0, KIND_ESCAPE0};
  uint32_t pixel = (uint32_t)py * (uint32_t)cam.full_w + (uint32_t)px;
  PathRng rng(tp.seed, pixel, sample, tp.frame);
  // Primary ray through the pixel centre (no jitter), camera -> world.
  float dc[3] = {((float)px + 0.5f - cam.cx) / cam.fx, ((float)py + 0.5f - cam.cy) / cam.fy, 1.0f};
  float nrm = std::sqrt((dc[0] * dc[0] + dc[1] * dc[1]) + dc[2] * dc[2]);
  dc[0] = dc[0] / nrm; dc[1] = dc[1] / nrm; dc[2] = dc[2] / nrm;
  const float* R = cam.R;
  float w[3], o[3];
  for (int i = 0; i < 3; ++i) w[i] = (R[0 + i] * dc[0] + R[3 + i] * dc[1]) + R[6 + i] * dc[2];
  for (int i = 0; i < 3; ++i) o[i] = -((R[0 + i] * cam.t[0] + R[3 + i] * cam.t[1]) + R[6 + i] * cam.t[2]);
  float t0, t1;
  if (!ora_box(o, w, &t0, &t1)) return out;
  const float sb = V.majorant;
  float tr_out[3] = {1.f, 1.f, 1.f}, raw[3] = {1.f, 1.f, 1.f};
  float beta = 1.0f;
  float L[3] = {0.f, 0.f, 0.f};
  int n = 0;
  const float INV4PI = (float)(0.25 / 3.14159265358979323846);
  for (;;) {
    // Free flight (delta tracking against the global majorant).
    float t = t0;
    bool collided = false;
    float x[3] = {0.f, 0.f, 0.f};
    for (uint32_t step = 0; step < MAX_STEPS; ++step) {
      float u = rng.uniform();
      t = t - ora_logf_impl(1.0f - u) / sb;
      if (t >= t1) break;
      for (int i = 0; i < 3; ++i) x[i] = o[i] + t * w[i];
      float u2 = rng.uniform();
      if (u2 < ora_sigma_t(V, x[0], x[1], x[2]) / sb) { collided = true; break; }
    }
    if (!collided) {
      // The path leaves the volume; from a vertex (not the camera) it may hit an area light.
      float le[3];
      if (n >= 1 && ora_escape_light(sph, ns, tp.strategy, o, w, le))
        for (int c = 0; c < 3; ++c) L[c] = L[c] + tr_out[c] * le[c];
      out.kind = (n == 0) ? KIND_ESCAPE0 : KIND_ESCAPE;
      break;
    }
    // The continuation after the last allowed vertex collided again: the path stops there.
    if ((uint32_t)n >= tp.max_bounces) { out.kind = KIND_MAXDEPTH; break; }
    // Real collision: vertex n.
    n += 1;
    float dd = ora_density(V, x[0], x[1], x[2]);
    float rgba[4];
    ora_tf(V, dd, rgba);
    for (int c = 0; c < 3; ++c) { raw[c] = raw[c] * rgba[c]; tr_out[c] = tr_out[c] * rgba[c]; }
    // Next-event estimation to every point light, ratio-tracked shadow transmittance.
    for (int l = 0; l < (tp.strategy == STRAT_NEE ? nl : 0); ++l) {
      const float* lp = lights + 6 * l;
      float dl[3] = {lp[0] - x[0], lp[1] - x[1], lp[2] - x[2]};
      float dist2 = (dl[0] * dl[0] + dl[1] * dl[1]) + dl[2] * dl[2];
      float dist = std::sqrt(dist2);
      float wl[3] = {dl[0] / dist, dl[1] / dist, dl[2] / dist};
      float b0, b1;
      float texit = dist;
      if (ora_box(x, wl, &b0, &b1)) texit = std::fmin(dist, b1);
      else texit = 0.0f;
      float T = 1.0f, ts = 0.0f;
      for (uint32_t step = 0; step < MAX_STEPS; ++step) {
        float u = rng.uniform();
        ts = ts - ora_logf_impl(1.0f - u) / sb;
        if (ts >= texit) break;
        float y0 = x[0] + ts * wl[0], y1 = x[1] + ts * wl[1], y2 = x[2] + ts * wl[2];
        T = T * (1.0f - ora_sigma_t(V, y0, y1, y2) / sb);
      }
      float g = (T / dist2) * INV4PI;
      for (int c = 0; c < 3; ++c) L[c] = L[c] + tr_out[c] * (lp[3 + c] * g);
    }
    // Next-event estimation to every sphere light: a direction uniform in the cone the sphere
    // subtends, its hit point, the shadow ray blocked by any other light in front of it, else
    // ratio-tracked through the volume.  Estimate phase * Le * T / p_light, times the MIS
    // weight p_light^2 / (p_light^2 + p_phase^2): together T * Le * 2 om / (om^2 + 4).
    for (int s = 0; s < (tp.strategy == STRAT_NEE ? ns : 0); ++s) {
      const float* sp = sph + 7 * s;
      float dl[3] = {sp[0] - x[0], sp[1] - x[1], sp[2] - x[2]};
      float d2 = odot(dl, dl);
      float d = std::sqrt(d2);
      float ax[3] = {dl[0] / d, dl[1] / d, dl[2] / d};
      float om = ora_cone_one_minus(sp[3], d2);
      float ua = rng.uniform(), ub = rng.uniform();
      float v = ua * om;                       // 1 - cos(theta), uniform in [0, om)
      float ct = 1.0f - v;
      float st = std::sqrt(std::fmax(0.0f, v * (2.0f - v)));
      float sphi, cphi;
      ora_sincosf_impl((float)(2.0 * 3.14159265358979323846) * ub, &sphi, &cphi);
      float b1[3], b2[3];
      ora_onb(ax, b1, b2);
      float wl[3];
      for (int i = 0; i < 3; ++i) wl[i] = ((st * cphi) * b1[i] + (st * sphi) * b2[i]) + ct * ax[i];
      // Hit distance on the sampled sphere (grazing directions: the tangent point).
      float bq = odot(wl, dl);
      float th = bq - std::sqrt(std::fmax(0.0f, bq * bq - (d2 - sp[3] * sp[3])));
      bool blocked = false;
      for (int m = 0; m < ns; ++m) {
        float tm;
        if (m != s && ora_sphere_hit(sph + 7 * m, x, wl, &tm) && tm < th) blocked = true;
      }
      if (blocked) continue;
      float b0, b1e;
      float texit = ora_box(x, wl, &b0, &b1e) ? std::fmin(th, b1e) : 0.0f;
      float T = 1.0f, ts = 0.0f;
      for (uint32_t step = 0; step < MAX_STEPS; ++step) {
        float u = rng.uniform();
        ts = ts - ora_logf_impl(1.0f - u) / sb;
        if (ts >= texit) break;
        float y0 = x[0] + ts * wl[0], y1 = x[1] + ts * wl[1], y2 = x[2] + ts * wl[2];
        T = T * (1.0f - ora_sigma_t(V, y0, y1, y2) / sb);
      }
      float g = T * ((2.0f * om) / (om * om + 4.0f));
      for (int c = 0; c < 3; ++c) L[c] = L[c] + tr_out[c] * (sp[4 + c] * g);
    }
    // After the last allowed vertex only a continuation that leaves the volume and reaches an
    // area light can still contribute; without area lights the path ends here.
    const bool last = (uint32_t)n >= tp.max_bounces;
    if (last && ns == 0) { out.kind = KIND_MAXDEPTH; break; }
    // Algorithm 1: early termination into the cache, cumulative throughput reading.
    if (!last && !tp.C_inf) {
      float lum = (0.2126f * raw[0] + 0.7152f * raw[1]) + 0.0722f * raw[2];
      float Tr = std::fmin(std::fmax(tp.C * lum, 0.0f), 1.0f);
      if (Tr < 0.9f) {
        float q = rng.uniform();
        if (q < 1.0f - Tr) { out.kind = KIND_EARLY; break; }
        for (int c = 0; c < 3; ++c) tr_out[c] = tr_out[c] / (Tr + tp.eps);
        beta = beta * Tr;
      }
    }
    // Isotropic phase function: uniform direction on the sphere.
    float u1 = rng.uniform(), u2 = rng.uniform();
    float z = 1.0f - 2.0f * u1;
    float r = std::sqrt(std::fmax(0.0f, 1.0f - z * z));
    float phi = (float)(2.0 * 3.14159265358979323846) * u2;
    float sp, cp;
    ora_sincosf_impl(phi, &sp, &cp);
    w[0] = r * cp; w[1] = r * sp; w[2] = z;
    for (int i = 0; i < 3; ++i) o[i] = x[i];
    float bb0, bb1;
    if (!ora_box(o, w, &bb0, &bb1)) {
      float le[3];
      if (ora_escape_light(sph, ns, tp.strategy, o, w, le))
        for (int c = 0; c < 3; ++c) L[c] = L[c] + tr_out[c] * le[c];
      out.kind = KIND_ESCAPE;
      break;
    }
    t0 = 0.0f; t1 = bb1;
  }
  out.L[0] = L[0]; out.L[1] = L[1]; out.L[2] = L[2];
  out.beta = beta; out.n = n;
  return out;
}

// ------------------------------------------------------------------------------------------
// Projection (fp32, bit-exact contract): activations, 3D covariance, EWA 2D covariance with
// 0.3 px^2 dilation, conic, 3-sigma radius, integer pixel window clamped to the render window,
// tile rectangle.
// ------------------------------------------------------------------------------------------
struct OProj {
  float u, v, A, B, Cc, o, z;
  int px0, px1, py0, py1;     // inclusive pixel window (full-frame)
  int tx0, tx1, ty0, ty1;     // inclusive tile rect (window-local)
  uint32_t tiles;             // 0 when culled
  int culled;
  float radius;
};

OProj ora_project_one(const float* pos, const float* rot, const float* ls, float logit,
                      const OCam& cam) {
  OProj P{};
  P.culled = 1; P.tiles = 0;
  float qw = rot[0], qx = rot[1], qy = rot[2], qz = rot[3];
  float qq = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  float qn = std::sqrt(qq);
  qw = qw / qn; qx = qx / qn; qy = qy / qn; qz = qz / qn;
  float Rq[9];
  Rq[0] = 1.0f - 2.0f * (qy * qy + qz * qz);
  Rq[1] = 2.0f * (qx * qy - qw * qz);
  Rq[2] = 2.0f * (qx * qz + qw * qy);
  Rq[3] = 2.0f * (qx * qy + qw * qz);
  Rq[4] = 1.0f - 2.0f * (qx * qx + qz * qz);
  Rq[5] = 2.0f * (qy * qz - qw * qx);
  Rq[6] = 2.0f * (qx * qz - qw * qy);
  Rq[7] = 2.0f * (qy * qz + qw * qx);
  Rq[8] = 1.0f - 2.0f * (qx * qx + qy * qy);
  float s[3] = {ora_expf_impl(ls[0]), ora_expf_impl(ls[1]), ora_expf_impl(ls[2])};
  P.o = 1.0f / (1.0f + ora_expf_impl(-logit));
  float M[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[3 * i + j] = Rq[3 * i + j] * s[j];
  float S[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      S[3 * i + j] = (M[3 * i + 0] * M[3 * j + 0] + M[3 * i + 1] * M[3 * j + 1]) + M[3 * i + 2] * M[3 * j + 2];
  const float* Rc = cam.R;
  float xc[3];
  for (int i = 0; i < 3; ++i)
    xc[i] = ((Rc[3 * i + 0] * pos[0] + Rc[3 * i + 1] * pos[1]) + Rc[3 * i + 2] * pos[2]) + cam.t[i];
  float x = xc[0], y = xc[1], z = xc[2];
  P.z = z;
  if (!(z > cam.znear) || !std::isfinite(x) || !std::isfinite(y)) return P;
  float iz = 1.0f / z;
  float limx = 1.3f * ((float)cam.full_w / (2.0f * cam.fx));
  float limy = 1.3f * ((float)cam.full_h / (2.0f * cam.fy));
  float txz = std::fmin(std::fmax(x * iz, -limx), limx);
  float tyz = std::fmin(std::fmax(y * iz, -limy), limy);
  float tx = txz * z, ty = tyz * z;
  float iz2 = iz * iz;
  float J00 = cam.fx * iz, J02 = -(cam.fx * tx) * iz2;
  float J11 = cam.fy * iz, J12 = -(cam.fy * ty) * iz2;
  float T[6];
  for (int j = 0; j < 3; ++j) {
    T[j] = J00 * Rc[j] + J02 * Rc[6 + j];
    T[3 + j] = J11 * Rc[3 + j] + J12 * Rc[6 + j];
  }
  float U[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j)
      U[3 * i + j] = (T[3 * i + 0] * S[0 + j] + T[3 * i + 1] * S[3 + j]) + T[3 * i + 2] * S[6 + j];
  float s00 = (U[0] * T[0] + U[1] * T[1]) + U[2] * T[2];
  float s01 = (U[0] * T[3] + U[1] * T[4]) + U[2] * T[5];
  float s11 = (U[3] * T[3] + U[4] * T[4]) + U[5] * T[5];
  float a = s00 + 0.3f, b = s01, c = s11 + 0.3f;
  float det = a * c - b * b;
  if (!(det > 0.0f)) return P;
  P.A = c / det; P.B = (-b) / det; P.Cc = a / det;
  float mid = 0.5f * (a + c);
  float lam = mid + std::sqrt(std::fmax(0.1f, mid * mid - det));
  float r = std::ceil(3.0f * std::sqrt(lam));
  P.radius = r;
  P.u = cam.fx * (x * iz) + (cam.cx - 0.5f);
  P.v = cam.fy * (y * iz) + (cam.cy - 0.5f);
  float fx0 = std::fmax((float)cam.x0, std::ceil(P.u - r));
  float fx1 = std::fmin((float)(cam.x0 + cam.w - 1), std::floor(P.u + r));
  float fy0 = std::fmax((float)cam.y0, std::ceil(P.v - r));
  float fy1 = std::fmin((float)(cam.y0 + cam.h - 1), std::floor(P.v + r));
  if (!(fx0 <= fx1) || !(fy0 <= fy1)) return P;
  P.px0 = (int)fx0; P.px1 = (int)fx1; P.py0 = (int)fy0; P.py1 = (int)fy1;
  P.tx0 = (P.px0 - cam.x0) / 16; P.tx1 = (P.px1 - cam.x0) / 16;
  P.ty0 = (P.py0 - cam.y0) / 16; P.ty1 = (P.py1 - cam.y0) / 16;
  P.tiles = (uint32_t)((P.tx1 - P.tx0 + 1) * (P.ty1 - P.ty0 + 1));
  P.culled = 0;
  return P;
}

inline uint32_t fbits(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }

OCam make_cam(const float* R, const float* t, const float* intr, const int* win, float znear) {
  OCam c;
  for (int i = 0; i < 9; ++i) c.R[i] = R[i];
  for (int i = 0; i < 3; ++i) c.t[i] = t[i];
  c.fx = intr[0]; c.fy = intr[1]; c.cx = intr[2]; c.cy = intr[3];
  c.full_w = win[0]; c.full_h = win[1]; c.x0 = win[2]; c.y0 = win[3]; c.w = win[4]; c.h = win[5];
  c.znear = znear;
  return c;
}

// Forward decisions for one pixel, fp32, given the depth-sorted covering list.
struct Blend { float C[3]; float T; int last; int nblend; int boundary; };

}  // namespace

extern "C" {

// ------------------------------------------------------------------------------------------
// Exported test entry points.  Camera arguments: R[9] row-major world->camera, t[3],
// intr = (fx, fy, cx, cy), win = (full_w, full_h, x0, y0, w, h), znear.
// ------------------------------------------------------------------------------------------
int ora_num_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// The constants of the portable transcendentals, for inspection by the tests.
void ora_constants(float* out) {
  out[0] = O_LN2_HI; out[1] = O_LN2_LO; out[2] = O_LOG2E;
  out[3] = O_PI.p1; out[4] = O_PI.p2; out[5] = O_PI.p3;
}

void ora_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  Philox::block(ctr, key, out);
}

// Draws k = 0..n-1 of the path stream (seed, pixel, sample, frame) as uniforms.
void ora_path_uniforms(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t frame, int n,
                       float* out) {
  PathRng r(seed, pixel, sample, frame);
  for (int i = 0; i < n; ++i) out[i] = r.uniform();
}

void ora_expf(const float* x, float* y, int64_t n) { for (int64_t i = 0; i < n; ++i) y[i] = ora_expf_impl(x[i]); }
void ora_logf(const float* x, float* y, int64_t n) { for (int64_t i = 0; i < n; ++i) y[i] = ora_logf_impl(x[i]); }
void ora_sincosf(const float* x, float* s, float* c, int64_t n) {
  for (int64_t i = 0; i < n; ++i) ora_sincosf_impl(x[i], &s[i], &c[i]);
}

void ora_density_at(const float* d, int nx, int ny, int nz, const float* p, int64_t n, float* out) {
  OVolume V{d, nx, ny, nz, 1.0f, nullptr, 0, 0.0f};
  for (int64_t i = 0; i < n; ++i) out[i] = ora_density(V, p[3 * i], p[3 * i + 1], p[3 * i + 2]);
}

void ora_tf_at(const float* tf, int P, float dmax, const float* d, int64_t n, float* out) {
  OVolume V{nullptr, 0, 0, 0, dmax, tf, P, 0.0f};
  for (int64_t i = 0; i < n; ++i) ora_tf(V, d[i], out + 4 * i);
}

// Transmittance estimate along a straight segment by ratio tracking (used by the NEE pins).
// Returns the mean of `n` independent estimates using stream (seed, i, 0, 0).
double ora_ratio_tracking_mean(const float* d, int nx, int ny, int nz, float dmax, const float* tf,
                               int P, const float* o, const float* w, float tmax, uint64_t seed,
                               int n) {
  float amax = 0.f;
  for (int i = 0; i < P; ++i) amax = std::fmax(amax, tf[4 * i + 3]);
  OVolume V{d, nx, ny, nz, dmax, tf, P, dmax * amax};
  double acc = 0.0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
  for (int i = 0; i < n; ++i) {
    PathRng r(seed, (uint32_t)i, 0, 0);
    float T = 1.0f, ts = 0.0f;
    for (;;) {
      float u = r.uniform();
      ts = ts - ora_logf_impl(1.0f - u) / V.majorant;
      if (ts >= tmax) break;
      T = T * (1.0f - ora_sigma_t(V, o[0] + ts * w[0], o[1] + ts * w[1], o[2] + ts * w[2]) / V.majorant);
    }
    acc += T;
  }
  return acc / n;
}

// The tracer.  targets [K][h][w][3] receive the per-level mean over spp of the path's NEE
// radiance (written to level min(n, K) - 1, zero elsewhere); targets_sq (optional) the per-level
// mean of squares; records (optional) [spp][h][w], five words per path:
// L[3] (f32), beta (f32), n | kind << 16 (u32); kind_counts (optional) [h][w][4] per-kind counts.
int ora_trace(const float* density, int nx, int ny, int nz, float dmax, const float* tf, int P,
              const float* lights, int nl, const float* spheres, int ns, int strategy,
              const float* R, const float* t, const float* intr,
              const int* win, float znear, uint64_t seed, uint32_t frame, uint32_t spp,
              uint32_t max_bounces, uint32_t K, float C, int C_inf, float eps, float* targets,
              float* targets_sq, uint32_t* records, uint32_t* path_stats, uint32_t* kind_counts) {
  float amax = 0.f;
  for (int i = 0; i < P; ++i) amax = std::fmax(amax, tf[4 * i + 3]);
  OVolume V{density, nx, ny, nz, dmax, tf, P, dmax * amax};
  OCam cam = make_cam(R, t, intr, win, znear);
  OTraceParams tp{seed, frame, spp, max_bounces, K, C, C_inf, eps, strategy};
  const int W = cam.w, H = cam.h;
  const size_t plane = (size_t)W * H;
  std::memset(targets, 0, sizeof(float) * 3 * plane * K);
  if (targets_sq) std::memset(targets_sq, 0, sizeof(float) * 3 * plane * K);
  if (kind_counts) std::memset(kind_counts, 0, sizeof(uint32_t) * 4 * plane);
  uint64_t total_len = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total_len)
  for (int64_t p = 0; p < (int64_t)plane; ++p) {
    int lx = (int)(p % W), ly = (int)(p / W);
    int px = cam.x0 + lx, py = cam.y0 + ly;
    std::vector<float> sum(3 * K, 0.f), sq(3 * K, 0.f);
    for (uint32_t s = 0; s < spp; ++s) {
      PathOut po = ora_trace_path(V, lights, nl, spheres, ns, cam, tp, px, py, s);
      if (records) {
        uint32_t* rec = records + 5 * ((size_t)s * plane + p);
        std::memcpy(&rec[0], &po.L[0], 4);
        std::memcpy(&rec[1], &po.L[1], 4);
        std::memcpy(&rec[2], &po.L[2], 4);
        std::memcpy(&rec[3], &po.beta, 4);
        rec[4] = (uint32_t)po.n | ((uint32_t)po.kind << 16);
      }
      total_len += (uint64_t)po.n;
      if (kind_counts) kind_counts[4 * p + po.kind] += 1u;
      if (po.n >= 1) {
        uint32_t lvl = std::min((uint32_t)po.n, K) - 1;
        for (int c = 0; c < 3; ++c) {
          sum[3 * lvl + c] = sum[3 * lvl + c] + po.L[c];
          sq[3 * lvl + c] = sq[3 * lvl + c] + po.L[c] * po.L[c];
        }
      }
    }
    for (uint32_t l = 0; l < K; ++l)
      for (int c = 0; c < 3; ++c) {
        size_t idx = ((size_t)l * plane + p) * 3 + c;
        targets[idx] = (spp == 1) ? sum[3 * l + c] : sum[3 * l + c] / (float)spp;
        if (targets_sq) targets_sq[idx] = (spp == 1) ? sq[3 * l + c] : sq[3 * l + c] / (float)spp;
      }
  }
  if (path_stats) { path_stats[0] = (uint32_t)(total_len & 0xFFFFFFFFu); path_stats[1] = (uint32_t)(total_len >> 32); }
  return 0;
}

// Projection of n Gaussians.  Outputs (each optional): screen [n][6] = (u, v, A, B, Cc, o),
// depth [n], window [n][4] = (px0, px1, py0, py1), rect [n][4] = (tx0, tx1, ty0, ty1),
// tiles [n] (0 when culled), radius [n].
void ora_project(const float* pos, const float* rot, const float* ls, const float* logit, int64_t n,
                 const float* R, const float* t, const float* intr, const int* win, float znear,
                 float* screen, float* depth, int32_t* window, int32_t* rect, uint32_t* tiles,
                 float* radius) {
  OCam cam = make_cam(R, t, intr, win, znear);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    OProj P = ora_project_one(pos + 3 * i, rot + 4 * i, ls + 3 * i, logit[i], cam);
    if (screen) { float* s = screen + 6 * i; s[0] = P.u; s[1] = P.v; s[2] = P.A; s[3] = P.B; s[4] = P.Cc; s[5] = P.o; }
    if (depth) depth[i] = P.z;
    if (window) { int32_t* w = window + 4 * i; w[0] = P.px0; w[1] = P.px1; w[2] = P.py0; w[3] = P.py1; if (P.culled) w[0] = w[1] = w[2] = w[3] = 0; }
    if (rect) { int32_t* r = rect + 4 * i; r[0] = P.tx0; r[1] = P.tx1; r[2] = P.ty0; r[3] = P.ty1; if (P.culled) r[0] = r[1] = r[2] = r[3] = 0; }
    if (tiles) tiles[i] = P.tiles;
    if (radius) radius[i] = P.culled ? 0.0f : P.radius;
  }
}

// Binning of one level, plain definition: for every non-culled Gaussian in id order and every
// tile of its rect in row-major order, the pair (key = (tile_base + ty*TX + tx) << 32 | bits(z),
// value = id); then sort by (key, value).  Returns the pair count; keys/values may be NULL to
// only count.
int64_t ora_bin_level(const float* depth, const int32_t* rect, const uint32_t* tiles, int64_t n,
                      int TX, uint32_t tile_base, uint64_t* keys, uint32_t* values) {
  int64_t total = 0;
  for (int64_t i = 0; i < n; ++i) total += tiles[i];
  if (!keys) return total;
  std::vector<std::pair<uint64_t, uint32_t>> pairs;
  pairs.reserve((size_t)total);
  for (int64_t i = 0; i < n; ++i) {
    if (tiles[i] == 0) continue;
    const int32_t* r = rect + 4 * i;
    for (int ty = r[2]; ty <= r[3]; ++ty)
      for (int tx = r[0]; tx <= r[1]; ++tx) {
        uint64_t tile = (uint64_t)tile_base + (uint64_t)ty * (uint64_t)TX + (uint64_t)tx;
        pairs.emplace_back((tile << 32) | fbits(depth[i]), (uint32_t)i);
      }
  }
  std::sort(pairs.begin(), pairs.end());
  for (size_t k = 0; k < pairs.size(); ++k) { keys[k] = pairs[k].first; values[k] = pairs[k].second; }
  return total;
}

// Per-tile [start, end) over the sorted key array; an empty tile gets (0, 0).
void ora_tile_ranges(const uint64_t* keys, int64_t n_keys, int64_t n_tiles, uint64_t* ranges) {
  for (int64_t tt = 0; tt < n_tiles; ++tt) { ranges[2 * tt] = 0; ranges[2 * tt + 1] = 0; }
  for (int64_t i = 0; i < n_keys; ++i) {
    uint64_t tile = keys[i] >> 32;
    if (i == 0 || (keys[i - 1] >> 32) != tile) ranges[2 * tile] = (uint64_t)i;
    ranges[2 * tile + 1] = (uint64_t)i + 1;
  }
}

// Brute-force forward splatting of one level, fp32 (no tiles).  For each pixel (i, j) of the
// render window: list = every non-culled Gaussian whose pixel window contains (i, j), sorted by
// (bits(depth), id); blend front to back with alpha = min(0.99, o exp(power)), skipping
// power > 0 and alpha < 1/255, stopping before T (1 - alpha) < 1e-4.
// Outputs image [h][w][3], final_T [h][w], last_id [h][w] (-1 when none), n_blend [h][w],
// boundary [h][w] (1 when a decision lies within the stated margins of its threshold).
// If list_off != NULL (size h*w + 1, exclusive prefix of n_blend filled by a first call) the
// blended ids are written to list_ids in blend order.
void ora_forward(const float* screen, const float* depth, const int32_t* window, const uint32_t* tiles,
                 const float* rgb, int64_t n, const int* win, float* image, float* final_T,
                 int32_t* last_id, int32_t* n_blend, uint8_t* boundary, const int64_t* list_off,
                 int32_t* list_ids, int64_t* pair_tests, int64_t* contributing) {
  const int x0 = win[2], y0 = win[3], W = win[4], H = win[5];
  std::vector<int64_t> live;
  for (int64_t g = 0; g < n; ++g) if (tiles[g] != 0) live.push_back(g);
  std::sort(live.begin(), live.end(), [&](int64_t a, int64_t b) {
    uint32_t ka = fbits(depth[a]), kb = fbits(depth[b]);
    return ka != kb ? ka < kb : a < b;
  });
  const float ALPHA_MIN = 1.0f / 255.0f;
  // Boundary flags: the GPU evaluates power, (1 - alpha) and T in the same fp32 operation order,
  // so its decisions can differ from these only through the exponential (a hardware exp within
  // EPS_EXP relative of a correctly rounded one for the arguments alpha >= 1/255 allows).  A
  // pixel is flagged when a decision lies within that uncertainty of its threshold: alpha vs
  // 1/255, o exp(power) vs the 0.99 clamp, and T (1 - alpha) vs 1e-4, whose relative
  // uncertainty accumulates EPS_EXP alpha / (1 - alpha) per blended pair.
  const double EPS_EXP = 5e-7;
  int64_t tests = 0, contrib = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : tests, contrib)
  for (int64_t p = 0; p < (int64_t)W * H; ++p) {
    int i = x0 + (int)(p % W), j = y0 + (int)(p / W);
    float T = 1.0f, C[3] = {0.f, 0.f, 0.f};
    int last = -1, nb = 0, bnd = 0;
    double terr = 0.0;
    int64_t wr = list_off ? list_off[p] : 0;
    for (size_t k = 0; k < live.size(); ++k) {
      int64_t g = live[k];
      const int32_t* wd = window + 4 * g;
      ++tests;
      if (i < wd[0] || i > wd[1] || j < wd[2] || j > wd[3]) continue;
      const float* s = screen + 6 * g;
      float dx = s[0] - (float)i, dy = s[1] - (float)j;
      float power = -0.5f * ((s[2] * dx) * dx + (s[4] * dy) * dy) - (s[3] * dx) * dy;
      if (power > 0.0f) continue;
      float e = std::exp(power);
      float oe = s[5] * e;
      if (std::fabs((double)oe - 0.99) <= EPS_EXP * oe) bnd = 1;
      float alpha = std::fmin(0.99f, oe);
      if (std::fabs((double)alpha - (double)ALPHA_MIN) <= EPS_EXP * alpha) bnd = 1;
      if (alpha < ALPHA_MIN) continue;
      float Tn = T * (1.0f - alpha);
      double da = (oe > 0.99f) ? 0.0 : EPS_EXP * alpha / (1.0 - alpha);
      if (std::fabs((double)Tn - 1e-4) <= 1e-4 * (terr + da + 1e-7)) bnd = 1;
      if (Tn < 1e-4f) break;
      for (int c = 0; c < 3; ++c) C[c] = C[c] + rgb[3 * g + c] * (alpha * T);
      T = Tn;
      terr += da;
      last = (int)g;
      ++contrib;
      if (list_off) list_ids[wr++] = (int32_t)g;
      ++nb;
    }
    image[3 * p] = C[0]; image[3 * p + 1] = C[1]; image[3 * p + 2] = C[2];
    final_T[p] = T;
    last_id[p] = last;
    if (n_blend) n_blend[p] = nb;
    if (boundary) boundary[p] = (uint8_t)bnd;
  }
  if (pair_tests) *pair_tests = tests;
  if (contributing) *contributing = contrib;
}


}  // extern "C"

// ------------------------------------------------------------------------------------------
// fp64 forward (plain mathematics in double, std::exp), for finite-difference pins of the
// gradient.  Same definitions as the fp32 path; decisions are taken in double.
// ------------------------------------------------------------------------------------------
namespace {
struct DProj { double u, v, A, B, Cc, o, z; double px0, px1, py0, py1; int culled; };

DProj ora_project_one_f64(const double* posf, const double* rotf, const double* lsf,
                          double logitf, const OCam& cam) {
  DProj P{};
  P.culled = 1;
  double pos[3] = {posf[0], posf[1], posf[2]};
  double qw = rotf[0], qx = rotf[1], qy = rotf[2], qz = rotf[3];
  double qn = std::sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  qw /= qn; qx /= qn; qy /= qn; qz /= qn;
  double Rq[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                  2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                  2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
  double s[3] = {std::exp((double)lsf[0]), std::exp((double)lsf[1]), std::exp((double)lsf[2])};
  P.o = 1.0 / (1.0 + std::exp(-(double)logitf));
  double M[9], S[9];
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) M[3 * i + j] = Rq[3 * i + j] * s[j];
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j)
    S[3 * i + j] = M[3 * i] * M[3 * j] + M[3 * i + 1] * M[3 * j + 1] + M[3 * i + 2] * M[3 * j + 2];
  double Rc[9], tc[3];
  for (int i = 0; i < 9; ++i) Rc[i] = cam.R[i];
  for (int i = 0; i < 3; ++i) tc[i] = cam.t[i];
  double xc[3];
  for (int i = 0; i < 3; ++i) xc[i] = Rc[3 * i] * pos[0] + Rc[3 * i + 1] * pos[1] + Rc[3 * i + 2] * pos[2] + tc[i];
  double x = xc[0], y = xc[1], z = xc[2];
  P.z = z;
  if (!(z > (double)cam.znear)) return P;
  double fx = cam.fx, fy = cam.fy;
  double limx = 1.3 * ((double)cam.full_w / (2.0 * fx)), limy = 1.3 * ((double)cam.full_h / (2.0 * fy));
  double tx = std::fmin(std::fmax(x / z, -limx), limx) * z;
  double ty = std::fmin(std::fmax(y / z, -limy), limy) * z;
  double J00 = fx / z, J02 = -fx * tx / (z * z), J11 = fy / z, J12 = -fy * ty / (z * z);
  double T[6];
  for (int j = 0; j < 3; ++j) { T[j] = J00 * Rc[j] + J02 * Rc[6 + j]; T[3 + j] = J11 * Rc[3 + j] + J12 * Rc[6 + j]; }
  double U[6];
  for (int i = 0; i < 2; ++i) for (int j = 0; j < 3; ++j)
    U[3 * i + j] = T[3 * i] * S[j] + T[3 * i + 1] * S[3 + j] + T[3 * i + 2] * S[6 + j];
  double a = U[0] * T[0] + U[1] * T[1] + U[2] * T[2] + 0.3;
  double b = U[0] * T[3] + U[1] * T[4] + U[2] * T[5];
  double c = U[3] * T[3] + U[4] * T[4] + U[5] * T[5] + 0.3;
  double det = a * c - b * b;
  if (!(det > 0)) return P;
  P.A = c / det; P.B = -b / det; P.Cc = a / det;
  double mid = 0.5 * (a + c);
  double r = std::ceil(3.0 * std::sqrt(mid + std::sqrt(std::fmax(0.1, mid * mid - det))));
  P.u = fx * (x / z) + ((double)cam.cx - 0.5);
  P.v = fy * (y / z) + ((double)cam.cy - 0.5);
  P.px0 = std::fmax((double)cam.x0, std::ceil(P.u - r));
  P.px1 = std::fmin((double)(cam.x0 + cam.w - 1), std::floor(P.u + r));
  P.py0 = std::fmax((double)cam.y0, std::ceil(P.v - r));
  P.py1 = std::fmin((double)(cam.y0 + cam.h - 1), std::floor(P.v + r));
  if (!(P.px0 <= P.px1) || !(P.py0 <= P.py1)) return P;
  P.culled = 0;
  return P;
}
}  // namespace

extern "C" {
// image [h][w][3] (double) and a per-pixel signature of the blended set and clamp states.
void ora_forward_f64(const double* pos, const double* rot, const double* ls, const double* logit,
                     const double* rgb, int64_t n, const float* R, const float* t, const float* intr,
                     const int* win, float znear, double* image, uint64_t* sig) {
  OCam cam = make_cam(R, t, intr, win, znear);
  std::vector<DProj> P((size_t)n);
  for (int64_t g = 0; g < n; ++g) P[g] = ora_project_one_f64(pos + 3 * g, rot + 4 * g, ls + 3 * g, logit[g], cam);
  std::vector<int64_t> live;
  for (int64_t g = 0; g < n; ++g) if (!P[g].culled) live.push_back(g);
  std::sort(live.begin(), live.end(), [&](int64_t a, int64_t b) {
    return P[a].z != P[b].z ? P[a].z < P[b].z : a < b;
  });
  const int W = cam.w, H = cam.h;
  for (int64_t p = 0; p < (int64_t)W * H; ++p) {
    double i = cam.x0 + (double)(p % W), j = cam.y0 + (double)(p / W);
    double T = 1.0, C[3] = {0, 0, 0};
    uint64_t h = 1469598103934665603ull;
    for (int64_t g : live) {
      const DProj& q = P[g];
      if (i < q.px0 || i > q.px1 || j < q.py0 || j > q.py1) continue;
      double dx = q.u - i, dy = q.v - j;
      double power = -0.5 * (q.A * dx * dx + q.Cc * dy * dy) - q.B * dx * dy;
      if (power > 0) continue;
      double oe = q.o * std::exp(power);
      int clamped = oe > 0.99;
      double alpha = clamped ? 0.99 : oe;
      if (alpha < 1.0 / 255.0) continue;
      double Tn = T * (1 - alpha);
      if (Tn < 1e-4) break;
      for (int c = 0; c < 3; ++c) C[c] += rgb[3 * g + c] * alpha * T;
      T = Tn;
      h = (h ^ (uint64_t)(2 * g + clamped)) * 1099511628211ull;
    }
    image[3 * p] = C[0]; image[3 * p + 1] = C[1]; image[3 * p + 2] = C[2];
    sig[p] = h;
  }
}
}  // extern "C"

// ------------------------------------------------------------------------------------------
// Cache initialisation points (Method: "Cache Initialization"): random rays are tracked through
// the volume by delta tracking until their first real interaction, whose position and albedo
// are recorded; a ray that leaves the volume is replaced by a fresh one.  Point i, attempt a
// draws from the Philox stream with counter (i, a, 0x494E4954, block): p = (u0, u1, u2) uniform
// in the cube, direction w from (u3, u4) uniform on the sphere (as the phase function), the ray
// starts at p - 2 w (outside the cube, through p), then free flight as in the tracer.
// ------------------------------------------------------------------------------------------
extern "C" {

int ora_init_points(const float* density, int nx, int ny, int nz, float dmax, const float* tf,
                    int P, int64_t n, uint64_t seed, int max_attempts, float* pos, float* albedo,
                    int32_t* attempts) {
  OVolume V{density, nx, ny, nz, dmax, tf, P, 0.0f};
  float amax = 0.0f;
  for (int i = 0; i < P; ++i) amax = std::fmax(amax, tf[4 * i + 3]);
  V.majorant = dmax * amax;
  const float sb = V.majorant;
  int failed = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(| : failed)
  for (int64_t i = 0; i < n; ++i) {
    bool found = false;
    int a = 0;
    for (; a < max_attempts && !found; ++a) {
      PathRng rng(seed, (uint32_t)i, (uint32_t)a, 0x494E4954u);
      float p[3];
      for (int k = 0; k < 3; ++k) p[k] = rng.uniform();
      float u3 = rng.uniform(), u4 = rng.uniform();
      float z = 1.0f - 2.0f * u3;
      float r = std::sqrt(std::fmax(0.0f, 1.0f - z * z));
      float phi = (float)(2.0 * 3.14159265358979323846) * u4;
      float sp, cp;
      ora_sincosf_impl(phi, &sp, &cp);
      float w[3] = {r * cp, r * sp, z};
      float o[3];
      for (int k = 0; k < 3; ++k) o[k] = p[k] - 2.0f * w[k];
      float t0, t1;
      if (!ora_box(o, w, &t0, &t1)) continue;
      float t = t0;
      for (uint32_t step = 0; step < MAX_STEPS; ++step) {
        float u = rng.uniform();
        t = t - ora_logf_impl(1.0f - u) / sb;
        if (t >= t1) break;
        float x[3];
        for (int k = 0; k < 3; ++k) x[k] = o[k] + t * w[k];
        float u2 = rng.uniform();
        if (u2 < ora_sigma_t(V, x[0], x[1], x[2]) / sb) {
          float d = ora_density(V, x[0], x[1], x[2]);
          float rgba[4];
          ora_tf(V, d, rgba);
          for (int k = 0; k < 3; ++k) { pos[3 * i + k] = x[k]; albedo[3 * i + k] = rgba[k]; }
          found = true;
          break;
        }
      }
    }
    attempts[i] = a;
    if (!found) failed = 1;
  }
  return failed;
}

}  // extern "C"
