// k_trace.hip -- the volume path tracer that produces GSCache's per-path-length training targets.
//
// One lane per pixel of a request, one path per sample: delta tracking against the global
// majorant (free flight), albedo-weighted real collisions, next-event estimation to every
// point light and every spherical area light (cone sampling, combined with the phase-sampled
// continuation that reaches the light by the power heuristic) with ratio-tracked shadow
// transmittance and the isotropic phase function, or phase sampling alone (the uniform
// baseline of the evaluation),
// Algorithm 1's early termination (cumulative throughput reading: the throughput is divided
// by the survival probability Tr and beta multiplied by it), uniform sphere directions.  The
// NEE radiance accumulated along the path is written to the target of its length (Method:
// "Path Termination Heuristics", "Throughput Importance Sampling", "Cascaded Cache Radiance
// Importance Sampling", "Cache Training").  Every fp32 operation is separately rounded in a
// fixed order, and the random numbers come from each pixel's own Philox stream, so the output
// does not depend on the launch shape.
#include "gsc_dev.h"

namespace gsc {

namespace {

constexpr uint32_t kMaxSteps = 1u << 20;   // per free-flight / shadow segment (never reached)
constexpr int kTraceBlock = 256;

struct Vol {
  const float* d;
  const float4* cells;     // cell-corner layout, or NULL for the plain grid
  int nx, ny, nz;
  float dmax;
  const float* tf;
  int P;
};

__device__ __forceinline__ float lerpf_(float a, float b, float f) { return a + f * (b - a); }

// Trilinear, cell-centred, clamp-to-edge density at a point of the unit cube.  The eight taps
// come either from the cell-corner copy (one 32-byte block per lookup) or from the plain grid;
// both give the same values and the interpolation is the same.
__device__ __forceinline__ float density(const Vol& V, float px, float py, float pz) {
  const float gx = px * (float)V.nx - 0.5f, gy = py * (float)V.ny - 0.5f, gz = pz * (float)V.nz - 0.5f;
  const float ix = floorf(gx), iy = floorf(gy), iz = floorf(gz);
  const float fx = gx - ix, fy = gy - iy, fz = gz - iz;
  const int x0i = (int)ix, y0i = (int)iy, z0i = (int)iz;
  float c00, c10, c01, c11;
  if (V.cells) {
    // Inside the cube x0i, y0i, z0i lie in [-1, n - 1]; clamp anyway so a lookup never leaves
    // the array.
    const int cx = min(max(x0i, -1), V.nx - 1) + 1, cy = min(max(y0i, -1), V.ny - 1) + 1;
    const int cz = min(max(z0i, -1), V.nz - 1) + 1;
    const int64_t ci = ((int64_t)cz * (V.ny + 1) + cy) * (V.nx + 1) + cx;
    const float4 a = V.cells[2 * ci], b = V.cells[2 * ci + 1];
    c00 = lerpf_(a.x, a.y, fx);
    c10 = lerpf_(a.z, a.w, fx);
    c01 = lerpf_(b.x, b.y, fx);
    c11 = lerpf_(b.z, b.w, fx);
  } else {
    const int x0 = min(max(x0i, 0), V.nx - 1), x1 = min(max(x0i + 1, 0), V.nx - 1);
    const int y0 = min(max(y0i, 0), V.ny - 1), y1 = min(max(y0i + 1, 0), V.ny - 1);
    const int z0 = min(max(z0i, 0), V.nz - 1), z1 = min(max(z0i + 1, 0), V.nz - 1);
    const int64_t sy = V.nx, sz = (int64_t)V.nx * V.ny;
    const float* p00 = V.d + z0 * sz + y0 * sy;
    const float* p10 = V.d + z0 * sz + y1 * sy;
    const float* p01 = V.d + z1 * sz + y0 * sy;
    const float* p11 = V.d + z1 * sz + y1 * sy;
    c00 = lerpf_(p00[x0], p00[x1], fx);
    c10 = lerpf_(p10[x0], p10[x1], fx);
    c01 = lerpf_(p01[x0], p01[x1], fx);
    c11 = lerpf_(p11[x0], p11[x1], fx);
  }
  const float c0 = lerpf_(c00, c10, fy), c1 = lerpf_(c01, c11, fy);
  return lerpf_(c0, c1, fz);
}

__device__ __forceinline__ void transfer(const Vol& V, float d, float* r, float* g, float* b, float* a) {
  float s = d / V.dmax;
  s = fminf(fmaxf(s, 0.0f), 1.0f) * (float)(V.P - 1);
  const int i = min((int)floorf(s), V.P - 2);
  const float f = s - (float)i;
  const float* c0 = V.tf + 4 * i;
  const float* c1 = c0 + 4;
  *r = lerpf_(c0[0], c1[0], f);
  *g = lerpf_(c0[1], c1[1], f);
  *b = lerpf_(c0[2], c1[2], f);
  *a = lerpf_(c0[3], c1[3], f);
}

__device__ __forceinline__ float opacity_only(const Vol& V, float d) {
  float s = d / V.dmax;
  s = fminf(fmaxf(s, 0.0f), 1.0f) * (float)(V.P - 1);
  const int i = min((int)floorf(s), V.P - 2);
  const float f = s - (float)i;
  return lerpf_(V.tf[4 * i + 3], V.tf[4 * i + 7], f);
}

__device__ __forceinline__ bool inside_cube(float x, float y, float z) {
  return x >= 0.0f && x <= 1.0f && y >= 0.0f && y <= 1.0f && z >= 0.0f && z <= 1.0f;
}

// sigma_t = d A(d) inside the unit cube, 0 outside; also returns d.
__device__ __forceinline__ float sigma_t(const Vol& V, float x, float y, float z, float* dout) {
  if (!inside_cube(x, y, z)) { *dout = 0.0f; return 0.0f; }
  const float d = density(V, x, y, z);
  *dout = d;
  return d * opacity_only(V, d);
}

// Slab test against [0,1]^3.
__device__ __forceinline__ bool box(float ox, float oy, float oz, float wx, float wy, float wz,
                                    float* t0, float* t1) {
  float tmin = -__int_as_float(0x7f800000), tmax = __int_as_float(0x7f800000);
  const float o[3] = {ox, oy, oz}, w[3] = {wx, wy, wz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (w[a] != 0.0f) {
      const float inv = 1.0f / w[a];
      const float ta = (0.0f - o[a]) * inv, tb = (1.0f - o[a]) * inv;
      tmin = fmaxf(tmin, fminf(ta, tb));
      tmax = fminf(tmax, fmaxf(ta, tb));
    } else if (o[a] < 0.0f || o[a] > 1.0f) {
      return false;
    }
  }
  const float lo = fmaxf(tmin, 0.0f);
  if (!(tmax > lo)) return false;
  *t0 = lo;
  *t1 = tmax;
  return true;
}

struct PathResult {
  float L0, L1, L2, beta;
  uint32_t n, kind;
};

// ---- spherical area lights (centre xyz, radius, radiance rgb), all outside the unit cube ----

__device__ __forceinline__ float dot3(float ax, float ay, float az, float bx, float by, float bz) {
  return (ax * bx + ay * by) + az * bz;
}

// 1 - cos(theta_max) of the cone a sphere of radius r subtends from squared distance d2, as
// sin^2 / (1 + cos) so that small cones keep their precision.
__device__ __forceinline__ float cone_one_minus(float r, float d2) {
  const float s2 = (r * r) / d2;
  return s2 / (1.0f + sqrtf(1.0f - s2));
}

// Nearer root of |o + t w - c|^2 = r^2 for an origin outside the sphere; false on a miss or a
// sphere behind the origin.
__device__ __forceinline__ bool sphere_hit(const float* sp, float ox, float oy, float oz, float wx,
                                           float wy, float wz, float* t) {
  const float cx = sp[0] - ox, cy = sp[1] - oy, cz = sp[2] - oz;
  const float b = dot3(wx, wy, wz, cx, cy, cz);
  const float c = dot3(cx, cy, cz, cx, cy, cz) - sp[3] * sp[3];
  const float disc = b * b - c;
  if (!(b > 0.0f) || !(disc >= 0.0f)) return false;
  *t = b - sqrtf(disc);
  return true;
}

// Radiance gathered by a continuation (o, w) that left the volume from a vertex: the nearest
// sphere light's radiance, with the phase sample's power-heuristic weight om^2 / (om^2 + 4)
// against cone sampling of that light (solid-angle pdfs 1/(4 pi) and 1/(2 pi om)) when next-
// event estimation is on, weight 1 for phase sampling alone.
__device__ __forceinline__ bool escape_light(const float* sph, int ns, uint32_t strategy, float ox,
                                             float oy, float oz, float wx, float wy, float wz,
                                             float* e0, float* e1, float* e2) {
  int best = -1;
  float tbest = __int_as_float(0x7f800000);
  for (int s = 0; s < ns; ++s) {
    float th;
    if (sphere_hit(sph + 7 * s, ox, oy, oz, wx, wy, wz, &th) && th < tbest) { tbest = th; best = s; }
  }
  if (best < 0) return false;
  const float* sp = sph + 7 * best;
  float wt = 1.0f;
  if (strategy == GSC_STRATEGY_NEE) {
    const float cx = sp[0] - ox, cy = sp[1] - oy, cz = sp[2] - oz;
    const float om = cone_one_minus(sp[3], dot3(cx, cy, cz, cx, cy, cz));
    wt = (om * om) / (om * om + 4.0f);
  }
  *e0 = sp[4] * wt; *e1 = sp[5] * wt; *e2 = sp[6] * wt;
  return true;
}

__device__ PathResult trace_path(const TraceDesc& D, const Vol& V, const float* lights,
                                 const float* sph, int px, int py, uint32_t sample) {
  PathResult res{0.0f, 0.0f, 0.0f, 1.0f, 0u, 0u};
  const DevCam& cam = D.cam;
  PathStream rng(D.seed, (uint32_t)py * (uint32_t)cam.full_w + (uint32_t)px, sample, D.frame);
  float d0 = ((float)px + 0.5f - cam.cx) / cam.fx;
  float d1 = ((float)py + 0.5f - cam.cy) / cam.fy;
  float d2 = 1.0f;
  const float nrm = sqrtf((d0 * d0 + d1 * d1) + d2 * d2);
  d0 = d0 / nrm; d1 = d1 / nrm; d2 = d2 / nrm;
  const float* R = cam.R;
  float wx = (R[0] * d0 + R[3] * d1) + R[6] * d2;
  float wy = (R[1] * d0 + R[4] * d1) + R[7] * d2;
  float wz = (R[2] * d0 + R[5] * d1) + R[8] * d2;
  float ox = -((R[0] * cam.t[0] + R[3] * cam.t[1]) + R[6] * cam.t[2]);
  float oy = -((R[1] * cam.t[0] + R[4] * cam.t[1]) + R[7] * cam.t[2]);
  float oz = -((R[2] * cam.t[0] + R[5] * cam.t[1]) + R[8] * cam.t[2]);
  float t0, t1;
  if (!box(ox, oy, oz, wx, wy, wz, &t0, &t1)) return res;
  const float sb = D.majorant;
  const int ns = D.n_spheres;
  // Next-event estimation only with that strategy: point lights and sphere lights sampled.
  const int nl = D.strategy == GSC_STRATEGY_NEE ? D.n_lights : 0;
  const int ne = D.strategy == GSC_STRATEGY_NEE ? ns : 0;
  float tr0 = 1.0f, tr1 = 1.0f, tr2 = 1.0f;
  float raw0 = 1.0f, raw1 = 1.0f, raw2 = 1.0f;
  float beta = 1.0f;
  float L0 = 0.0f, L1 = 0.0f, L2 = 0.0f;
  uint32_t n = 0u;
  uint32_t kind = GSC_KIND_ESCAPE0;
  for (;;) {
    float t = t0;
    bool collided = false;
    float x = 0.0f, y = 0.0f, z = 0.0f, dcol = 0.0f;
    for (uint32_t step = 0; step < kMaxSteps; ++step) {
      const float u = rng.uniform();
      t = t - glog(1.0f - u) / sb;
      if (t >= t1) break;
      x = ox + t * wx; y = oy + t * wy; z = oz + t * wz;
      const float u2 = rng.uniform();
      float dd;
      const float st = sigma_t(V, x, y, z, &dd);
      if (u2 < st / sb) { collided = true; dcol = dd; break; }
    }
    if (!collided) {
      // Leaving the volume; from a vertex (not the camera) the ray may reach an area light.
      float e0, e1, e2;
      if (n > 0u && escape_light(sph, ns, D.strategy, ox, oy, oz, wx, wy, wz, &e0, &e1, &e2)) {
        L0 = L0 + tr0 * e0; L1 = L1 + tr1 * e1; L2 = L2 + tr2 * e2;
      }
      kind = (n == 0u) ? GSC_KIND_ESCAPE0 : GSC_KIND_ESCAPE;
      break;
    }
    // The continuation sampled after the last allowed vertex collided again.
    if (n >= D.max_bounces) { kind = GSC_KIND_MAXDEPTH; break; }
    n += 1u;
    float ar, ag, ab, aa;
    transfer(V, dcol, &ar, &ag, &ab, &aa);
    raw0 = raw0 * ar; raw1 = raw1 * ag; raw2 = raw2 * ab;
    tr0 = tr0 * ar; tr1 = tr1 * ag; tr2 = tr2 * ab;
    for (int l = 0; l < nl; ++l) {
      const float* lp = lights + 6 * l;
      const float dl0 = lp[0] - x, dl1 = lp[1] - y, dl2 = lp[2] - z;
      const float dist2 = (dl0 * dl0 + dl1 * dl1) + dl2 * dl2;
      const float dist = sqrtf(dist2);
      const float l0 = dl0 / dist, l1 = dl1 / dist, l2 = dl2 / dist;
      float b0, b1;
      float texit;
      if (box(x, y, z, l0, l1, l2, &b0, &b1)) texit = fminf(dist, b1);
      else texit = 0.0f;
      float Tsh = 1.0f, ts = 0.0f;
      for (uint32_t step = 0; step < kMaxSteps; ++step) {
        const float u = rng.uniform();
        ts = ts - glog(1.0f - u) / sb;
        if (ts >= texit) break;
        float dd;
        const float st = sigma_t(V, x + ts * l0, y + ts * l1, z + ts * l2, &dd);
        Tsh = Tsh * (1.0f - st / sb);
      }
      const float g = (Tsh / dist2) * kInv4Pi;
      L0 = L0 + tr0 * (lp[3] * g);
      L1 = L1 + tr1 * (lp[4] * g);
      L2 = L2 + tr2 * (lp[5] * g);
    }
    // Sphere lights: one direction uniform in the subtended cone (1 - cos theta = u_a om,
    // phi = 2 pi u_b, around the axis by the Duff et al. 2017 orthonormal basis), its hit
    // point, blocked if another sphere is nearer, else ratio-tracked.  phase * Le * T / p_light
    // with the power-heuristic weight p_light^2 / (p_light^2 + p_phase^2) is
    // Le * T * 2 om / (om^2 + 4).
    for (int s = 0; s < ne; ++s) {
      const float* sp = sph + 7 * s;
      const float dl0 = sp[0] - x, dl1 = sp[1] - y, dl2 = sp[2] - z;
      const float d2 = dot3(dl0, dl1, dl2, dl0, dl1, dl2);
      const float d = sqrtf(d2);
      const float a0 = dl0 / d, a1 = dl1 / d, a2 = dl2 / d;
      const float om = cone_one_minus(sp[3], d2);
      const float ua = rng.uniform(), ub = rng.uniform();
      const float v = ua * om;
      const float ct = 1.0f - v;
      const float st = sqrtf(fmaxf(0.0f, v * (2.0f - v)));
      float sphi, cphi;
      gsincos(kTwoPi * ub, &sphi, &cphi);
      const float sg = copysignf(1.0f, a2);
      const float k = -1.0f / (sg + a2);
      const float m = (a0 * a1) * k;
      const float b10 = 1.0f + ((sg * a0) * a0) * k, b11 = sg * m, b12 = -(sg * a0);
      const float b20 = m, b21 = sg + (a1 * a1) * k, b22 = -a1;
      const float sc = st * cphi, ss = st * sphi;
      const float l0 = (sc * b10 + ss * b20) + ct * a0;
      const float l1 = (sc * b11 + ss * b21) + ct * a1;
      const float l2 = (sc * b12 + ss * b22) + ct * a2;
      const float bq = dot3(l0, l1, l2, dl0, dl1, dl2);
      const float th = bq - sqrtf(fmaxf(0.0f, bq * bq - (d2 - sp[3] * sp[3])));
      bool blocked = false;
      for (int mm = 0; mm < ns; ++mm) {
        float tm;
        if (mm != s && sphere_hit(sph + 7 * mm, x, y, z, l0, l1, l2, &tm) && tm < th) blocked = true;
      }
      if (blocked) continue;
      float b0, b1;
      const float texit = box(x, y, z, l0, l1, l2, &b0, &b1) ? fminf(th, b1) : 0.0f;
      float Tsh = 1.0f, ts = 0.0f;
      for (uint32_t step = 0; step < kMaxSteps; ++step) {
        const float u = rng.uniform();
        ts = ts - glog(1.0f - u) / sb;
        if (ts >= texit) break;
        float dd;
        const float stt = sigma_t(V, x + ts * l0, y + ts * l1, z + ts * l2, &dd);
        Tsh = Tsh * (1.0f - stt / sb);
      }
      const float g = Tsh * ((2.0f * om) / (om * om + 4.0f));
      L0 = L0 + tr0 * (sp[4] * g);
      L1 = L1 + tr1 * (sp[5] * g);
      L2 = L2 + tr2 * (sp[6] * g);
    }
    // After the last allowed vertex only a continuation reaching an area light can still add
    // radiance; without area lights the path ends here.
    const bool last = n >= D.max_bounces;
    if (last && ns == 0) { kind = GSC_KIND_MAXDEPTH; break; }
    if (!last && !D.C_inf) {
      const float lum = (0.2126f * raw0 + 0.7152f * raw1) + 0.0722f * raw2;
      const float Tr = fminf(fmaxf(D.C * lum, 0.0f), 1.0f);
      if (Tr < 0.9f) {
        const float q = rng.uniform();
        if (q < 1.0f - Tr) { kind = GSC_KIND_EARLY; break; }
        tr0 = tr0 / (Tr + D.eps);
        tr1 = tr1 / (Tr + D.eps);
        tr2 = tr2 / (Tr + D.eps);
        beta = beta * Tr;
      }
    }
    const float u1 = rng.uniform(), u2 = rng.uniform();
    const float cz = 1.0f - 2.0f * u1;
    const float r = sqrtf(fmaxf(0.0f, 1.0f - cz * cz));
    float sp, cp;
    gsincos(kTwoPi * u2, &sp, &cp);
    wx = r * cp; wy = r * sp; wz = cz;
    ox = x; oy = y; oz = z;
    float bb0, bb1;
    if (!box(ox, oy, oz, wx, wy, wz, &bb0, &bb1)) {
      float e0, e1, e2;
      if (escape_light(sph, ns, D.strategy, ox, oy, oz, wx, wy, wz, &e0, &e1, &e2)) {
        L0 = L0 + tr0 * e0; L1 = L1 + tr1 * e1; L2 = L2 + tr2 * e2;
      }
      kind = GSC_KIND_ESCAPE;
      break;
    }
    t0 = 0.0f;
    t1 = bb1;
  }
  res.L0 = L0; res.L1 = L1; res.L2 = L2;
  res.beta = beta;
  res.n = n;
  res.kind = kind;
  return res;
}

// Each request's pixels start at a multiple of kTraceBlock in the launch index space, so a
// workgroup never straddles two requests: the request index is workgroup-uniform (scalar
// descriptor loads) and the transfer function and lights are staged once in LDS.
__global__ void __launch_bounds__(kTraceBlock) trace_kernel(const TraceDesc* __restrict__ descs,
                                                            const int64_t* __restrict__ req_pstart,
                                                            int R, unsigned long long* path_vertices) {
  __shared__ float s_tf[kMaxTf * 4];
  __shared__ float s_lights[kMaxLights * 6];
  __shared__ float s_spheres[kMaxLights * 7];
  const int64_t block0 = (int64_t)blockIdx.x * kTraceBlock;
  const int r = find_segment(req_pstart, R, block0);
  const TraceDesc& D = descs[r];
  for (int i = threadIdx.x; i < 4 * D.P; i += kTraceBlock) s_tf[i] = D.tf[i];
  for (int i = threadIdx.x; i < 6 * D.n_lights; i += kTraceBlock) s_lights[i] = D.lights[i];
  for (int i = threadIdx.x; i < 7 * D.n_spheres; i += kTraceBlock) s_spheres[i] = D.spheres[i];
  __syncthreads();
  const int W = D.cam.w, H = D.cam.h;
  const int64_t plane = (int64_t)W * H;
  const int64_t lp = block0 + threadIdx.x - D.pix_off;
  uint64_t verts = 0;
  if (lp < plane) {
    const Vol V{D.density, D.cells, D.nx, D.ny, D.nz, D.dmax, s_tf, D.P};
    const int lx = (int)(lp % W), ly = (int)(lp / W);
    const int px = D.cam.x0 + lx, py = D.cam.y0 + ly;
    const uint32_t K = D.K;
    if (D.spp == 1u) {
      const PathResult pr = trace_path(D, V, s_lights, s_spheres, px, py, 0u);
      verts = pr.n;
      const uint32_t lvl = pr.n ? (min(pr.n, K) - 1u) : 0xFFFFFFFFu;
      for (uint32_t l = 0; l < K; ++l) {
        float* o = D.targets + 3 * (l * plane + lp);
        const bool mine = (l == lvl);
        o[0] = mine ? pr.L0 : 0.0f;
        o[1] = mine ? pr.L1 : 0.0f;
        o[2] = mine ? pr.L2 : 0.0f;
      }
      if (D.records) {
        uint32_t* rec = (uint32_t*)D.records + 5 * lp;
        rec[0] = __float_as_uint(pr.L0);
        rec[1] = __float_as_uint(pr.L1);
        rec[2] = __float_as_uint(pr.L2);
        rec[3] = __float_as_uint(pr.beta);
        rec[4] = pr.n | (pr.kind << 16);
      }
    } else {
      for (uint32_t l = 0; l < K; ++l) {
        float* o = D.targets + 3 * (l * plane + lp);
        o[0] = 0.0f; o[1] = 0.0f; o[2] = 0.0f;
      }
      for (uint32_t smp = 0; smp < D.spp; ++smp) {
        const PathResult pr = trace_path(D, V, s_lights, s_spheres, px, py, smp);
        verts += pr.n;
        if (D.records) {
          uint32_t* rec = (uint32_t*)D.records + 5 * ((int64_t)smp * plane + lp);
          rec[0] = __float_as_uint(pr.L0);
          rec[1] = __float_as_uint(pr.L1);
          rec[2] = __float_as_uint(pr.L2);
          rec[3] = __float_as_uint(pr.beta);
          rec[4] = pr.n | (pr.kind << 16);
        }
        if (pr.n) {
          float* o = D.targets + 3 * ((min(pr.n, K) - 1u) * plane + lp);
          o[0] = o[0] + pr.L0;
          o[1] = o[1] + pr.L1;
          o[2] = o[2] + pr.L2;
        }
      }
      const float fs = (float)D.spp;
      for (uint32_t l = 0; l < K; ++l) {
        float* o = D.targets + 3 * (l * plane + lp);
        o[0] = o[0] / fs; o[1] = o[1] / fs; o[2] = o[2] / fs;
      }
    }
  }
  if (path_vertices) {
    // Wave-level pre-reduction before the single 64-bit atomic.
    unsigned long long v = verts;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (__lane_id() == 0 && v) atomicAdd(path_vertices, v);
  }
}

// Cache initialisation points (Method: "Cache Initialization"): one lane per point; random rays
// are tracked through the volume by delta tracking until their first real interaction, whose
// position and albedo (the transfer function's colour at that density) are recorded; a ray that
// leaves the volume is replaced by a fresh one.  Attempt a of point i draws from the Philox
// stream with counter (i, a, 0x494E4954, block): a point p uniform in the cube (3 draws), a
// direction w uniform on the sphere (2 draws, as the phase function), the ray starts at
// p - 2 w, outside the cube, and passes through p.  tries[i] = attempts used, 0 if none found.
__global__ void __launch_bounds__(kTraceBlock) init_points_kernel(const TraceDesc* __restrict__ D,
                                                                  int64_t n, int max_attempts,
                                                                  float* __restrict__ pos,
                                                                  float* __restrict__ albedo,
                                                                  int32_t* __restrict__ tries) {
  __shared__ float s_tf[kMaxTf * 4];
  for (int k = threadIdx.x; k < 4 * D->P; k += kTraceBlock) s_tf[k] = D->tf[k];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kTraceBlock + threadIdx.x;
  if (i >= n) return;
  const Vol V{D->density, D->cells, D->nx, D->ny, D->nz, D->dmax, s_tf, D->P};
  const float sb = D->majorant;
  int32_t used = 0;
  for (int a = 0; a < max_attempts; ++a) {
    PathStream rng(D->seed, (uint32_t)i, (uint32_t)a, 0x494E4954u);
    const float p0 = rng.uniform(), p1 = rng.uniform(), p2 = rng.uniform();
    const float u3 = rng.uniform(), u4 = rng.uniform();
    const float cz = 1.0f - 2.0f * u3;
    const float r = sqrtf(fmaxf(0.0f, 1.0f - cz * cz));
    float sp, cp;
    gsincos(kTwoPi * u4, &sp, &cp);
    const float wx = r * cp, wy = r * sp, wz = cz;
    const float ox = p0 - 2.0f * wx, oy = p1 - 2.0f * wy, oz = p2 - 2.0f * wz;
    float t0, t1;
    if (!box(ox, oy, oz, wx, wy, wz, &t0, &t1)) continue;
    float t = t0;
    bool hit = false;
    for (uint32_t step = 0; step < kMaxSteps; ++step) {
      const float u = rng.uniform();
      t = t - glog(1.0f - u) / sb;
      if (t >= t1) break;
      const float x = ox + t * wx, y = oy + t * wy, z = oz + t * wz;
      const float u2 = rng.uniform();
      float dd;
      const float st = sigma_t(V, x, y, z, &dd);
      if (u2 < st / sb) {
        float ar, ag, ab, aa;
        transfer(V, dd, &ar, &ag, &ab, &aa);
        pos[3 * i + 0] = x; pos[3 * i + 1] = y; pos[3 * i + 2] = z;
        albedo[3 * i + 0] = ar; albedo[3 * i + 1] = ag; albedo[3 * i + 2] = ab;
        hit = true;
        break;
      }
    }
    if (hit) { used = a + 1; break; }
  }
  tries[i] = used;
}

// One thread per cell (x0, y0, z0) in [-1, n-1]^3: the clamped corners in the order
// (x0,y0,z0) (x1,y0,z0) (x0,y1,z0) (x1,y1,z0) (x0,y0,z1) (x1,y0,z1) (x0,y1,z1) (x1,y1,z1).
__global__ void __launch_bounds__(256) build_cells_kernel(const float* __restrict__ d, int nx, int ny,
                                                          int nz, float4* __restrict__ cells) {
  const int64_t n = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int cx = (int)(i % (nx + 1)) - 1;
  const int cy = (int)((i / (nx + 1)) % (ny + 1)) - 1;
  const int cz = (int)(i / ((int64_t)(nx + 1) * (ny + 1))) - 1;
  const int x0 = max(cx, 0), x1 = min(cx + 1, nx - 1);
  const int y0 = max(cy, 0), y1 = min(cy + 1, ny - 1);
  const int z0 = max(cz, 0), z1 = min(cz + 1, nz - 1);
  const int64_t sy = nx, sz = (int64_t)nx * ny;
  const float* p00 = d + z0 * sz + y0 * sy;
  const float* p10 = d + z0 * sz + y1 * sy;
  const float* p01 = d + z1 * sz + y0 * sy;
  const float* p11 = d + z1 * sz + y1 * sy;
  cells[2 * i] = make_float4(p00[x0], p00[x1], p10[x0], p10[x1]);
  cells[2 * i + 1] = make_float4(p01[x0], p01[x1], p11[x0], p11[x1]);
}

}  // namespace

int64_t trace_align(int64_t pixels) { return (pixels + kTraceBlock - 1) / kTraceBlock * kTraceBlock; }

// total_launch: the sum over requests of trace_align(w h); each request's pix_off and
// req_pstart entry are its aligned start in that space.
hipError_t launch_trace(hipStream_t st, const TraceDesc* descs, const int64_t* req_pstart, int R,
                        int64_t total_launch, unsigned long long* path_vertices) {
  if (total_launch == 0) return hipSuccess;
  hipLaunchKernelGGL(trace_kernel, dim3((unsigned)(total_launch / kTraceBlock)), dim3(kTraceBlock), 0,
                     st, descs, req_pstart, R, path_vertices);
  return hipGetLastError();
}

size_t cells_bytes(int nx, int ny, int nz) {
  return 32 * (size_t)(nx + 1) * (size_t)(ny + 1) * (size_t)(nz + 1);
}

hipError_t launch_build_cells(hipStream_t st, const float* density, int nx, int ny, int nz,
                              float4* cells) {
  const int64_t n = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  hipLaunchKernelGGL(build_cells_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, density,
                     nx, ny, nz, cells);
  return hipGetLastError();
}

hipError_t launch_init_points(hipStream_t st, const TraceDesc* desc, int64_t n, int max_attempts,
                              float* pos, float* albedo, int32_t* tries) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(init_points_kernel, dim3((unsigned)((n + kTraceBlock - 1) / kTraceBlock)),
                     dim3(kTraceBlock), 0, st, desc, n, max_attempts, pos, albedo, tries);
  return hipGetLastError();
}

}  // namespace gsc
