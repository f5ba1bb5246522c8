// k_project.hip -- projection of the Gaussians of every segment to screen-space conics, and the
// adjoint of that projection (3D Gaussian splatting, the rasteriser GSCache adapts as its
// cache; Method: "A Path Space Radiance Cache").
#include "gsc_dev.h"

namespace gsc {

namespace {

constexpr uint64_t kEmptyRect = 0x0000000100000001ull;   // tx0 = 1 > tx1 = 0: covers nothing

// Saturation core of a projected Gaussian, for cutting tile lists where they can no longer reach
// a pixel: the tiles all of whose in-window pixels lie inside the Gaussian's integer window and
// inside the rectangle |u - i| <= hx, |v - j| <= hy inscribed in the ellipse
// Q(u - i, v - j) <= kCoreQ.  There the splat's alpha = min(0.99, o exp(-Q / 2)) is at least
// o exp(-kCoreQ / 2) > o / 2 (kCoreQ = 1.3 < 2 ln 2 leaves room for rounding and the hardware
// exp), so every such pixel that has not terminated multiplies its transmittance by at most
// 1 - o / 2.  The weight is -ln(1 - o / 2) in 2^-16 units, rounded down.  No core when
// o / 2 < 1/255 (such a pair may be skipped) or when the conic is too close to singular for its
// quadratic form to keep its sign under rounding.  Packed in one word: tile columns cx0, cx1 and
// rows cy0, cy1 in 11-bit fields (bits 0, 11, 22, 33), the weight (< 2^16) in bits 48..63; a
// Gaussian without a core has weight 0.
constexpr float kCoreQ = 1.3f;

__device__ __forceinline__ uint64_t saturation_core(const Projected& P, const DevCam& cam,
                                                    int tsx, int tsy) {
  if (!P.tiles || !(P.o >= (2.0f / 255.0f) * 1.01f)) return 0ull;
  const float rho = fabsf(P.B) / sqrtf(P.A * P.Cc);
  if (!(rho < 0.999f)) return 0ull;
  // Corner value A hx^2 + 2 |B| hx hy + C hy^2 = kCoreQ for hx = sqrt(kCoreQ / (2 A (1 + rho))).
  const float hx = sqrtf(kCoreQ / ((2.0f * P.A) * (1.0f + rho)));
  const float hy = sqrtf(kCoreQ / ((2.0f * P.Cc) * (1.0f + rho)));
  const int i0 = max(P.px0, (int)ceilf(P.u - hx)), i1 = min(P.px1, (int)floorf(P.u + hx));
  const int j0 = max(P.py0, (int)ceilf(P.v - hy)), j1 = min(P.py1, (int)floorf(P.v + hy));
  if (i0 > i1 || j0 > j1) return 0ull;
  // Window-local tiles whose pixels (clipped to the render window) lie in [i0, i1] x [j0, j1].
  const int tw = 1 << tsx, th = 1 << tsy;        // tiles are tw x th pixels
  const int TX = (cam.w + tw - 1) >> tsx, TY = (cam.h + th - 1) >> tsy;
  const int lx0 = i0 - cam.x0, lx1 = i1 - cam.x0, ly0 = j0 - cam.y0, ly1 = j1 - cam.y0;
  const int cx0 = (lx0 + tw - 1) >> tsx, cy0 = (ly0 + th - 1) >> tsy;
  const int cx1 = (lx1 >= cam.w - 1) ? TX - 1 : ((lx1 + 1) >> tsx) - 1;
  const int cy1 = (ly1 >= cam.h - 1) ? TY - 1 : ((ly1 + 1) >> tsy) - 1;
  if (cx0 > cx1 || cy0 > cy1) return 0ull;
  const uint64_t w = (uint64_t)(-logf(1.0f - 0.5f * P.o) * (65536.0f * 0.999f));
  return (uint64_t)cx0 | ((uint64_t)cx1 << 11) | ((uint64_t)cy0 << 22) | ((uint64_t)cy1 << 33) |
         (w << 48);
}

__global__ void __launch_bounds__(256) project_kernel(const Seg* __restrict__ segs,
                                                      const int64_t* __restrict__ seg_gstart, int S,
                                                      const DevCam* __restrict__ cams, int64_t G,
                                                      SplatRec* __restrict__ rec,
                                                      uint32_t* __restrict__ depth_key,
                                                      uint64_t* __restrict__ rect,
                                                      uint32_t* __restrict__ tiles,
                                                      uint32_t* __restrict__ ids,
                                                      uint64_t* __restrict__ core) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G) return;
  const int s = find_segment(seg_gstart, S, i);
  const Seg sg = segs[s];
  const int64_t lid = i - sg.g_off;
  const DevCam cam = cams[sg.cam];
  const Projected P = project_one(sg.pos + 3 * lid, sg.rot + 4 * lid, sg.ls + 3 * lid,
                                  sg.logit[lid], cam, sg.tsx, sg.tsy);
  const float* c = sg.rgb + 3 * lid;
  SplatRec r;
  r.q0 = make_float4(P.u, P.v, P.A, P.B);
  r.q1 = make_float4(P.Cc, P.o, c[0], c[1]);
  const uint32_t wx = (uint32_t)P.px0 | ((uint32_t)P.px1 << 16);
  const uint32_t wy = (uint32_t)P.py0 | ((uint32_t)P.py1 << 16);
  r.q2 = make_float4(c[2], __uint_as_float(wx), __uint_as_float(wy), __uint_as_float((uint32_t)lid));
  rec[i] = r;
  depth_key[i] = P.tiles ? __float_as_uint(P.z) : 0xFFFFFFFFu;
  rect[i] = P.tiles ? ((uint64_t)P.tx0 | ((uint64_t)P.tx1 << 16) | ((uint64_t)P.ty0 << 32) |
                       ((uint64_t)P.ty1 << 48))
                    : kEmptyRect;
  tiles[i] = P.tiles;
  ids[i] = (uint32_t)lid;
  if (core) core[i] = saturation_core(P, cam, sg.tsx, sg.tsy);
}

// Adjoint of the projection.  grad2d holds a 64-byte record per Gaussian, [G][kGrad2dStride]:
// du, dv, dA, dB, dCc, do, dr, dg, db (accumulated by the splat backward).  Writes (overwrites)
// the gradients of the 14 parameters.
// The forward quantities are recomputed in fp32 exactly as the projection computes them.
// Chain rule of one Gaussian (level-local index lid of segment sg) from the screen-space
// gradients (u, v, conic A, B, C, opacity o) to its mean, quaternion, log-scales and opacity
// logit.  Reads the Gaussian's parameters; writes gp[3], gq[4], gs[3] and *gl.
__device__ __forceinline__ void project_grads(const Seg& sg, const DevCam& cam, int64_t lid,
                                              float gu, float gv, float gA, float gB, float gC,
                                              float go, float* gp, float* gq, float* gs,
                                              float* gl) {
  const float* pos = sg.pos + 3 * lid;
  const float* rot = sg.rot + 4 * lid;
  const float* ls = sg.ls + 3 * lid;
  const float logit = sg.logit[lid];
  const Projected P = project_one(pos, rot, ls, logit, cam, sg.tsx, sg.tsy);
  // Opacity: o = sigmoid(logit).
  *gl = go * (P.o * (1.0f - P.o));
  if (P.tiles == 0u) {
    gp[0] = gp[1] = gp[2] = 0.0f;
    gq[0] = gq[1] = gq[2] = gq[3] = 0.0f;
    gs[0] = gs[1] = gs[2] = 0.0f;
    return;
  }
  const float* Rc = cam.R;
  const float p0 = pos[0], p1 = pos[1], p2 = pos[2];
  const float x = ((Rc[0] * p0 + Rc[1] * p1) + Rc[2] * p2) + cam.t[0];
  const float y = ((Rc[3] * p0 + Rc[4] * p1) + Rc[5] * p2) + cam.t[1];
  const float z = ((Rc[6] * p0 + Rc[7] * p1) + Rc[8] * p2) + cam.t[2];
  const float qn = sqrtf(((rot[0] * rot[0] + rot[1] * rot[1]) + rot[2] * rot[2]) + rot[3] * rot[3]);
  const float qw = rot[0] / qn, qx = rot[1] / qn, qy = rot[2] / qn, qz = rot[3] / qn;
  const float s3[3] = {gexp(ls[0]), gexp(ls[1]), gexp(ls[2])};
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
  float M[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) M[3 * a + b] = Rq[3 * a + b] * s3[b];
  float S3[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      S3[3 * a + b] = (M[3 * a] * M[3 * b] + M[3 * a + 1] * M[3 * b + 1]) + M[3 * a + 2] * M[3 * b + 2];
  const float iz = 1.0f / z;
  const float limx = 1.3f * ((float)cam.full_w / (2.0f * cam.fx));
  const float limy = 1.3f * ((float)cam.full_h / (2.0f * cam.fy));
  const float xz = x * iz, yz = y * iz;
  const bool clx = (xz < -limx) || (xz > limx);
  const bool cly = (yz < -limy) || (yz > limy);
  const float txz = fminf(fmaxf(xz, -limx), limx);
  const float tyz = fminf(fmaxf(yz, -limy), limy);
  const float iz2 = iz * iz;
  const float J00 = cam.fx * iz, J02 = -(cam.fx * (txz * z)) * iz2;
  const float J11 = cam.fy * iz, J12 = -(cam.fy * (tyz * z)) * iz2;
  float T[6];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    T[b] = J00 * Rc[b] + J02 * Rc[6 + b];
    T[3 + b] = J11 * Rc[3 + b] + J12 * Rc[6 + b];
  }
  // Sigma2' = T S3 T^T + 0.3 I = [[a, b], [b, c]].
  float U[6];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      U[3 * a + b] = (T[3 * a] * S3[b] + T[3 * a + 1] * S3[3 + b]) + T[3 * a + 2] * S3[6 + b];
  const float a2 = ((U[0] * T[0] + U[1] * T[1]) + U[2] * T[2]) + 0.3f;
  const float b2 = (U[0] * T[3] + U[1] * T[4]) + U[2] * T[5];
  const float c2 = ((U[3] * T[3] + U[4] * T[4]) + U[5] * T[5]) + 0.3f;
  const float det = a2 * c2 - b2 * b2;
  const float id2 = 1.0f / (det * det);
  // conic (A, B, C) = (c, -b, a) / det  ->  d/d(a, b, c).
  const float da = (-c2 * c2 * gA + b2 * c2 * gB - b2 * b2 * gC) * id2;
  const float db = (2.0f * b2 * c2 * gA - (a2 * c2 + b2 * b2) * gB + 2.0f * a2 * b2 * gC) * id2;
  const float dc = (-b2 * b2 * gA + a2 * b2 * gB - a2 * a2 * gC) * id2;
  // Symmetric gradient of Sigma2: G2 = [[da, db/2], [db/2, dc]].
  const float G00 = da, G01 = 0.5f * db, G11 = dc;
  // dS3 = T^T G2 T ; dT = 2 G2 T S3.
  float GT[6];   // G2 T  (2x3)
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    GT[b] = G00 * T[b] + G01 * T[3 + b];
    GT[3 + b] = G01 * T[b] + G11 * T[3 + b];
  }
  float dS[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) dS[3 * a + b] = T[a] * GT[b] + T[3 + a] * GT[3 + b];
  float dT[6];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      dT[3 * a + b] = 2.0f * ((GT[3 * a] * S3[b] + GT[3 * a + 1] * S3[3 + b]) + GT[3 * a + 2] * S3[6 + b]);
  // dJ = dT Rc^T  (only the four nonzero entries of J matter).
  const float dJ00 = (dT[0] * Rc[0] + dT[1] * Rc[1]) + dT[2] * Rc[2];
  const float dJ02 = (dT[0] * Rc[6] + dT[1] * Rc[7]) + dT[2] * Rc[8];
  const float dJ11 = (dT[3] * Rc[3] + dT[4] * Rc[4]) + dT[5] * Rc[5];
  const float dJ12 = (dT[3] * Rc[6] + dT[4] * Rc[7]) + dT[5] * Rc[8];
  // Through J(x, z): J00 = fx/z, J11 = fy/z, J02 = -fx txz / z with txz = clamp(x/z).
  float dx = 0.0f, dy = 0.0f, dz = 0.0f;
  dz += -cam.fx * iz2 * dJ00 - cam.fy * iz2 * dJ11;
  if (!clx) { dx += -cam.fx * iz2 * dJ02; dz += 2.0f * cam.fx * x * iz2 * iz * dJ02; }
  else { dz += cam.fx * txz * iz2 * dJ02; }
  if (!cly) { dy += -cam.fy * iz2 * dJ12; dz += 2.0f * cam.fy * y * iz2 * iz * dJ12; }
  else { dz += cam.fy * tyz * iz2 * dJ12; }
  // Through the screen mean u = fx x/z + cx - 1/2, v = fy y/z + cy - 1/2.
  dx += cam.fx * iz * gu;
  dy += cam.fy * iz * gv;
  dz += -cam.fx * x * iz2 * gu - cam.fy * y * iz2 * gv;
  // x_c = Rc pos + t.
  gp[0] = (Rc[0] * dx + Rc[3] * dy) + Rc[6] * dz;
  gp[1] = (Rc[1] * dx + Rc[4] * dy) + Rc[7] * dz;
  gp[2] = (Rc[2] * dx + Rc[5] * dy) + Rc[8] * dz;
  // Sigma3 = M M^T: dM = 2 dS M ; M = Rq diag(s).
  float dM[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      dM[3 * a + b] = 2.0f * ((dS[3 * a] * M[b] + dS[3 * a + 1] * M[3 + b]) + dS[3 * a + 2] * M[6 + b]);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const float dsb = (dM[b] * Rq[b] + dM[3 + b] * Rq[3 + b]) + dM[6 + b] * Rq[6 + b];
    gs[b] = dsb * s3[b];
  }
  float dR[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) dR[3 * a + b] = dM[3 * a + b] * s3[b];
  // R(q) -> unit quaternion (w, x, y, z).
  const float dqw = 2.0f * (-qz * dR[1] + qy * dR[2] + qz * dR[3] - qx * dR[5] - qy * dR[6] + qx * dR[7]);
  const float dqx = 2.0f * (qy * dR[1] + qz * dR[2] + qy * dR[3] - 2.0f * qx * dR[4] - qw * dR[5] +
                            qz * dR[6] + qw * dR[7] - 2.0f * qx * dR[8]);
  const float dqy = 2.0f * (-2.0f * qy * dR[0] + qx * dR[1] + qw * dR[2] + qx * dR[3] + qz * dR[5] -
                            qw * dR[6] + qz * dR[7] - 2.0f * qy * dR[8]);
  const float dqz = 2.0f * (-2.0f * qz * dR[0] - qw * dR[1] + qx * dR[2] + qw * dR[3] -
                            2.0f * qz * dR[4] + qy * dR[5] + qx * dR[6] + qy * dR[7]);
  // Normalisation q^ = q / |q|: dq = (dq^ - q^ (q^ . dq^)) / |q|.
  const float dot = ((qw * dqw + qx * dqx) + qy * dqy) + qz * dqz;
  const float iq = 1.0f / qn;
  gq[0] = (dqw - qw * dot) * iq;
  gq[1] = (dqx - qx * dot) * iq;
  gq[2] = (dqy - qy * dot) * iq;
  gq[3] = (dqz - qz * dot) * iq;
}

// The nine screen-space gradients of Gaussian i (three aligned 16-byte loads of its record).
__device__ __forceinline__ void load_grad2d(const float* __restrict__ grad2d, int64_t i, float g[12]) {
  const float4* r = reinterpret_cast<const float4*>(grad2d + i * kGrad2dStride);
  const float4 a = r[0], b = r[1], c = r[2];
  g[0] = a.x; g[1] = a.y; g[2] = a.z; g[3] = a.w;
  g[4] = b.x; g[5] = b.y; g[6] = b.z; g[7] = b.w;
  g[8] = c.x; g[9] = c.y; g[10] = c.z; g[11] = c.w;
}

__global__ void __launch_bounds__(256) project_backward_kernel(
    const Seg* __restrict__ segs, const int64_t* __restrict__ seg_gstart, int S,
    const DevCam* __restrict__ cams, int64_t G, const float* __restrict__ grad2d,
    float* __restrict__ grads14) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G) return;
  const int s = find_segment(seg_gstart, S, i);
  const Seg sg = segs[s];
  const int64_t lid = i - sg.g_off;
  // Gradient layout per segment: [pos 3n][rot 4n][log_scale 3n][rgb 3n][opacity_logit n].
  float* base = grads14 + 14 * sg.g_off;
  const int64_t nn = sg.n;
  float* gc = base + 10 * nn + 3 * lid;
  float g[12];
  load_grad2d(grad2d, i, g);
  gc[0] = g[6];
  gc[1] = g[7];
  gc[2] = g[8];
  project_grads(sg, cams[sg.cam], lid, g[0], g[1], g[2], g[3], g[4], g[5], base + 3 * lid,
                base + 3 * nn + 4 * lid, base + 7 * nn + 3 * lid, base + 13 * nn + lid);
}

// The chain rule and the AdamW step in one pass.  Each thread takes the chain rule of one
// Gaussian; its 14 gradients go to LDS, and when the workgroup's 256 Gaussians lie in one
// segment (all but the few workgroups that straddle a boundary) the AdamW updates then run
// over each parameter group's contiguous range, so every parameter, moment and gradient access
// is coalesced.  A straddling workgroup updates each Gaussian from its own thread.
constexpr int kGradWidth[5] = {3, 4, 3, 3, 1};
constexpr int kGradFirst[5] = {0, 3, 7, 10, 13};

__global__ void __launch_bounds__(256) project_backward_adam_kernel(
    const Seg* __restrict__ segs, const int64_t* __restrict__ seg_gstart, int S,
    const DevCam* __restrict__ cams, int64_t G, const float* __restrict__ grad2d,
    const AdamGroup* __restrict__ groups) {
  __shared__ float gsh[14][256];
  const int tid = threadIdx.x;
  const int64_t first = (int64_t)blockIdx.x * 256;
  const int64_t i = first + tid;
  const int count = (int)((G - first) < 256 ? (G - first) : 256);
  const int s_first = find_segment(seg_gstart, S, first);
  const int s_last = find_segment(seg_gstart, S, first + count - 1);
  float gr14[14];
  int s = s_first;
  bool live = false;
  if (i < G) {
    s = find_segment(seg_gstart, S, i);
    const AdamGroup& g0 = groups[5 * s];
    live = g0.p != nullptr && !(g0.guard && !isfinite(*g0.guard));
    if (live) {
      const Seg sg = segs[s];
      const int64_t lid = i - sg.g_off;
      float g[12];
      load_grad2d(grad2d, i, g);
      project_grads(sg, cams[sg.cam], lid, g[0], g[1], g[2], g[3], g[4], g[5], gr14, gr14 + 3,
                    gr14 + 7, gr14 + 13);
      gr14[10] = g[6];
      gr14[11] = g[7];
      gr14[12] = g[8];
    }
  }
  if (s_first != s_last) {                 // straddles a segment boundary: per-thread updates
    if (!live) return;
    const Seg sg = segs[s];
    const int64_t lid = i - sg.g_off;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const AdamGroup& gk = groups[5 * s + k];
#pragma unroll
      for (int c = 0; c < kGradWidth[k]; ++c)
        adamw_element(gk.p, gk.m, gk.v, kGradWidth[k] * lid + c, gr14[kGradFirst[k] + c], gk);
    }
    return;
  }
  // One segment: liveness is uniform over the workgroup.
  const AdamGroup& g0 = groups[5 * s_first];
  if (g0.p == nullptr || (g0.guard && !isfinite(*g0.guard))) return;
#pragma unroll
  for (int k = 0; k < 14; ++k) gsh[k][tid] = gr14[k];
  __syncthreads();
  const int64_t lid0 = first - segs[s_first].g_off;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const AdamGroup& gk = groups[5 * s_first + k];
    const int w = kGradWidth[k];
    for (int e = tid; e < w * count; e += 256)
      adamw_element(gk.p, gk.m, gk.v, w * lid0 + e, gsh[kGradFirst[k] + e % w][e / w], gk);
  }
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_project(hipStream_t st, const Seg* segs, const int64_t* seg_gstart, int S,
                          const DevCam* cams, int64_t G, SplatRec* rec, uint32_t* depth_key,
                          uint64_t* rect, uint32_t* tiles, uint32_t* ids, uint64_t* core) {
  if (G == 0) return hipSuccess;
  hipLaunchKernelGGL(project_kernel, dim3(blocks_for(G, 256)), dim3(256), 0, st, segs, seg_gstart,
                     S, cams, G, rec, depth_key, rect, tiles, ids, core);
  return hipGetLastError();
}

hipError_t launch_project_backward(hipStream_t st, const Seg* segs, const int64_t* seg_gstart, int S,
                                   const DevCam* cams, int64_t G, const float* grad2d,
                                   float* grads14) {
  if (G == 0) return hipSuccess;
  hipLaunchKernelGGL(project_backward_kernel, dim3(blocks_for(G, 256)), dim3(256), 0, st, segs,
                     seg_gstart, S, cams, G, grad2d, grads14);
  return hipGetLastError();
}

hipError_t launch_project_backward_adam(hipStream_t st, const Seg* segs, const int64_t* seg_gstart,
                                        int S, const DevCam* cams, int64_t G, const float* grad2d,
                                        const AdamGroup* groups) {
  if (G == 0) return hipSuccess;
  hipLaunchKernelGGL(project_backward_adam_kernel, dim3(blocks_for(G, 256)), dim3(256), 0, st, segs,
                     seg_gstart, S, cams, G, grad2d, groups);
  return hipGetLastError();
}

hipError_t launch_fill_u32(hipStream_t st, uint32_t* p, uint32_t value, int64_t count) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, st, p, value,
                     count);
  return hipGetLastError();
}

}  // namespace gsc
