// Shading consumers of the field (Sec. III-C; Sec. IV-F, Table VI): the primary G-buffer from
// the exact scene, the secondary rays a renderer sends (one shadow ray toward a point light,
// K ambient-occlusion rays over the normal's hemisphere), and the per-pixel shadow and AO
// maps from the answers.  Between the second and third step the caller queries the field
// (either field, any precision) or, for the reference maps, the exact ray cast.
#include <math.h>

#include <cmath>

#include "ddf_internal.h"
#include "ddf_train.h"

namespace ddf {
namespace {

constexpr int kShadeThreads = 256;
constexpr int kPrimFloats = 16;    // center, 1/axes, R^T row-major, pad
constexpr int kPrimChunk = 256;    // primitives staged in LDS per pass

// First root t > 0 of the ray x + t d against primitive q (its unit-sphere frame: the
// quadratic |l + t e|^2 = 1 with l = R^T (x - c) / a, e = R^T d / a), or +inf.
__device__ __forceinline__ float prim_hit(const float* q, float x0, float x1, float x2, float d0, float d1,
                                          float d2) {
  const float r0 = x0 - q[0], r1 = x1 - q[1], r2 = x2 - q[2];
  const float l0 = (q[6] * r0 + q[7] * r1 + q[8] * r2) * q[3];
  const float l1 = (q[9] * r0 + q[10] * r1 + q[11] * r2) * q[4];
  const float l2 = (q[12] * r0 + q[13] * r1 + q[14] * r2) * q[5];
  const float e0 = (q[6] * d0 + q[7] * d1 + q[8] * d2) * q[3];
  const float e1 = (q[9] * d0 + q[10] * d1 + q[11] * d2) * q[4];
  const float e2 = (q[12] * d0 + q[13] * d1 + q[14] * d2) * q[5];
  const float A = e0 * e0 + e1 * e1 + e2 * e2;
  const float B = l0 * e0 + l1 * e1 + l2 * e2;
  const float C = l0 * l0 + l1 * l1 + l2 * l2 - 1.f;
  const float disc = B * B - A * C;
  if (!(disc >= 0.f)) return __builtin_inff();
  const float k = -(B + copysignf(sqrtf(disc), B));   // the numerically stable root pair
  const float ra = k / A;
  const float rb = k != 0.f ? C / k : -B / A;
  const float lo = fminf(ra, rb), hi = fmaxf(ra, rb);
  return lo > 0.f ? lo : (hi > 0.f ? hi : __builtin_inff());
}

struct CamArgs {
  float eye[3], f[3], r[3], u[3];   // position and orthonormal frame (view, right, up)
  float tx, ty;                     // tan(fov_y / 2) W / H and tan(fov_y / 2)
  int W, H;
};

// One pixel per thread: the camera ray, the nearest primitive (all primitives, staged through
// LDS), the hit point and the outward normal R (q / a) of the primitive hit.
__global__ __launch_bounds__(kShadeThreads) void gbuffer_kernel(CamArgs c, const float* __restrict__ prims,
                                                                int n_prims, float* __restrict__ gbuf,
                                                                uint8_t* __restrict__ hit) {
  __shared__ float sp[kPrimChunk * kPrimFloats];
  const int64_t P = (int64_t)c.W * c.H;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int px = (int)(i % c.W), py = (int)(i / c.W);
  const float sx = (2.f * (px + 0.5f) / c.W - 1.f) * c.tx;
  const float sy = (1.f - 2.f * (py + 0.5f) / c.H) * c.ty;
  float d0 = c.f[0] + sx * c.r[0] + sy * c.u[0];
  float d1 = c.f[1] + sx * c.r[1] + sy * c.u[1];
  float d2 = c.f[2] + sx * c.r[2] + sy * c.u[2];
  const float inv = 1.f / sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
  d0 *= inv; d1 *= inv; d2 *= inv;
  float best = __builtin_inff();
  int bp = -1;
  for (int base = 0; base < n_prims; base += kPrimChunk) {
    const int cnt = min(kPrimChunk, n_prims - base);
    __syncthreads();
    for (int j = threadIdx.x; j < cnt * kPrimFloats; j += blockDim.x) sp[j] = prims[(int64_t)base * kPrimFloats + j];
    __syncthreads();
    for (int p = 0; p < cnt; ++p) {
      const float t = prim_hit(sp + p * kPrimFloats, c.eye[0], c.eye[1], c.eye[2], d0, d1, d2);
      if (t < best) { best = t; bp = base + p; }
    }
  }
  if (i >= P) return;
  float o[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (bp >= 0) {
    const float* q = prims + (int64_t)bp * kPrimFloats;
    o[0] = c.eye[0] + best * d0; o[1] = c.eye[1] + best * d1; o[2] = c.eye[2] + best * d2;
    const float r0 = o[0] - q[0], r1 = o[1] - q[1], r2 = o[2] - q[2];
    // q / a with q = R^T (p - c) / a, i.e. R^T (p - c) / a^2, then R times that
    const float g0 = (q[6] * r0 + q[7] * r1 + q[8] * r2) * q[3] * q[3];
    const float g1 = (q[9] * r0 + q[10] * r1 + q[11] * r2) * q[4] * q[4];
    const float g2 = (q[12] * r0 + q[13] * r1 + q[14] * r2) * q[5] * q[5];
    float n0 = q[6] * g0 + q[9] * g1 + q[12] * g2;
    float n1 = q[7] * g0 + q[10] * g1 + q[13] * g2;
    float n2 = q[8] * g0 + q[11] * g1 + q[14] * g2;
    const float nn = 1.f / sqrtf(n0 * n0 + n1 * n1 + n2 * n2);
    o[3] = n0 * nn; o[4] = n1 * nn; o[5] = n2 * nn;
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) gbuf[k * P + i] = o[k];
  hit[i] = bp >= 0 ? 1 : 0;
}

// One secondary ray per thread, pixel-major (ray g = i (1 + K) + j): j = 0 the shadow ray
// toward the light, j = 1..K cosine-weighted AO rays (Malley: r = sqrt(u1), phi = 2 pi u2 on
// the unit disk, lifted to the hemisphere) in the basis of Duff et al. (2017) around n.
// Background pixels get (p, +z): finite rays whose answers are never used.
__global__ __launch_bounds__(kShadeThreads) void secondary_kernel(const float* __restrict__ gbuf,
                                                                  const uint8_t* __restrict__ hit, int64_t P,
                                                                  float lx, float ly, float lz, int K,
                                                                  const float* __restrict__ u, float offset,
                                                                  float* __restrict__ rays) {
  const int64_t N = P * (1 + K);
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int64_t i = g / (1 + K);
  const int j = (int)(g - i * (1 + K));
  const float p0 = gbuf[i], p1 = gbuf[P + i], p2 = gbuf[2 * P + i];
  const float n0 = gbuf[3 * P + i], n1 = gbuf[4 * P + i], n2 = gbuf[5 * P + i];
  float o0 = p0, o1 = p1, o2 = p2, d0 = 0.f, d1 = 0.f, d2 = 1.f;
  if (hit[i]) {
    o0 = p0 + offset * n0; o1 = p1 + offset * n1; o2 = p2 + offset * n2;
    if (j == 0) {
      d0 = lx - o0; d1 = ly - o1; d2 = lz - o2;
    } else {
      const int64_t k = i * K + (j - 1);
      const float u1 = u[k], u2 = u[P * K + k];
      const float r = sqrtf(u1);
      float sn, cs;
      sincospif(2.f * u2, &sn, &cs);
      const float ax = r * cs, ay = r * sn, az = sqrtf(fmaxf(0.f, 1.f - u1));
      const float sg = n2 >= 0.f ? 1.f : -1.f;
      const float a = -1.f / (sg + n2);
      const float b = n0 * n1 * a;
      const float t0 = 1.f + sg * n0 * n0 * a, t1 = sg * b, t2 = -sg * n0;
      const float b0 = b, b1 = sg + n1 * n1 * a, b2 = -n1;
      d0 = ax * t0 + ay * b0 + az * n0;
      d1 = ax * t1 + ay * b1 + az * n1;
      d2 = ax * t2 + ay * b2 + az * n2;
    }
    const float inv = 1.f / sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
    d0 *= inv; d1 *= inv; d2 *= inv;
  }
  rays[g] = o0; rays[N + g] = o1; rays[2 * N + g] = o2;
  rays[3 * N + g] = d0; rays[4 * N + g] = d1; rays[5 * N + g] = d2;
}

// One pixel per thread: shadow = the shadow ray hits closer than the light; AO = the share of
// AO rays that hit within ao_radius.  A ray hits when xi > 0.5 (the field's answer) or, with
// xi == NULL, when ray_hit is set (the exact cast).
__global__ __launch_bounds__(kShadeThreads) void shade_kernel(const float* __restrict__ t,
                                                              const float* __restrict__ xi,
                                                              const uint8_t* __restrict__ ray_hit,
                                                              const float* __restrict__ gbuf,
                                                              const uint8_t* __restrict__ hit, int64_t P, float lx,
                                                              float ly, float lz, int K, float offset,
                                                              float ao_radius, float* __restrict__ shadow,
                                                              float* __restrict__ ao) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  float s = 0.f, a = 0.f;
  if (hit[i]) {
    const float o0 = gbuf[i] + offset * gbuf[3 * P + i];
    const float o1 = gbuf[P + i] + offset * gbuf[4 * P + i];
    const float o2 = gbuf[2 * P + i] + offset * gbuf[5 * P + i];
    const float e0 = lx - o0, e1 = ly - o1, e2 = lz - o2;
    const float dist = sqrtf(e0 * e0 + e1 * e1 + e2 * e2);
    const int64_t g = i * (1 + K);
    const bool h0 = xi ? xi[g] > 0.5f : ray_hit[g] != 0;
    s = (h0 && t[g] < dist) ? 1.f : 0.f;
    int cnt = 0;
    for (int k = 1; k <= K; ++k) {
      const bool hk = xi ? xi[g + k] > 0.5f : ray_hit[g + k] != 0;
      cnt += (hk && t[g + k] < ao_radius) ? 1 : 0;
    }
    a = K > 0 ? (float)cnt / (float)K : 0.f;
  }
  shadow[i] = s;
  ao[i] = a;
}

// Trilinear surface radiance of the res^3 vertex grid R ([z][y][x]) over [-h, h]^3 at q (clamped
// to the box; a NaN coordinate clamps to the low face, so every read stays in the grid).
__device__ __forceinline__ float radiance_at(const float* __restrict__ R, int res, float h, float q0, float q1,
                                             float q2) {
  const float inv = 0.5f / h, sc = (float)(res - 1);
  const float s0 = fminf(fmaxf((q0 + h) * inv, 0.f), 1.f) * sc;
  const float s1 = fminf(fmaxf((q1 + h) * inv, 0.f), 1.f) * sc;
  const float s2 = fminf(fmaxf((q2 + h) * inv, 0.f), 1.f) * sc;
  const int c0 = min((int)floorf(s0), res - 2), c1 = min((int)floorf(s1), res - 2), c2 = min((int)floorf(s2), res - 2);
  const float w0 = s0 - (float)c0, w1 = s1 - (float)c1, w2 = s2 - (float)c2;
  const int64_t sy = res, sz = (int64_t)res * res;
  const float* b = R + c2 * sz + c1 * sy + c0;
  const float x00 = b[0] + w0 * (b[1] - b[0]);
  const float x10 = b[sy] + w0 * (b[sy + 1] - b[sy]);
  const float x01 = b[sz] + w0 * (b[sz + 1] - b[sz]);
  const float x11 = b[sz + sy] + w0 * (b[sz + sy + 1] - b[sz + sy]);
  const float y0 = x00 + w1 * (x10 - x00), y1 = x01 + w1 * (x11 - x01);
  return y0 + w2 * (y1 - y0);
}

// One bounce, one pixel per thread: the mean over the pixel's K hemisphere rays (rays
// i (1 + K) + 1 .. i (1 + K) + K of the pixel-major secondary rays) of the radiance each ray
// sees, the surface radiance at o + t d when it hits, the sky when it misses.
__global__ __launch_bounds__(kShadeThreads) void bounce_kernel(const float* __restrict__ t,
                                                               const float* __restrict__ xi,
                                                               const uint8_t* __restrict__ ray_hit,
                                                               const float* __restrict__ rays,
                                                               const uint8_t* __restrict__ hit, int64_t P, int K,
                                                               const float* __restrict__ R, int res, float h,
                                                               float sky_lo, float sky_hi, float* __restrict__ gi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  float acc = 0.f;
  if (hit[i]) {
    const int64_t N = P * (1 + K);
    for (int k = 1; k <= K; ++k) {
      const int64_t g = i * (1 + K) + k;
      const float d0 = rays[3 * N + g], d1 = rays[4 * N + g], d2 = rays[5 * N + g];
      const bool hk = xi ? xi[g] > 0.5f : ray_hit[g] != 0;
      float L;
      if (hk) {
        const float tk = t[g];
        L = radiance_at(R, res, h, fmaf(tk, d0, rays[g]), fmaf(tk, d1, rays[N + g]), fmaf(tk, d2, rays[2 * N + g]));
      } else {
        L = sky_lo + (sky_hi - sky_lo) * (d1 + 1.f) * 0.5f;
      }
      acc += L;
    }
    acc = K > 0 ? acc / (float)K : 0.f;
  }
  gi[i] = acc;
}

// ---- training rays: area-weighted surface rays and free rays, with rejection

// Cumulative surface-area weights of the primitives (Knud Thomsen's ellipsoid area
// approximation, exact for spheres), normalised to end at 1; one thread, in double.
__global__ void area_cdf_kernel(const float* __restrict__ prims, int n_prims, float* __restrict__ cdf) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  constexpr double kP = 1.6075;
  double total = 0.0;
  for (int k = 0; k < n_prims; ++k) {
    const float* q = prims + (int64_t)k * kPrimFloats;
    const double a = pow(1.0 / q[3], kP), b = pow(1.0 / q[4], kP), c = pow(1.0 / q[5], kP);
    total += pow((a * b + a * c + b * c) / 3.0, 1.0 / kP);
  }
  double acc = 0.0;
  for (int k = 0; k < n_prims; ++k) {
    const float* q = prims + (int64_t)k * kPrimFloats;
    const double a = pow(1.0 / q[3], kP), b = pow(1.0 / q[4], kP), c = pow(1.0 / q[5], kP);
    acc += pow((a * b + a * c + b * c) / 3.0, 1.0 / kP);
    cdf[k] = k == n_prims - 1 ? 1.f : (float)(acc / total);
  }
}

// |R^T (x - c) / a|^2 - 1 (negative strictly inside).
__device__ __forceinline__ float prim_implicit(const float* q, float x0, float x1, float x2) {
  const float r0 = x0 - q[0], r1 = x1 - q[1], r2 = x2 - q[2];
  const float l0 = (q[6] * r0 + q[7] * r1 + q[8] * r2) * q[3];
  const float l1 = (q[9] * r0 + q[10] * r1 + q[11] * r2) * q[4];
  const float l2 = (q[12] * r0 + q[13] * r1 + q[14] * r2) * q[5];
  return l0 * l0 + l1 * l1 + l2 * l2 - 1.f;
}

__device__ __forceinline__ void sphere_pt(float u1, float u2, float& s0, float& s1, float& s2) {
  const float z = 1.f - 2.f * u1;
  const float r = sqrtf(fmaxf(0.f, 1.f - z * z));
  float sn, cs;
  sincospif(2.f * u2, &sn, &cs);
  s0 = r * cs; s1 = r * sn; s2 = z;
}

// One ray per thread from uniforms u [3 tries + 2][n]: candidate j uses rows 3j .. 3j + 2, the
// direction the last two rows.  Surface rays: primitive k by binary search in the cumulative
// area weights, point c + R (a s), normal R (s / a); rejected when strictly inside another
// primitive.  Free rays: origin in the box, rejected when strictly inside any primitive.
// The last candidate is kept when every one was rejected.
__global__ __launch_bounds__(kShadeThreads) void sample_kernel(const float* __restrict__ prims,
                                                               const float* __restrict__ cdf, int n_prims,
                                                               const float* __restrict__ u, int64_t n, int mode,
                                                               float box_half, float offset, int tries,
                                                               float* __restrict__ rays) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool surf = mode == 0 || (mode == 2 && (i & 1) == 0 && i < 2 * (n / 2));
  float o0 = 0.f, o1 = 0.f, o2 = 0.f;
  for (int j = 0; j < tries; ++j) {
    const float ua = u[(3 * j) * n + i], ub = u[(3 * j + 1) * n + i], uc = u[(3 * j + 2) * n + i];
    float x0, x1, x2, c0, c1, c2;
    int k = -1;
    if (surf) {
      int lo = 0, hi = n_prims - 1;   // first index whose weight exceeds ua
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cdf[mid] > ua) hi = mid; else lo = mid + 1;
      }
      k = lo;
      const float* q = prims + (int64_t)k * kPrimFloats;
      float s0, s1, s2;
      sphere_pt(ub, uc, s0, s1, s2);
      const float a0 = 1.f / q[3], a1 = 1.f / q[4], a2 = 1.f / q[5];
      // R v = sum_row (R^T)[row][m] v_row
      const float v0 = a0 * s0, v1 = a1 * s1, v2 = a2 * s2;
      x0 = q[0] + q[6] * v0 + q[9] * v1 + q[12] * v2;
      x1 = q[1] + q[7] * v0 + q[10] * v1 + q[13] * v2;
      x2 = q[2] + q[8] * v0 + q[11] * v1 + q[14] * v2;
      const float w0 = s0 * q[3], w1 = s1 * q[4], w2 = s2 * q[5];
      float n0 = q[6] * w0 + q[9] * w1 + q[12] * w2;
      float n1 = q[7] * w0 + q[10] * w1 + q[13] * w2;
      float n2 = q[8] * w0 + q[11] * w1 + q[14] * w2;
      const float nn = 1.f / sqrtf(n0 * n0 + n1 * n1 + n2 * n2);
      c0 = x0 + offset * (n0 * nn); c1 = x1 + offset * (n1 * nn); c2 = x2 + offset * (n2 * nn);
    } else {
      x0 = -box_half + 2.f * box_half * ua;
      x1 = -box_half + 2.f * box_half * ub;
      x2 = -box_half + 2.f * box_half * uc;
      c0 = x0; c1 = x1; c2 = x2;
    }
    bool inside = false;
    for (int m = 0; m < n_prims && !inside; ++m)
      inside = m != k && prim_implicit(prims + (int64_t)m * kPrimFloats, x0, x1, x2) < 0.f;
    o0 = c0; o1 = c1; o2 = c2;
    if (!inside) break;
  }
  float d0, d1, d2;
  sphere_pt(u[(3 * tries) * n + i], u[(3 * tries + 1) * n + i], d0, d1, d2);
  rays[i] = o0; rays[n + i] = o1; rays[2 * n + i] = o2;
  rays[3 * n + i] = d0; rays[4 * n + i] = d1; rays[5 * n + i] = d2;
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kShadeThreads - 1) / kShadeThreads); }

}  // namespace
}  // namespace ddf

using namespace ddf;

extern "C" {

int ddf_primary_gbuffer(const ddf_camera* cam, const float* prims, int32_t n_prims, float* gbuf, uint8_t* hit,
                        void* stream) {
  int rc;
  if (!cam) return fail(DDF_ERR_INVALID_ARG, "cam is NULL");
  if (cam->width < 1 || cam->height < 1 || (int64_t)cam->width * cam->height > (int64_t)INT32_MAX)
    return fail(DDF_ERR_INVALID_ARG, "image size %d x %d out of range", cam->width, cam->height);
  if (!(cam->fov_y > 0.f && cam->fov_y < 3.1f)) return fail(DDF_ERR_INVALID_ARG, "fov_y out of (0, 3.1)");
  if (n_prims < 1) return fail(DDF_ERR_INVALID_ARG, "n_prims must be >= 1");
  if ((rc = check_ptr(prims, "prims")) || (rc = check_ptr(gbuf, "gbuf")) || (rc = check_ptr(hit, "hit"))) return rc;
  // the camera frame in double on the host
  double f[3], r[3], u[3];
  for (int k = 0; k < 3; ++k) f[k] = (double)cam->target[k] - cam->eye[k];
  const double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  r[0] = f[1] * cam->up[2] - f[2] * cam->up[1];
  r[1] = f[2] * cam->up[0] - f[0] * cam->up[2];
  r[2] = f[0] * cam->up[1] - f[1] * cam->up[0];
  const double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (!(fl > 0) || !(rl > 1e-12 * fl)) return fail(DDF_ERR_INVALID_ARG, "degenerate camera (eye == target or up parallel to the view)");
  for (int k = 0; k < 3; ++k) { f[k] /= fl; r[k] /= rl; }
  u[0] = r[1] * f[2] - r[2] * f[1];
  u[1] = r[2] * f[0] - r[0] * f[2];
  u[2] = r[0] * f[1] - r[1] * f[0];
  CamArgs c{};
  for (int k = 0; k < 3; ++k) {
    c.eye[k] = cam->eye[k]; c.f[k] = (float)f[k]; c.r[k] = (float)r[k]; c.u[k] = (float)u[k];
  }
  const double th = std::tan((double)cam->fov_y / 2);
  c.tx = (float)(th * cam->width / cam->height);
  c.ty = (float)th;
  c.W = cam->width;
  c.H = cam->height;
  g_err_clear();
  const int64_t P = (int64_t)cam->width * cam->height;
  gbuffer_kernel<<<grid_for(P), kShadeThreads, 0, (hipStream_t)stream>>>(c, prims, n_prims, gbuf, hit);
  return hip_status(hipGetLastError(), "ddf_primary_gbuffer launch");
}

int ddf_secondary_rays(const float* gbuf, const uint8_t* hit, int64_t n_px, const float* light, int32_t n_ao,
                       const float* u, float offset, float* rays, void* stream) {
  int rc;
  if (n_ao < 0 || n_ao > 1024) return fail(DDF_ERR_INVALID_ARG, "n_ao = %d out of 0..1024", n_ao);
  if (n_px < 0 || n_px * (1 + n_ao) > (int64_t)INT32_MAX)
    return fail(DDF_ERR_INVALID_ARG, "n_px = %lld out of range", (long long)n_px);
  if (!light) return fail(DDF_ERR_INVALID_ARG, "light is NULL");
  if (!(offset >= 0.f)) return fail(DDF_ERR_INVALID_ARG, "offset must be >= 0");
  if (n_px == 0) return DDF_OK;
  if ((rc = check_ptr(gbuf, "gbuf")) || (rc = check_ptr(hit, "hit")) || (rc = check_ptr(rays, "rays"))) return rc;
  if (n_ao > 0 && (rc = check_ptr(u, "u"))) return rc;
  g_err_clear();
  const int64_t N = n_px * (1 + n_ao);
  secondary_kernel<<<grid_for(N), kShadeThreads, 0, (hipStream_t)stream>>>(gbuf, hit, n_px, light[0], light[1],
                                                                            light[2], n_ao, u, offset, rays);
  return hip_status(hipGetLastError(), "ddf_secondary_rays launch");
}

int ddf_shade(const float* t, const float* xi, const uint8_t* ray_hit, const float* gbuf, const uint8_t* hit,
              int64_t n_px, const float* light, int32_t n_ao, float offset, float ao_radius, float* shadow, float* ao,
              void* stream) {
  int rc;
  if (n_ao < 0 || n_ao > 1024) return fail(DDF_ERR_INVALID_ARG, "n_ao = %d out of 0..1024", n_ao);
  if (n_px < 0 || n_px * (1 + n_ao) > (int64_t)INT32_MAX)
    return fail(DDF_ERR_INVALID_ARG, "n_px = %lld out of range", (long long)n_px);
  if (!light) return fail(DDF_ERR_INVALID_ARG, "light is NULL");
  if (!(offset >= 0.f) || !(ao_radius > 0.f)) return fail(DDF_ERR_INVALID_ARG, "offset < 0 or ao_radius <= 0");
  if ((xi == nullptr) == (ray_hit == nullptr)) return fail(DDF_ERR_INVALID_ARG, "pass exactly one of xi and ray_hit");
  if (n_px == 0) return DDF_OK;
  if ((rc = check_ptr(t, "t")) || (rc = check_ptr(gbuf, "gbuf")) || (rc = check_ptr(hit, "hit")) ||
      (rc = check_ptr(shadow, "shadow")) || (rc = check_ptr(ao, "ao")))
    return rc;
  if ((rc = check_ptr(xi ? (const void*)xi : (const void*)ray_hit, xi ? "xi" : "ray_hit"))) return rc;
  g_err_clear();
  shade_kernel<<<grid_for(n_px), kShadeThreads, 0, (hipStream_t)stream>>>(t, xi, ray_hit, gbuf, hit, n_px, light[0],
                                                                          light[1], light[2], n_ao, offset, ao_radius,
                                                                          shadow, ao);
  return hip_status(hipGetLastError(), "ddf_shade launch");
}

int ddf_bounce(const float* t, const float* xi, const uint8_t* ray_hit, const float* rays, const uint8_t* hit,
               int64_t n_px, int32_t n_ao, const float* radiance, int32_t res, float box_half, float sky_lo,
               float sky_hi, float* gi, void* stream) {
  int rc;
  if (n_ao < 0 || n_ao > 1024) return fail(DDF_ERR_INVALID_ARG, "n_ao = %d out of 0..1024", n_ao);
  if (n_px < 0 || n_px * (1 + n_ao) > (int64_t)INT32_MAX)
    return fail(DDF_ERR_INVALID_ARG, "n_px = %lld out of range", (long long)n_px);
  if (res < 2 || res > 1024) return fail(DDF_ERR_INVALID_ARG, "res = %d out of 2..1024", res);
  if (!(box_half > 0.f) || !std::isfinite(box_half)) return fail(DDF_ERR_INVALID_ARG, "box_half must be > 0");
  if (!std::isfinite(sky_lo) || !std::isfinite(sky_hi)) return fail(DDF_ERR_INVALID_ARG, "sky radiance not finite");
  if ((xi == nullptr) == (ray_hit == nullptr)) return fail(DDF_ERR_INVALID_ARG, "pass exactly one of xi and ray_hit");
  if (n_px == 0) return DDF_OK;
  if ((rc = check_ptr(t, "t")) || (rc = check_ptr(rays, "rays")) || (rc = check_ptr(hit, "hit")) ||
      (rc = check_ptr(radiance, "radiance")) || (rc = check_ptr(gi, "gi")))
    return rc;
  if ((rc = check_ptr(xi ? (const void*)xi : (const void*)ray_hit, xi ? "xi" : "ray_hit"))) return rc;
  g_err_clear();
  bounce_kernel<<<grid_for(n_px), kShadeThreads, 0, (hipStream_t)stream>>>(t, xi, ray_hit, rays, hit, n_px, n_ao,
                                                                           radiance, res, box_half, sky_lo, sky_hi,
                                                                           gi);
  return hip_status(hipGetLastError(), "ddf_bounce launch");
}

int ddf_prim_area_cdf(const float* prims, int32_t n_prims, float* cdf, void* stream) {
  int rc;
  if (n_prims < 1) return fail(DDF_ERR_INVALID_ARG, "n_prims must be >= 1");
  if ((rc = check_ptr(prims, "prims")) || (rc = check_ptr(cdf, "cdf"))) return rc;
  g_err_clear();
  area_cdf_kernel<<<1, 64, 0, (hipStream_t)stream>>>(prims, n_prims, cdf);
  return hip_status(hipGetLastError(), "ddf_prim_area_cdf launch");
}

int ddf_sample_rays(const float* prims, int32_t n_prims, const float* cdf, const float* u, int64_t n, int32_t mode,
                    float box_half, float offset, int32_t tries, float* rays, void* stream) {
  int rc;
  if (n_prims < 1) return fail(DDF_ERR_INVALID_ARG, "n_prims must be >= 1");
  if (n < 0 || n > (int64_t)INT32_MAX / 32) return fail(DDF_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (mode < 0 || mode > 2) return fail(DDF_ERR_INVALID_ARG, "mode must be 0, 1 or 2");
  if (tries < 1 || tries > 16) return fail(DDF_ERR_INVALID_ARG, "tries must be in 1..16");
  if (!(box_half > 0.f) || !(offset >= 0.f)) return fail(DDF_ERR_INVALID_ARG, "box_half <= 0 or offset < 0");
  if (n == 0) return DDF_OK;
  if ((rc = check_ptr(prims, "prims")) || (rc = check_ptr(cdf, "cdf")) || (rc = check_ptr(u, "u")) ||
      (rc = check_ptr(rays, "rays")))
    return rc;
  g_err_clear();
  sample_kernel<<<grid_for(n), kShadeThreads, 0, (hipStream_t)stream>>>(prims, cdf, n_prims, u, n, mode, box_half,
                                                                        offset, tries, rays);
  return hip_status(hipGetLastError(), "ddf_sample_rays launch");
}

}  // extern "C"
