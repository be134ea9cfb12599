// C ABI of libddf: host-side validation and dispatch (declared in include/ddf.h).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>

#include "ddf_fwd.h"
#include "ddf_internal.h"
#include "ddf_train.h"

namespace ddf {

static thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

void g_err_clear() { g_err[0] = 0; }

int hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return DDF_OK;
  return fail(DDF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int check_desc(const ddf_net_desc* d) {
  if (!d) return fail(DDF_ERR_INVALID_ARG, "desc is NULL");
  if (d->n_in != 6 && d->n_in != 3) return fail(DDF_ERR_INVALID_ARG, "n_in must be 6 or 3, got %d", d->n_in);
  if (d->n_freq < 1 || d->n_freq > 12) return fail(DDF_ERR_INVALID_ARG, "n_freq must be in 1..12, got %d", d->n_freq);
  if (d->n_hidden < 1 || d->n_hidden > kMaxLayers)
    return fail(DDF_ERR_INVALID_ARG, "n_hidden must be in 1..%d, got %d", kMaxLayers, d->n_hidden);
  if (d->n_out != 1 && d->n_out != 2) return fail(DDF_ERR_INVALID_ARG, "n_out must be 1 or 2, got %d", d->n_out);
  if (d->precision < DDF_FP32 || d->precision > DDF_FP8_E4M3)
    return fail(DDF_ERR_INVALID_ARG, "unknown precision %d", d->precision);
  if (d->width != 128 && d->width != 256 && d->width != 512 && d->width != 1024)
    return fail(DDF_ERR_UNSUPPORTED, "width must be 128, 256, 512 or 1024, got %d", d->width);
  Layout L = make_layout(*d);
  if (L.k1 > d->width)
    return fail(DDF_ERR_UNSUPPORTED, "padded layer-1 input (%d) wider than the hidden width (%d)", L.k1, d->width);
  if (d->precision == DDF_FP8_E4M3 && (d->width < 256 || L.k1 > 256))
    return fail(DDF_ERR_UNSUPPORTED, "fp8 needs width >= 256 and at most 128 padded input features");
  return DDF_OK;
}

int check_ptr(const void* p, const char* name) {
  if (!p) return fail(DDF_ERR_INVALID_ARG, "%s is NULL", name);
  if (!aligned16(p)) return fail(DDF_ERR_INVALID_ARG, "%s is not 16-byte aligned", name);
  return DDF_OK;
}

FwdArgs base_args(const ddf_net_desc& d, const void* packed) {
  FwdArgs a{};
  a.packed = static_cast<const uint8_t*>(packed);
  a.lay = make_layout(d);
  a.n_in = d.n_in; a.n_freq = d.n_freq; a.n_hidden = d.n_hidden; a.n_out = d.n_out;
  a.l_begin = 0; a.l_end = d.n_hidden;
  return a;
}

// ------------------------------------------------------------------ sphere tracing

__global__ void trace_init_kernel(int64_t n, int32_t* idx0, int32_t* counts, int n_counts,
                                  float* t, uint8_t* hit, int32_t* steps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_counts) counts[i] = i == 0 ? (int32_t)n : 0;
  if (i < n) {
    idx0[i] = (int32_t)i;
    t[i] = 0.f;
    hit[i] = 0;
    if (steps) steps[i] = 0;
  }
}

__global__ void zero_u32_kernel(unsigned int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Smallest power of two s with amax / s <= 448 (1 for amax <= 0).
static float pow2_scale_e4m3(float amax) {
  if (!(amax > 0.f)) return 1.f;
  int e;
  const float m = frexpf(amax, &e);   // amax = m 2^e, 0.5 <= m < 1
  return ldexpf(1.f, e - 9 + (2.f * m > 1.75f ? 1 : 0));
}

// ------------------------------------------------------------------ supervision targets

__global__ void cast_kernel(const float* prims, int n_prims, const float* rays, int64_t n,
                            float* t_gt, uint8_t* hit) {
  extern __shared__ float sp[];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float x0 = 0, x1 = 0, x2 = 0, d0 = 0, d1 = 0, d2 = 0;
  if (i < n) {
    x0 = rays[i]; x1 = rays[n + i]; x2 = rays[2 * n + i];
    d0 = rays[3 * n + i]; d1 = rays[4 * n + i]; d2 = rays[5 * n + i];
  }
  float best = __builtin_inff();
  constexpr int kChunk = 256;
  for (int base = 0; base < n_prims; base += kChunk) {
    const int cnt = min(kChunk, n_prims - base);
    __syncthreads();
    for (int j = threadIdx.x; j < cnt * 16; j += blockDim.x) sp[j] = prims[(int64_t)base * 16 + j];
    __syncthreads();
    for (int p = 0; p < cnt; ++p) {
      const float* q = sp + p * 16;
      const float r0 = x0 - q[0], r1 = x1 - q[1], r2 = x2 - q[2];
      // local frame: R^T (x - c) / a and R^T d / a
      const float l0 = (q[6] * r0 + q[7] * r1 + q[8] * r2) * q[3];
      const float l1 = (q[9] * r0 + q[10] * r1 + q[11] * r2) * q[4];
      const float l2 = (q[12] * r0 + q[13] * r1 + q[14] * r2) * q[5];
      const float e0 = (q[6] * d0 + q[7] * d1 + q[8] * d2) * q[3];
      const float e1 = (q[9] * d0 + q[10] * d1 + q[11] * d2) * q[4];
      const float e2 = (q[12] * d0 + q[13] * d1 + q[14] * d2) * q[5];
      const float A = e0 * e0 + e1 * e1 + e2 * e2;
      const float B = l0 * e0 + l1 * e1 + l2 * e2;
      const float Cc = l0 * l0 + l1 * l1 + l2 * l2 - 1.f;
      const float disc = B * B - A * Cc;
      if (disc >= 0.f) {
        const float sq = sqrtf(disc);
        const float k = -(B + copysignf(sq, B));
        const float ra = k / A;
        const float rb = k != 0.f ? Cc / k : -B / A;
        const float lo = fminf(ra, rb), hi = fmaxf(ra, rb);
        const float tt = lo > 0.f ? lo : (hi > 0.f ? hi : __builtin_inff());
        best = fminf(best, tt);
      }
    }
  }
  if (i < n) {
    t_gt[i] = best;
    hit[i] = best < __builtin_inff() ? 1 : 0;
  }
}

__global__ void scene_sdf_kernel(const float* prims, int n_prims, const float* pts, int64_t n, float* out) {
  extern __shared__ float sp[];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float x0 = 0, x1 = 0, x2 = 0;
  if (i < n) { x0 = pts[i]; x1 = pts[n + i]; x2 = pts[2 * n + i]; }
  float best = __builtin_inff();
  constexpr int kChunk = 256;
  for (int base = 0; base < n_prims; base += kChunk) {
    const int cnt = min(kChunk, n_prims - base);
    __syncthreads();
    for (int j = threadIdx.x; j < cnt * 16; j += blockDim.x) sp[j] = prims[(int64_t)base * 16 + j];
    __syncthreads();
    for (int p = 0; p < cnt; ++p) {
      const float* q = sp + p * 16;
      const float r0 = x0 - q[0], r1 = x1 - q[1], r2 = x2 - q[2];
      const float l0 = (q[6] * r0 + q[7] * r1 + q[8] * r2) * q[3];
      const float l1 = (q[9] * r0 + q[10] * r1 + q[11] * r2) * q[4];
      const float l2 = (q[12] * r0 + q[13] * r1 + q[14] * r2) * q[5];
      best = fminf(best, (sqrtf(l0 * l0 + l1 * l1 + l2 * l2) - 1.f) * q[15]);
    }
  }
  if (i < n) out[i] = best;
}

}  // namespace ddf

using namespace ddf;

extern "C" {

const char* ddf_status_string(int s) {
  switch (s) {
    case DDF_OK: return "ok";
    case DDF_ERR_INVALID_ARG: return "invalid argument";
    case DDF_ERR_UNSUPPORTED: return "unsupported";
    case DDF_ERR_WORKSPACE: return "workspace too small";
    case DDF_ERR_HIP: return "hip error";
  }
  return "unknown status";
}

const char* ddf_last_error(void) { return g_err; }

size_t ddf_param_count(const ddf_net_desc* d) {
  if (check_desc(d) != DDF_OK) return 0;
  size_t nf = (size_t)d->n_in * (1 + 2 * d->n_freq);
  size_t w = d->width;
  return w * nf + w + (size_t)(d->n_hidden - 1) * (w * w + w) + (size_t)d->n_out * w + d->n_out;
}

int ddf_param_offsets(const ddf_net_desc* d, int32_t layer, size_t* w_off, size_t* b_off) {
  int rc;
  if ((rc = check_desc(d))) return rc;
  if (layer < 0 || layer > d->n_hidden)
    return fail(DDF_ERR_INVALID_ARG, "layer = %d must be in 0..%d (n_hidden = the head)", layer, d->n_hidden);
  if (!w_off || !b_off) return fail(DDF_ERR_INVALID_ARG, "w_off and b_off must not be NULL");
  const size_t nf = (size_t)d->n_in * (1 + 2 * d->n_freq);
  const size_t w = d->width;
  size_t off = 0;
  for (int l = 0; l < layer; ++l) off += (l == 0 ? nf : w) * w + w;
  *w_off = off;
  *b_off = off + (layer == d->n_hidden ? (size_t)d->n_out * w : (layer == 0 ? nf : w) * w);
  return DDF_OK;
}

size_t ddf_packed_bytes(const ddf_net_desc* d) {
  if (check_desc(d) != DDF_OK) return 0;
  return (size_t)make_layout(*d).total;
}

int ddf_pack(const ddf_net_desc* d, const float* master, const float* act_scales, void* packed,
             void* stream) {
  int rc;
  if ((rc = check_desc(d))) return rc;
  if ((rc = check_ptr(master, "master"))) return rc;
  if ((rc = check_ptr(packed, "packed"))) return rc;
  if (d->precision == DDF_FP8_E4M3) {
    if (!act_scales && d->n_hidden > 1) return fail(DDF_ERR_INVALID_ARG, "fp8 packing needs act_scales");
    for (int l = 0; l + 1 < d->n_hidden; ++l) {
      float s = act_scales[l];
      int e;
      if (!(s > 0.f) || !std::isfinite(s) || frexpf(s, &e) != 0.5f)
        return fail(DDF_ERR_INVALID_ARG, "act_scales[%d] = %g is not a positive power of two", l, s);
    }
  }
  g_err[0] = 0;
  return hip_status(launch_pack(*d, master, act_scales, packed, (hipStream_t)stream, true),
                    "ddf_pack launch");
}

int ddf_query(const ddf_net_desc* d, const void* packed, const float* rays, int64_t n, float* t,
              float* xi, void* stream) {
  int rc;
  if ((rc = check_desc(d))) return rc;
  if (d->n_in != 6 || d->n_out != 2) return fail(DDF_ERR_INVALID_ARG, "ddf_query needs n_in 6 and n_out 2");
  if (n < 0 || n > (int64_t)INT32_MAX) return fail(DDF_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (n == 0) return DDF_OK;
  if ((rc = check_ptr(packed, "packed")) || (rc = check_ptr(rays, "rays")) ||
      (rc = check_ptr(t, "t")) || (rc = check_ptr(xi, "xi")))
    return rc;
  FwdArgs a = base_args(*d, packed);
  a.in = rays; a.n = n; a.stride = n; a.mode = kModeQuery; a.out0 = t; a.out1 = xi;
  g_err[0] = 0;
  return hip_status(launch_forward(*d, a, n, (hipStream_t)stream), "ddf_query launch");
}

int ddf_query_hidden(const ddf_net_desc* d, const void* packed, const float* in, int64_t n, float* h,
                     void* stream) {
  int rc;
  if ((rc = check_desc(d))) return rc;
  if (n < 0 || n > (int64_t)INT32_MAX) return fail(DDF_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (n == 0) return DDF_OK;
  if ((rc = check_ptr(packed, "packed")) || (rc = check_ptr(in, "rays")) || (rc = check_ptr(h, "h")))
    return rc;
  FwdArgs a = base_args(*d, packed);
  a.in = in; a.n = n; a.stride = n; a.mode = kModeHidden; a.out0 = h;
  g_err[0] = 0;
  return hip_status(launch_forward(*d, a, n, (hipStream_t)stream), "ddf_query_hidden launch");
}

int sdf_eval(const ddf_net_desc* d, const void* packed, const float* points, int64_t n, float* sdf,
             void* stream) {
  int rc;
  if ((rc = check_desc(d))) return rc;
  if (d->n_in != 3 || d->n_out != 1) return fail(DDF_ERR_INVALID_ARG, "sdf_eval needs n_in 3 and n_out 1");
  if (n < 0 || n > (int64_t)INT32_MAX) return fail(DDF_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (n == 0) return DDF_OK;
  if ((rc = check_ptr(packed, "packed")) || (rc = check_ptr(points, "points")) ||
      (rc = check_ptr(sdf, "sdf")))
    return rc;
  FwdArgs a = base_args(*d, packed);
  a.in = points; a.n = n; a.stride = n; a.mode = kModeSdf; a.out0 = sdf;
  g_err[0] = 0;
  return hip_status(launch_forward(*d, a, n, (hipStream_t)stream), "sdf_eval launch");
}

size_t ddf_fp8_calib_workspace_bytes(const ddf_net_desc* d, int64_t n) {
  if (check_desc(d) != DDF_OK || n < 0) return 0;
  return 256 + (size_t)align256(4 * n) * 2;
}

int ddf_fp8_act_scales(const ddf_net_desc* d, const void* packed_fp32, const float* rays, int64_t n,
                       float* act_scales_host, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_desc(d))) return rc;
  if (d->n_in != 6 || d->n_out != 2) return fail(DDF_ERR_INVALID_ARG, "calibration needs a DDF net (n_in 6, n_out 2)");
  if (n < 1 || n > (int64_t)INT32_MAX) return fail(DDF_ERR_INVALID_ARG, "calibration needs 1..2^31-1 rays");
  if (!act_scales_host) return fail(DDF_ERR_INVALID_ARG, "act_scales_host is NULL");
  if ((rc = check_ptr(packed_fp32, "packed_fp32")) || (rc = check_ptr(rays, "rays")) || (rc = check_ptr(ws, "ws")))
    return rc;
  if (ws_bytes < ddf_fp8_calib_workspace_bytes(d, n))
    return fail(DDF_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, ddf_fp8_calib_workspace_bytes(d, n));
  ddf_net_desc d32 = *d;
  d32.precision = DDF_FP32;
  hipStream_t st = (hipStream_t)stream;
  uint8_t* w = static_cast<uint8_t*>(ws);
  unsigned int* amax = reinterpret_cast<unsigned int*>(w);
  zero_u32_kernel<<<1, 64, 0, st>>>(amax, kMaxLayers);
  if ((rc = hip_status(hipGetLastError(), "calibration init"))) return rc;
  FwdArgs a = base_args(d32, packed_fp32);
  a.in = rays; a.n = n; a.stride = n; a.mode = kModeCalib;
  a.out0 = reinterpret_cast<float*>(w + 256);
  a.out1 = reinterpret_cast<float*>(w + 256 + align256(4 * n));
  a.amax = amax;
  g_err[0] = 0;
  if ((rc = hip_status(launch_forward(d32, a, n, st), "calibration launch"))) return rc;
  unsigned int host[kMaxLayers];
  if ((rc = hip_status(hipMemcpyAsync(host, amax, sizeof(host), hipMemcpyDeviceToHost, st), "calibration copy")))
    return rc;
  if ((rc = hip_status(hipStreamSynchronize(st), "calibration sync"))) return rc;
  for (int l = 0; l + 1 < d->n_hidden; ++l) {
    float m;
    memcpy(&m, &host[l], 4);
    act_scales_host[l] = pow2_scale_e4m3(m);
  }
  return DDF_OK;
}

__global__ void pool_init_kernel(int64_t n, unsigned long long* pool, float* t, uint8_t* hit, int32_t* steps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *pool = 0ull;
  if (i < n) {
    t[i] = 0.f;
    hit[i] = 0;
    if (steps) steps[i] = 0;
  }
}

// Compute units of the current device (the persistent trace's grid: one workgroup per CU).
static int device_cus() {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
    cached[dev] = c;
  }
  return cached[dev];
}

size_t sdf_trace_workspace_bytes(int64_t n) {
  if (n < 0) return 0;
  // two active lists of n int32 and (max steps + 1) counters, max steps <= 4096
  return (size_t)align256(4 * n) * 2 + (size_t)align256(4 * 4097);
}

int sdf_sphere_trace(const ddf_net_desc* d, const void* packed, const float* rays, int64_t n,
                     int32_t max_steps, float hit_eps, float t_max, float* t, uint8_t* hit,
                     int32_t* steps, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_desc(d))) return rc;
  if (d->n_in != 3 || d->n_out != 1) return fail(DDF_ERR_INVALID_ARG, "sphere tracing needs an SDF net (n_in 3, n_out 1)");
  if (n < 0 || n > (int64_t)INT32_MAX) return fail(DDF_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (max_steps < 1 || max_steps > 4096) return fail(DDF_ERR_INVALID_ARG, "max_steps must be in 1..4096");
  if (!(hit_eps > 0.f) || !(t_max > 0.f)) return fail(DDF_ERR_INVALID_ARG, "hit_eps and t_max must be positive");
  if (n == 0) return DDF_OK;
  if ((rc = check_ptr(packed, "packed")) || (rc = check_ptr(rays, "rays")) || (rc = check_ptr(t, "t")) ||
      (rc = check_ptr(hit, "hit")) || (rc = check_ptr(ws, "ws")))
    return rc;
  if (steps && (rc = check_ptr(steps, "steps"))) return rc;
  if (ws_bytes < sdf_trace_workspace_bytes(n))
    return fail(DDF_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, sdf_trace_workspace_bytes(n));
  hipStream_t st = (hipStream_t)stream;
  uint8_t* w = static_cast<uint8_t*>(ws);
  int32_t* lists[2] = {reinterpret_cast<int32_t*>(w), reinterpret_cast<int32_t*>(w + align256(4 * n))};
  int32_t* counts = reinterpret_cast<int32_t*>(w + 2 * align256(4 * n));
  const int64_t init_n = n > max_steps + 1 ? n : max_steps + 1;
  trace_init_kernel<<<(unsigned)((init_n + 255) / 256), 256, 0, st>>>(n, lists[0], counts, max_steps + 1, t,
                                                                     hit, steps);
  if ((rc = hip_status(hipGetLastError(), "trace init"))) return rc;
  FwdArgs a = base_args(*d, packed);
  a.in = rays; a.n = n; a.stride = n; a.mode = kModeTrace;
  a.t_state = t; a.hit = hit; a.steps = steps; a.hit_eps = hit_eps; a.t_max = t_max;
  g_err[0] = 0;
  for (int s = 0; s < max_steps; ++s) {
    a.idx = lists[s & 1]; a.count = counts + s;
    a.next_idx = lists[(s + 1) & 1]; a.next_count = counts + s + 1;
    a.step = s;
    if ((rc = hip_status(launch_forward(*d, a, n, st), "sphere-trace step launch"))) return rc;
  }
  return DDF_OK;
}

int sdf_sphere_trace_pool(const ddf_net_desc* d, const void* packed, const float* rays, int64_t n,
                          int32_t max_steps, float hit_eps, float t_max, float* t, uint8_t* hit, int32_t* steps,
                          void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_desc(d))) return rc;
  if (d->n_in != 3 || d->n_out != 1) return fail(DDF_ERR_INVALID_ARG, "sphere tracing needs an SDF net (n_in 3, n_out 1)");
  if (d->precision == DDF_FP8_E4M3 || d->width < 256)
    return fail(DDF_ERR_UNSUPPORTED, "the persistent trace is built for fp32 and bf16 nets of width 256..1024");
  if (n < 0 || n > (int64_t)INT32_MAX) return fail(DDF_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (max_steps < 1 || max_steps > 4096) return fail(DDF_ERR_INVALID_ARG, "max_steps must be in 1..4096");
  if (!(hit_eps > 0.f) || !(t_max > 0.f)) return fail(DDF_ERR_INVALID_ARG, "hit_eps and t_max must be positive");
  if (n == 0) return DDF_OK;
  if ((rc = check_ptr(packed, "packed")) || (rc = check_ptr(rays, "rays")) || (rc = check_ptr(t, "t")) ||
      (rc = check_ptr(hit, "hit")) || (rc = check_ptr(ws, "ws")))
    return rc;
  if (steps && (rc = check_ptr(steps, "steps"))) return rc;
  if (ws_bytes < 256) return fail(DDF_ERR_WORKSPACE, "workspace %zu < 256 bytes", ws_bytes);
  hipStream_t st = (hipStream_t)stream;
  unsigned long long* pool = static_cast<unsigned long long*>(ws);
  pool_init_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, pool, t, hit, steps);
  if ((rc = hip_status(hipGetLastError(), "trace init"))) return rc;
  FwdArgs a = base_args(*d, packed);
  a.in = rays; a.n = n; a.stride = n; a.mode = kModePool;
  a.t_state = t; a.hit = hit; a.steps = steps; a.hit_eps = hit_eps; a.t_max = t_max;
  a.max_steps = max_steps; a.pool = pool;
  const int64_t tiles = (n + geo_of(d->precision).rays_per_wg - 1) / geo_of(d->precision).rays_per_wg;
  const int n_wg = (int)(tiles < device_cus() ? tiles : device_cus());
  g_err[0] = 0;
  return hip_status(launch_pool_trace(*d, a, n_wg, st), "persistent trace launch");
}

int ddf_cast_targets(const float* prims, int32_t n_prims, const float* rays, int64_t n, float* t_gt,
                     uint8_t* hit, void* stream) {
  int rc;
  if (n_prims < 1) return fail(DDF_ERR_INVALID_ARG, "n_prims must be >= 1");
  if (n < 0 || n > (int64_t)INT32_MAX) return fail(DDF_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (n == 0) return DDF_OK;
  if ((rc = check_ptr(prims, "prims")) || (rc = check_ptr(rays, "rays")) || (rc = check_ptr(t_gt, "t_gt")) ||
      (rc = check_ptr(hit, "hit")))
    return rc;
  g_err[0] = 0;
  cast_kernel<<<(unsigned)((n + 255) / 256), 256, 256 * 16 * sizeof(float), (hipStream_t)stream>>>(
      prims, n_prims, rays, n, t_gt, hit);
  return hip_status(hipGetLastError(), "ddf_cast_targets launch");
}

// Self-consistency points (Sec. III-B, III-D): slot i with u[0][i] < frac takes the first hit
// ray j among the kShiftWalk rays from floor(u[1][i] n) on (cyclically) and moves its origin
// forward by s = u[2][i] t_j, target t_j - s; other slots (and a selected slot that finds no
// hit) are copied.
constexpr int64_t kShiftWalk = 1024;

__global__ void shift_kernel(const float* rays, const float* t_gt, const uint8_t* hit, const float* u, float frac,
                             int64_t n, float* rays_out, float* t_out, uint8_t* hit_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t j = i;
  float s = 0.f;
  bool shifted = false;
  if (u[i] < frac) {
    int64_t c = (int64_t)(u[n + i] * (float)n);
    if (c >= n) c = n - 1;
    const int64_t walk = n < kShiftWalk ? n : kShiftWalk;
    for (int64_t k = 0; k < walk; ++k, c = c + 1 == n ? 0 : c + 1)
      if (hit[c]) { j = c; shifted = true; break; }
    if (shifted) s = u[2 * n + i] * t_gt[j];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float x = rays[a * n + j], d = rays[(3 + a) * n + j];
    rays_out[a * n + i] = shifted ? fmaf(s, d, x) : x;
    rays_out[(3 + a) * n + i] = d;
  }
  t_out[i] = shifted ? t_gt[j] - s : t_gt[i];
  hit_out[i] = shifted ? 1 : hit[i];
}

int ddf_shift_rays(const float* rays, const float* t_gt, const uint8_t* hit, const float* u, float frac, int64_t n,
                   float* rays_out, float* t_out, uint8_t* hit_out, void* stream) {
  int rc;
  if (n < 0 || n > (int64_t)INT32_MAX) return fail(DDF_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (!(frac >= 0.f && frac <= 1.f)) return fail(DDF_ERR_INVALID_ARG, "frac must be in [0, 1]");
  if (n == 0) return DDF_OK;
  if ((rc = check_ptr(rays, "rays")) || (rc = check_ptr(t_gt, "t_gt")) || (rc = check_ptr(hit, "hit")) ||
      (rc = check_ptr(u, "u")) || (rc = check_ptr(rays_out, "rays_out")) || (rc = check_ptr(t_out, "t_out")) ||
      (rc = check_ptr(hit_out, "hit_out")))
    return rc;
  if (rays_out == rays || t_out == t_gt || hit_out == hit)
    return fail(DDF_ERR_INVALID_ARG, "outputs must not alias the inputs");
  g_err[0] = 0;
  shift_kernel<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(rays, t_gt, hit, u, frac, n, rays_out,
                                                                            t_out, hit_out);
  return hip_status(hipGetLastError(), "ddf_shift_rays launch");
}

float ddf_lr_cosine(int64_t step, int64_t total, float lr0, float final_frac) {
  const double s = (double)(step < 0 ? 0 : (step > total ? total : step));
  const double lo = (double)lr0 * final_frac;
  const double c = total > 0 ? cos(M_PI * s / (double)total) : 1.0;
  return (float)(lo + 0.5 * ((double)lr0 - lo) * (1.0 + c));
}

int ddf_scene_sdf(const float* prims, int32_t n_prims, const float* points, int64_t n, float* sdf, void* stream) {
  int rc;
  if (n_prims < 1) return fail(DDF_ERR_INVALID_ARG, "n_prims must be >= 1");
  if (n < 0 || n > (int64_t)INT32_MAX) return fail(DDF_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (n == 0) return DDF_OK;
  if ((rc = check_ptr(prims, "prims")) || (rc = check_ptr(points, "points")) || (rc = check_ptr(sdf, "sdf")))
    return rc;
  g_err[0] = 0;
  scene_sdf_kernel<<<(unsigned)((n + 255) / 256), 256, 256 * 16 * sizeof(float), (hipStream_t)stream>>>(
      prims, n_prims, points, n, sdf);
  return hip_status(hipGetLastError(), "ddf_scene_sdf launch");
}

}  // extern "C"
