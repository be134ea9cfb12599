// The hash-grid DDF (Sec. III-D): the ray origin through a multiresolution hash encoding
// (L levels, 2 features each, trilinear lookups in per-level tables), the direction through
// sinusoidal bands, then a ReLU MLP of width 64 and the two heads.
//
// Parameters are one fp32 vector: the table (level after level, 2 floats per entry), then
// W1 [64][D], b1, hidden W_l [64][64], b_l, heads [n_out][64], [n_out] (D = 2 L + 3 (1 + 2
// bands) <= 64).  No packing: the lookups gather straight from the table, and every block
// stages the MLP (transposed, one row per input) in LDS.
//
// Query: one ray per thread; the 8 L corner gathers are the traffic (random 8-byte reads of
// a 52 MB table that the 256 MB Infinity Cache holds); the MLP is fp32 FMA with the weights
// broadcast from LDS.  Training: the same forward writes the logits; the backward kernel
// re-runs it per ray, keeps the layer inputs and deltas for the weight-gradient reduction
// (fixed order), and scatters the position-code gradient into the table gradient with
// float atomics (the one reduction here whose order is not fixed).
#include <math.h>

#include <algorithm>
#include <mutex>

#include <hip/hip_fp16.h>

#include "ddf_chain.h"
#include "ddf_internal.h"
#include "ddf_train.h"

namespace ddf {

namespace {

constexpr int kHMaxLevels = 24;
constexpr int kHW = 64;           // MLP width
constexpr int kHIn = 64;          // padded MLP input
constexpr int kHMaxHidden = 2;   // the compiled kernels run two hidden layers
constexpr int kHT = 256;          // threads per block, one ray each
constexpr int kHRC = 64;          // rays per weight-gradient block
constexpr uint32_t kPrime1 = 2654435761u, kPrime2 = 805459861u;

struct HashLayout {
  int n_levels, d_in, n_dir, n_hidden, n_out, dir_bands;
  int res[kHMaxLevels];
  int dense[kHMaxLevels];
  int64_t off[kHMaxLevels];       // entry offset of each level
  uint32_t tmask;                 // entries per hashed level - 1
  int64_t entries;                // all table entries
  int64_t w_off[kHMaxHidden + 1], b_off[kHMaxHidden + 1];   // float offsets, heads last
  int64_t wh_off, bh_off;         // the heads' offsets again (read on the device without an index)
  int64_t params;
  float box_half;
};

HashLayout make_hash_layout(const ddf_hash_desc& d) {
  HashLayout L{};
  L.n_levels = d.n_levels;
  L.dir_bands = d.dir_bands;
  L.n_dir = 3 * (1 + 2 * d.dir_bands);
  L.d_in = 2 * d.n_levels + L.n_dir;
  L.n_hidden = d.n_hidden;
  L.n_out = d.n_out;
  L.box_half = d.box_half;
  const int64_t T = 1ll << d.log2_table;
  L.tmask = (uint32_t)(T - 1);
  int64_t off = 0;
  for (int l = 0; l < d.n_levels; ++l) {
    const int N = (int)floor((double)d.base_res * pow((double)d.growth, (double)l));
    const int64_t full = (int64_t)(N + 1) * (N + 1) * (N + 1);
    L.res[l] = N;
    L.dense[l] = full <= T;
    L.off[l] = off;
    off += full <= T ? full : T;
  }
  L.entries = off;
  int64_t p = 2 * off;
  int fan_in = L.d_in;
  for (int l = 0; l <= d.n_hidden; ++l) {
    const int o = l < d.n_hidden ? kHW : d.n_out;
    L.w_off[l] = p; p += (int64_t)o * fan_in;
    L.b_off[l] = p; p += o;
    fan_in = o;
  }
  L.params = p;
  L.wh_off = L.w_off[d.n_hidden];
  L.bh_off = L.b_off[d.n_hidden];
  return L;
}

bool hash_shape_supported(int nl, int nb, int nh);

int check_hash_desc(const ddf_hash_desc* d) {
  if (!d) return fail(DDF_ERR_INVALID_ARG, "desc is NULL");
  if (d->n_feat != 2) return fail(DDF_ERR_UNSUPPORTED, "n_feat must be 2");
  if (d->width != kHW) return fail(DDF_ERR_UNSUPPORTED, "width must be 64");
  if (d->n_hidden != kHMaxHidden) return fail(DDF_ERR_UNSUPPORTED, "n_hidden must be 2");
  if (d->n_out != 2) return fail(DDF_ERR_UNSUPPORTED, "n_out must be 2 (t, xi)");
  if (d->n_levels < 1 || d->n_levels > kHMaxLevels) return fail(DDF_ERR_UNSUPPORTED, "n_levels must be 1..24");
  if (d->log2_table < 4 || d->log2_table > 24) return fail(DDF_ERR_UNSUPPORTED, "log2_table must be 4..24");
  if (d->dir_bands < 0 || 2 * d->n_levels + 3 * (1 + 2 * d->dir_bands) > kHIn)
    return fail(DDF_ERR_UNSUPPORTED, "2 n_levels + 3 (1 + 2 dir_bands) must be <= 64");
  if (d->base_res < 1 || !(d->growth >= 1.f && d->growth <= 8.f) || !(d->box_half > 0.f))
    return fail(DDF_ERR_INVALID_ARG, "base_res, growth or box_half out of range");
  if (!hash_shape_supported(d->n_levels, d->dir_bands, d->n_hidden))
    return fail(DDF_ERR_UNSUPPORTED, "compiled shapes: 16 or 6 levels, 4 direction bands, 2 hidden layers");
  const double top = (double)d->base_res * pow((double)d->growth, (double)(d->n_levels - 1));
  if (!(top < 1.0e6)) return fail(DDF_ERR_UNSUPPORTED, "finest resolution must stay below 1e6");
  return DDF_OK;
}

// The MLP staged in LDS: every layer transposed (row i = the weights of input i into the 64
// outputs, zero rows past the input width), the heads row-major, the biases.
struct HashSmem {
  float wt[kHMaxHidden][kHIn][kHW];
  float b[kHMaxHidden][kHW];
  float wh[2][kHW];
  float bh[2];
};

__device__ __forceinline__ void stage_mlp(const HashLayout& L, const float* __restrict__ params, HashSmem& s) {
#pragma unroll
  for (int l = 0; l < kHMaxHidden; ++l) {   // static indices into the argument block
    if (l >= L.n_hidden) break;
    const int fan_in = l == 0 ? L.d_in : kHW;
    const float* W = params + L.w_off[l];
    for (int k = threadIdx.x; k < kHIn * kHW; k += blockDim.x) {
      const int i = k / kHW, j = k % kHW;
      s.wt[l][i][j] = i < fan_in ? W[(int64_t)j * fan_in + i] : 0.f;
    }
    for (int j = threadIdx.x; j < kHW; j += blockDim.x) s.b[l][j] = params[L.b_off[l] + j];
  }
  for (int k = threadIdx.x; k < 2 * kHW; k += blockDim.x) s.wh[k / kHW][k % kHW] = params[L.wh_off + k];
  if (threadIdx.x < 2) s.bh[threadIdx.x] = params[L.bh_off + threadIdx.x];
}

// The per-level lookup constants, staged in LDS so that no helper holds a reference to the
// kernel's argument block (which would force a private copy of it).
struct LevelTab {
  int res[kHMaxLevels];
  int dense[kHMaxLevels];
  int64_t off[kHMaxLevels];
  uint32_t tmask;
  float box_half;
};

__device__ __forceinline__ void stage_levels(const HashLayout& L, LevelTab& t) {
  if (threadIdx.x < kHMaxLevels) {
    t.res[threadIdx.x] = L.res[threadIdx.x];
    t.dense[threadIdx.x] = L.dense[threadIdx.x];
    t.off[threadIdx.x] = L.off[threadIdx.x];
  }
  if (threadIdx.x == 0) {
    t.tmask = L.tmask;
    t.box_half = L.box_half;
  }
}

// Cell of point p (unit cube) at level l: lower vertex c and weights w.
__device__ __forceinline__ void cell(float N, const float (&p)[3], uint32_t (&c)[3], float (&w)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float sv = p[a] * N;
    const float fl = fminf(floorf(sv), N - 1.f);
    w[a] = sv - fl;
    c[a] = (uint32_t)fl;
  }
}

// Table entry and trilinear weight of corner k (bit a of k: +1 along axis a).
__device__ __forceinline__ void corner(const LevelTab& L, int l, const uint32_t (&c)[3], const float (&w)[3], int k,
                              int64_t& entry, float& wt) {
  const uint32_t v0 = c[0] + (k & 1), v1 = c[1] + ((k >> 1) & 1), v2 = c[2] + ((k >> 2) & 1);
  const uint32_t n1 = (uint32_t)L.res[l] + 1u;
  const uint32_t idx = L.dense[l] ? v0 + n1 * (v1 + n1 * v2) : ((v0 ^ (v1 * kPrime1) ^ (v2 * kPrime2)) & L.tmask);
  entry = L.off[l] + idx;
  wt = ((k & 1) ? w[0] : 1.f - w[0]) * (((k >> 1) & 1) ? w[1] : 1.f - w[1]) * (((k >> 2) & 1) ? w[2] : 1.f - w[2]);
}

__device__ __forceinline__ void unit_point(const LevelTab& L, const float (&x)[3], float (&p)[3]) {
  const float inv = 0.5f / L.box_half;
#pragma unroll
  for (int a = 0; a < 3; ++a) p[a] = fminf(fmaxf((x[a] + L.box_half) * inv, 0.f), 1.f);
}

// h[j] += row[j] v for the 64 outputs (row: one input's weights, LDS).
__device__ __forceinline__ void axpy_row(const float* row, float v, float (&h)[kHW]) {
  const f32x4* r4 = reinterpret_cast<const f32x4*>(row);
#pragma unroll
  for (int q = 0; q < kHW / 4; ++q) {
    const f32x4 w4 = r4[q];
#pragma unroll
    for (int e = 0; e < 4; ++e) h[4 * q + e] = fmaf(w4[e], v, h[4 * q + e]);
  }
}

// The first layer's pre-activation of one ray, fused with the encoding: each input feature
// is added into h = b1 + W1 g as soon as it exists, so the 64-wide input vector is never held.
// Features in order: the trilinear lookup of every level (2 each), then the direction code
// [d, sin(pi 2^k d), cos(pi 2^k d)]_{k < NB}.  With `keep`, every feature is also stored to
// keep[i] (the backward pass's copy of the layer input, 64 floats per ray).  Two levels' gathers are in
// flight at a time.
template <int NL, int NB>
__device__ __forceinline__ void encode_layer1(const LevelTab& L, const HashSmem& s, const float* __restrict__ table,
                                     const float (&x)[3], const float (&dv)[3], float (&h)[kHW], float* keep) {
#pragma unroll
  for (int j = 0; j < kHW; ++j) h[j] = s.b[0][j];
  float p[3];
  unit_point(L, x, p);
  const float2* tab = reinterpret_cast<const float2*>(table);
  float f[2 * NL];   // the lookups first (all gathers in flight together), then the products
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    uint32_t c[3];
    float w[3];
    cell((float)L.res[l], p, c, w);
    float f0 = 0.f, f1 = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      int64_t e;
      float wt;
      corner(L, l, c, w, k, e, wt);
      const float2 t = tab[e];
      f0 = fmaf(wt, t.x, f0);
      f1 = fmaf(wt, t.y, f1);
    }
    f[2 * l] = f0;
    f[2 * l + 1] = f1;
    if ((l & 3) == 3) __builtin_amdgcn_sched_barrier(0);   // at most 4 levels of gathers in flight
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int i = 0; i < 2 * NL; ++i) {
    axpy_row(s.wt[0][i], f[i], h);
    if (keep) keep[i] = f[i];
    if ((i & 3) == 3) __builtin_amdgcn_sched_barrier(0);
  }
  constexpr int D0 = 2 * NL;
#pragma unroll
  for (int k = -1; k < NB; ++k)
#pragma unroll
    for (int part = 0; part < (k < 0 ? 1 : 2); ++part)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        float v;
        if (k < 0) {
          v = dv[a];
        } else {
          float sn, cs;
          sincospif(ldexpf(dv[a], k), &sn, &cs);
          v = part == 0 ? sn : cs;
        }
        const int i = k < 0 ? D0 + a : D0 + 3 + 6 * k + 3 * part + a;
        axpy_row(s.wt[0][i], v, h);
        if (keep) keep[i] = v;
        __builtin_amdgcn_sched_barrier(0);
      }
  if (keep) {
#pragma unroll
    for (int i = D0 + 3 * (1 + 2 * NB); i < kHIn; ++i) keep[i] = 0.f;
  }
}

// out = ReLU(b + W in) for a square hidden layer (weights transposed in LDS).
__device__ __forceinline__ void hidden_relu(const float (&wt)[kHIn][kHW], const float (&b)[kHW], const float (&in)[kHW],
                                   float (&out)[kHW]) {
#pragma unroll
  for (int j = 0; j < kHW; ++j) out[j] = b[j];
#pragma unroll
  for (int i = 0; i < kHW; ++i) {
    axpy_row(wt[i], in[i], out);
    if ((i & 3) == 3) __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int j = 0; j < kHW; ++j) out[j] = fmaxf(out[j], 0.f);
}

struct HashArgs {
  HashLayout L;
  const float* params;
  const float* rays;      // [6][n]
  int64_t n;
  int mode;               // 0: t, xi   1: logits
  float* out0;
  float* out1;
  // backward
  const float* dzt;
  const float* dzx;
  float* acts;            // [n_hidden + 1][R][64]: the input code, then each hidden layer's output
  float* deltas;          // [n_hidden][R][64]: dL/da of each hidden layer
  float* gtab;            // table gradient [entries][2] (atomics)
  int64_t R;
  const __half* table16;  // float16 copy of the table for the reduced-precision lookups
};

template <int NL, int NB, int NH>
__global__ __launch_bounds__(kHT) void hash_fwd_kernel(HashArgs a) {
  __shared__ __attribute__((aligned(16))) HashSmem s;
  __shared__ LevelTab lt;
  stage_mlp(a.L, a.params, s);
  stage_levels(a.L, lt);
  __syncthreads();
  // one ray per thread and no loop over rays: the weights read from LDS are then not
  // loop-invariant, so they are never hoisted into registers
  {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n) return;
    float x[3], dv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) { x[c] = a.rays[c * a.n + r]; dv[c] = a.rays[(3 + c) * a.n + r]; }
    float h[kHW], h2[kHW];
    encode_layer1<NL, NB>(lt, s, a.params, x, dv, h2, nullptr);
#pragma unroll
    for (int j = 0; j < kHW; ++j) h[j] = fmaxf(h2[j], 0.f);
#pragma unroll
    for (int l = 1; l < NH; ++l) {
      hidden_relu(s.wt[l], s.b[l], h, h2);
#pragma unroll
      for (int j = 0; j < kHW; ++j) h[j] = h2[j];
    }
    float z0 = s.bh[0], z1 = s.bh[1];
#pragma unroll
    for (int j = 0; j < kHW; ++j) {
      z0 = fmaf(s.wh[0][j], h[j], z0);
      z1 = fmaf(s.wh[1][j], h[j], z1);
    }
    if (a.mode == 0) {
      a.out0[r] = softplusf_(z0);
      a.out1[r] = sigmoidf_(z1);
    } else {
      a.out0[r] = z0;
      a.out1[r] = z1;
    }
  }
}

// ---- the two-pass query: the lookups with level groups pinned to XCDs, then the MLP
// The table's levels form 8 groups of at most 2.  Workgroups are dispatched to the 8 XCDs
// round-robin by index, so a lookup workgroup with index = g (mod 8) runs on XCD g and reads
// group g only: each XCD's L2 holds its own group's levels instead of all of them (48 MB of
// hashed levels against 4 MB of L2 per XCD).  The 16-level grouping pairs each of the four
// small dense levels with one hashed level and the remaining eight hashed levels two by two.
// Correctness does not depend on the placement, only the hit rate does.
constexpr int kHGroups = 8;

template <int NL>
__device__ __forceinline__ int grp_level(int g, int slot) {
  if (NL == 16) return g < 4 ? g + 4 * slot : 8 + 2 * (g - 4) + slot;
  return (slot == 0 && g < NL) ? g : -1;
}

// G[g][r] (16 bytes): the features of group g's levels for ray r, in slot order.
// Table entries (2 features) of either storage type, as float2: one entry, or the pair at
// entries i and i + 1 in one load (16 bytes for float32, 8 for float16; 4-byte aligned).
__device__ __forceinline__ float2 entry1(const float* b, uint32_t i) {
  return *reinterpret_cast<const float2*>(b + 2 * (size_t)i);
}
__device__ __forceinline__ void entry2(const float* b, uint32_t i, float2& e0, float2& e1) {
  const f32x4 q = *reinterpret_cast<const f32x4*>(b + 2 * (size_t)i);
  e0 = float2{q[0], q[1]};
  e1 = float2{q[2], q[3]};
}
__device__ __forceinline__ float2 entry1(const __half* b, uint32_t i) {
  return __half22float2(*reinterpret_cast<const __half2*>(b + 2 * (size_t)i));
}
__device__ __forceinline__ void entry2(const __half* b, uint32_t i, float2& e0, float2& e1) {
  const uint2 q = *reinterpret_cast<const uint2*>(b + 2 * (size_t)i);
  e0 = __half22float2(__builtin_bit_cast(__half2, q.x));
  e1 = __half22float2(__builtin_bit_cast(__half2, q.y));
}

// G[g][r] (16 bytes): the features of group g's levels for ray r, in slot order.  TE: the
// table's storage type (float, or the float16 copy of the reduced-precision query).
template <int NL, typename TE>
__global__ __launch_bounds__(kHT) void hash_pos_kernel(HashArgs a, float* G) {
  __shared__ LevelTab lt;
  stage_levels(a.L, lt);
  __syncthreads();
  const int g = blockIdx.x % kHGroups;
  const int64_t r = (int64_t)(blockIdx.x / kHGroups) * blockDim.x + threadIdx.x;
  if (r >= a.n) return;
  float x[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) x[c] = a.rays[c * a.n + r];
  float p[3];
  unit_point(lt, x, p);
  const TE* table;
  if constexpr (sizeof(TE) == 4) table = reinterpret_cast<const TE*>(a.params);
  else table = reinterpret_cast<const TE*>(a.table16);
  float o[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int slot = 0; slot < 2; ++slot) {
    const int l = grp_level<NL>(g, slot);
    if (l < 0) continue;
    uint32_t c[3];
    float w[3];
    cell((float)lt.res[l], p, c, w);
    const uint32_t n1 = (uint32_t)lt.res[l] + 1u;
    const TE* base = table + 2 * lt.off[l];
    const bool dense = lt.dense[l];
    float f0 = 0.f, f1 = 0.f;
    // the 8 corners as 4 pairs along x, (v0, v1, v2) and (v0 + 1, v1, v2): densely indexed,
    // the pair is contiguous; hashed, x enters the hash with multiplier 1, so for an even v0
    // the pair is the aligned {i & ~1, i | 1} and only an odd v0 needs a second load.
    // Products and sums in the same order as corner-by-corner.
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const uint32_t v0 = c[0], v1 = c[1] + (m & 1), v2 = c[2] + (m >> 1);
      const float wy = (m & 1) ? w[1] : 1.f - w[1], wz = (m >> 1) ? w[2] : 1.f - w[2];
      const float wa = ((1.f - w[0]) * wy) * wz, wb = (w[0] * wy) * wz;
      float2 ca, cb;
      if (dense) {
        entry2(base, v0 + n1 * (v1 + n1 * v2), ca, cb);
      } else {
        const uint32_t h = (v1 * kPrime1) ^ (v2 * kPrime2);
        const uint32_t i0 = (v0 ^ h) & lt.tmask;
        float2 e0, e1;
        entry2(base, i0 & ~1u, e0, e1);
        const bool odd = i0 & 1u;
        ca = odd ? e1 : e0;
        if (v0 & 1u)
          cb = entry1(base, ((v0 + 1u) ^ h) & lt.tmask);
        else
          cb = odd ? e0 : e1;
      }
      f0 = fmaf(wa, ca.x, f0);
      f1 = fmaf(wa, ca.y, f1);
      f0 = fmaf(wb, cb.x, f0);
      f1 = fmaf(wb, cb.y, f1);
    }
    o[2 * slot] = f0;
    o[2 * slot + 1] = f1;
  }
  reinterpret_cast<f32x4*>(G)[g * a.n + r] = f32x4{o[0], o[1], o[2], o[3]};
}

// The float16 copy of the table (round to nearest even).
__global__ void table_to_f16_kernel(const float* __restrict__ src, int64_t n, __half* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = __float2half_rn(src[i]);
}

// The MLP of the two-pass query on the matrix cores (fp32 32x32x2 MFMA), with the rays as the
// product's columns: C[neuron][ray] = sum_k W[neuron][k] X[ray][k].  At step s lane l supplies
// W[n0 + l % 32][k(s, l / 32)] and X[ray0 + l % 32][k(s, l / 32)] and holds neurons
// n0 + acc_row(v, l) of ray ray0 + l % 32.  After bias and ReLU these are exactly the values
// lane l supplies at step s = 16 ct + v of the next layer when that layer takes its inputs in
// the order k(s, p) = 32 (s / 16) + 8 ((s % 16) / 4) + 4 p + s % 4 (the weights are staged in
// that order), so the hidden activations never leave the registers.  The first layer takes
// its inputs in the natural order k(s, p) = 2 s + p.
struct HashFrag {
  f32x4 w1[2][8][64];     // [neuron tile][step / 4][lane] -> steps 4j .. 4j + 3
  f32x4 w2[2][8][64];
  float b1[kHW], b2[kHW];
  float wh[2][kHW];
  float bh[2];
};

__device__ __forceinline__ int hid_k(int s, int p) { return 32 * (s >> 4) + 8 * ((s & 15) >> 2) + 4 * p + (s & 3); }

__device__ __forceinline__ void stage_frag(const HashLayout& L, const float* __restrict__ params, HashFrag& f) {
  const float* W1 = params + L.w_off[0];
  const float* W2 = params + L.w_off[1];
  float* w1 = reinterpret_cast<float*>(f.w1);
  float* w2 = reinterpret_cast<float*>(f.w2);
  for (int e = threadIdx.x; e < 2 * 32 * 64; e += blockDim.x) {
    const int ct = e >> 11, st = (e >> 6) & 31, ln = e & 63;
    const int n = ct * 32 + (ln & 31), p = ln >> 5;
    const int k1 = 2 * st + p;
    const int dst = ((ct * 8 + (st >> 2)) * 64 + ln) * 4 + (st & 3);
    w1[dst] = k1 < L.d_in ? W1[n * L.d_in + k1] : 0.f;
    w2[dst] = W2[n * kHW + hid_k(st, p)];
  }
  for (int j = threadIdx.x; j < kHW; j += blockDim.x) {
    f.b1[j] = params[L.b_off[0] + j];
    f.b2[j] = params[L.b_off[1] + j];
    f.wh[0][j] = params[L.wh_off + j];
    f.wh[1][j] = params[L.wh_off + kHW + j];
  }
  if (threadIdx.x < 2) f.bh[threadIdx.x] = params[L.bh_off + threadIdx.x];
}

// One layer: acc[rt][ct] = b + W X^T over the 32 steps (wf: the layer's staged fragments).
__device__ __forceinline__ void frag_layer(const f32x4 (&wf)[2][8][64], const float* b, const float (&x)[2][32],
                                           int lane, f32x16 (&acc)[2][2]) {
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float bv = b[ct * 32 + acc_row(v, lane)];
      acc[0][ct][v] = bv;
      acc[1][ct][v] = bv;
    }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const f32x4 wa = wf[0][j][lane], wb = wf[1][j][lane];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        acc[rt][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(wa[q], x[rt][4 * j + q], acc[rt][0], 0, 0, 0);
        acc[rt][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(wb[q], x[rt][4 * j + q], acc[rt][1], 0, 0, 0);
      }
  }
}

// Each wave takes 64 rays (two 32-ray column tiles); lane l works on rays l % 32 of both tiles
// and, of each layer's inputs, on the half with parity l / 32.
template <int NL, int NB>
__global__ __launch_bounds__(kHT) void hash_mlp_kernel(HashArgs a, const float* G) {
  __shared__ __attribute__((aligned(16))) HashFrag f;
  stage_frag(a.L, a.params, f);
  __syncthreads();
  const int lane = threadIdx.x & 63, p = lane >> 5;
  const int64_t ray0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
  if (ray0 >= a.n) return;   // whole waves only
  constexpr int ND = 3 * (1 + 2 * NB);
  float x[2][32];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    // rays past n repeat the last ray and are not stored
    const int64_t r = min(ray0 + rt * 32 + (lane & 31), a.n - 1);
#pragma unroll
    for (int g = 0; g < kHGroups; ++g) {
      if (grp_level<NL>(g, 0) < 0) continue;
      const f32x4 v = reinterpret_cast<const f32x4*>(G)[g * a.n + r];
#pragma unroll
      for (int slot = 0; slot < 2; ++slot) {
        const int l = grp_level<NL>(g, slot);
        if (l < 0) continue;
        x[rt][l] = p ? v[2 * slot + 1] : v[2 * slot];
      }
    }
    float dv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) dv[c] = a.rays[(3 + c) * a.n + r];
    float df[ND + 1];
#pragma unroll
    for (int c = 0; c < 3; ++c) df[c] = dv[c];
#pragma unroll
    for (int k = 0; k < NB; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float sn, cs;
        sincospif(ldexpf(dv[c], k), &sn, &cs);
        df[3 + 6 * k + c] = sn;
        df[6 + 6 * k + c] = cs;
      }
    df[ND] = 0.f;
#pragma unroll
    for (int st = NL; st < 32; ++st) {
      const int i0 = 2 * (st - NL);
      const float v0 = i0 < ND ? df[i0] : 0.f, v1 = i0 + 1 < ND ? df[i0 + 1] : 0.f;
      x[rt][st] = p ? v1 : v0;
    }
  }
  f32x16 acc[2][2];
  frag_layer(f.w1, f.b1, x, lane, acc);
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int v = 0; v < 16; ++v) x[rt][16 * ct + v] = fmaxf(acc[rt][ct][v], 0.f);
  frag_layer(f.w2, f.b2, x, lane, acc);
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    float z0 = 0.f, z1 = 0.f;
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int n = ct * 32 + acc_row(v, lane);
        const float hv = fmaxf(acc[rt][ct][v], 0.f);
        z0 = fmaf(f.wh[0][n], hv, z0);
        z1 = fmaf(f.wh[1][n], hv, z1);
      }
    z0 = z0 + __shfl_xor(z0, 32) + f.bh[0];
    z1 = z1 + __shfl_xor(z1, 32) + f.bh[1];
    const int64_t r = ray0 + rt * 32 + (lane & 31);
    if (p == rt && r < a.n) {
      if (a.mode == 0) {
        a.out0[r] = softplusf_(z0);
        a.out1[r] = sigmoidf_(z1);
      } else {
        a.out0[r] = z0;
        a.out1[r] = z1;
      }
    }
  }
}

// ---- training: one simple kernel per stage, activations in memory ([R][64] per layer)

// The input code of every ray (rows n .. R - 1: the code of the box centre, zero direction).
// kESub lanes share a ray: lane s looks up the levels l = s (mod kESub) and forms the
// direction bands k = s (mod kESub); lane 0 also writes the raw direction and the zero
// padding.  Each feature is computed as with one lane per ray (bit-identical); the split
// only spreads a training batch over more workgroups.
constexpr int kESub = 4;
template <int NL, int NB>
__global__ __launch_bounds__(kHT) void hash_encode_kernel(HashArgs a) {
  __shared__ LevelTab lt;
  stage_levels(a.L, lt);
  __syncthreads();
  const int s = threadIdx.x % kESub;
  const int64_t r = (int64_t)blockIdx.x * (kHT / kESub) + threadIdx.x / kESub;
  if (r >= a.R) return;
  float x[3] = {0.f, 0.f, 0.f}, dv[3] = {0.f, 0.f, 0.f};
  if (r < a.n) {
#pragma unroll
    for (int c = 0; c < 3; ++c) { x[c] = a.rays[c * a.n + r]; dv[c] = a.rays[(3 + c) * a.n + r]; }
  }
  float p[3];
  unit_point(lt, x, p);
  const float2* tab = reinterpret_cast<const float2*>(a.params);
  float* dst = a.acts + r * kHIn;
#pragma unroll
  for (int j = 0; j < (NL + kESub - 1) / kESub; ++j) {
    const int l = s + kESub * j;
    if (l < NL) {
      uint32_t c[3];
      float w[3];
      cell((float)lt.res[l], p, c, w);
      float f0 = 0.f, f1 = 0.f;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        int64_t e;
        float wt;
        corner(lt, l, c, w, k, e, wt);
        const float2 t = tab[e];
        f0 = fmaf(wt, t.x, f0);
        f1 = fmaf(wt, t.y, f1);
      }
      *reinterpret_cast<float2*>(dst + 2 * l) = make_float2(f0, f1);
    }
  }
  constexpr int D0 = 2 * NL;
  if (s == 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) dst[D0 + q] = dv[q];
#pragma unroll
    for (int i = D0 + 3 * (1 + 2 * NB); i < kHIn; ++i) dst[i] = 0.f;
  }
#pragma unroll
  for (int j = 0; j < (NB + kESub - 1) / kESub; ++j) {
    const int k = s + kESub * j;
    if (k < NB) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        float sn, cs;
        sincospif(ldexpf(dv[q], k), &sn, &cs);
        dst[D0 + 3 + 6 * k + q] = sn;
        dst[D0 + 6 + 6 * k + q] = cs;
      }
    }
  }
}

// h[j] += row[j] v, j < N (row: N consecutive weights in LDS, 16-byte aligned when N % 4 == 0).
template <int N>
__device__ __forceinline__ void axpy_n(const float* row, float v, float (&h)[N]) {
  if constexpr (N % 4 == 0) {
    const f32x4* r4 = reinterpret_cast<const f32x4*>(row);
#pragma unroll
    for (int q = 0; q < N / 4; ++q) {
      const f32x4 w4 = r4[q];
#pragma unroll
      for (int e = 0; e < 4; ++e) h[4 * q + e] = fmaf(w4[e], v, h[4 * q + e]);
    }
  } else {
#pragma unroll
    for (int j = 0; j < N; ++j) h[j] = fmaf(row[j], v, h[j]);
  }
}

// The [64][64] LDS image of a layer's weights, element (u, v) = W[row(u, v)][col(u, v)] or 0
// outside [O][fan_in]; every thread's 16 loads are issued before its LDS writes.
template <bool kTransposed>
__device__ __forceinline__ void stage_weights(const float* W, int O, int fan_in, float (*dst)[kHW]) {
  static_assert(kHIn == kHW && (kHIn * kHW) % kHT == 0, "square 64 x 64 image, whole rounds");
  constexpr int kRounds = kHIn * kHW / kHT;
  float v[kRounds];
#pragma unroll
  for (int it = 0; it < kRounds; ++it) {
    const int k = it * kHT + (int)threadIdx.x;
    const int u = k / kHW, c = k % kHW;
    const int o = kTransposed ? c : u, i = kTransposed ? u : c;
    v[it] = (i < fan_in && o < O) ? W[(int64_t)o * fan_in + i] : 0.f;
  }
#pragma unroll
  for (int it = 0; it < kRounds; ++it) {
    const int k = it * kHT + (int)threadIdx.x;
    dst[k / kHW][k % kHW] = v[it];
  }
}

// out[r][o] = act(b[o] + sum_i W[o][i] in[r][i]) for O <= 64 outputs (W [O][fan_in], master
// layout); act = ReLU, or none for the heads, whose two logits go to out0 / out1.  S lanes share
// a ray, lane s computing outputs s OL .. s OL + OL - 1, each summed over i in increasing
// order: the split changes no rounding, it only spreads a batch over S times the workgroups.
// The heads run with S = 1, OL = 2 (only the two logits are formed).
template <int S, int OL>
__global__ __launch_bounds__(kHT) void dense_fwd_kernel(const float* in, const float* W, const float* b, int O,
                                                        int fan_in, int64_t R, int relu, float* out, float* out0,
                                                        float* out1) {
  static_assert(S * OL <= kHW && kHT % S == 0, "lane split");
  __shared__ __attribute__((aligned(16))) float wt[kHIn][kHW];   // transposed, zero padded
  __shared__ float bs[kHW];
  stage_weights<true>(W, O, fan_in, wt);
  for (int o = threadIdx.x; o < kHW; o += blockDim.x) bs[o] = o < O ? b[o] : 0.f;
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * (kHT / S) + threadIdx.x / S;
  if (r >= R) return;
  const int o0 = (int)(threadIdx.x % S) * OL;
  float acc[OL];
#pragma unroll
  for (int j = 0; j < OL; ++j) acc[j] = bs[o0 + j];
  const f32x4* src = reinterpret_cast<const f32x4*>(in + r * kHIn);
#pragma unroll 2
  for (int q = 0; q < kHIn / 4; ++q) {   // (fully unrolled, the weight reads all hoist: 272 VGPRs)
    const f32x4 x4 = src[q];
#pragma unroll
    for (int e = 0; e < 4; ++e) axpy_n<OL>(&wt[4 * q + e][o0], x4[e], acc);
  }
  if (out) {
    f32x4* dst = reinterpret_cast<f32x4*>(out + r * kHW + o0);
#pragma unroll
    for (int m = 0; m < OL / 4; ++m) {
      f32x4 y;
#pragma unroll
      for (int e = 0; e < 4; ++e) y[e] = relu ? fmaxf(acc[4 * m + e], 0.f) : acc[4 * m + e];
      dst[m] = y;
    }
  } else {
    out0[r] = acc[0];
    out1[r] = acc[1];
  }
}

// d_in[r][i] = mask(in[r][i] > 0) sum_o W[o][i] d_out[r][o] for the hidden layers (W [O][fan_in]
// master layout, d_out [R][64]); `mask_src` null: no mask.  With dz0 / dz1 set, d_out is the
// pair of logit gradients instead (the heads).  S lanes share a ray, lane s forming inputs
// s IL .. s IL + IL - 1, each summed over o in increasing order (no rounding changes).
template <int S, int IL>
__global__ __launch_bounds__(kHT) void dense_bwd_kernel(const float* d_out, const float* dz0, const float* dz1,
                                                        const float* W, int O, int fan_in, int64_t R,
                                                        const float* mask_src, float* d_in) {
  static_assert(S * IL == kHIn && IL % 4 == 0 && kHT % S == 0, "lane split");
  __shared__ __attribute__((aligned(16))) float wr[kHW][kHIn];   // rows of W, zero padded
  stage_weights<false>(W, O, fan_in, wr);
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * (kHT / S) + threadIdx.x / S;
  if (r >= R) return;
  const int i0 = (int)(threadIdx.x % S) * IL;
  float acc[IL];
#pragma unroll
  for (int j = 0; j < IL; ++j) acc[j] = 0.f;
  if (dz0) {
    axpy_n<IL>(&wr[0][i0], dz0[r], acc);
    axpy_n<IL>(&wr[1][i0], dz1[r], acc);
  } else {
    const f32x4* src = reinterpret_cast<const f32x4*>(d_out + r * kHW);
    for (int q = 0; q < kHW / 4; ++q) {
      const f32x4 d4 = src[q];
#pragma unroll
      for (int e = 0; e < 4; ++e) axpy_n<IL>(&wr[4 * q + e][i0], d4[e], acc);
    }
  }
  if (mask_src) {
    const f32x4* m4 = reinterpret_cast<const f32x4*>(mask_src + r * kHIn + i0);
#pragma unroll
    for (int q = 0; q < IL / 4; ++q) {
      const f32x4 h4 = m4[q];
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[4 * q + e] = h4[e] > 0.f ? acc[4 * q + e] : 0.f;
    }
  }
  f32x4* dst = reinterpret_cast<f32x4*>(d_in + r * kHIn + i0);
#pragma unroll
  for (int q = 0; q < IL / 4; ++q) dst[q] = f32x4{acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]};
}

// The position-code gradient dg [R][64] (first 2 NL entries) of every live ray scattered to
// the 8 corners of every level with the lookup weights (float atomics).  Like the lookups,
// the work goes out as 8 x (ray blocks) workgroups, workgroup index g (mod 8) taking level
// group g: all updates of a group's table entries then come from one XCD.  Four lanes share
// a ray, lane s of the four taking the corners at x offset s / 2 and feature s % 2: in each
// atomic instruction the lanes of a ray address the two features of the two x-neighbour
// corners, 16 contiguous bytes on the dense levels and on hashed levels when the lower
// corner's x is even (x enters the hash with multiplier 1), so the updates of one ray leave
// as one request per line instead of four.
constexpr int kHSub = 4;                  // lanes per ray in the scatter
template <int NL>
__global__ __launch_bounds__(kHT) void hash_scatter_kernel(HashArgs a, const float* dg) {
  __shared__ LevelTab lt;
  stage_levels(a.L, lt);
  __syncthreads();
  const int g = blockIdx.x % kHGroups;
  const int sub = threadIdx.x % kHSub;
  const int64_t r = (int64_t)(blockIdx.x / kHGroups) * (kHT / kHSub) + threadIdx.x / kHSub;
  if (r >= a.n) return;
  float x[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) x[c] = a.rays[c * a.n + r];
  float p[3];
  unit_point(lt, x, p);
  // the lane's feature, and the low corner bits it owns (the rest run in the loop)
  const int f = sub & 1, klo = sub >> 1;
  constexpr int kLoBits = kHSub == 2 ? 0 : (kHSub == 4 ? 1 : 2);
#pragma unroll
  for (int slot = 0; slot < 2; ++slot) {
    const int l = grp_level<NL>(g, slot);
    if (l < 0) continue;
    const float gl = dg[r * kHIn + 2 * l + f];
    uint32_t c[3];
    float w[3];
    cell((float)lt.res[l], p, c, w);
#pragma unroll
    for (int j = 0; j < (8 >> kLoBits); ++j) {
      int64_t e;
      float wt;
      corner(lt, l, c, w, klo | (j << kLoBits), e, wt);
      atomicAdd(a.gtab + 2 * e + f, wt * gl);
    }
  }
}

// part[blk][o 64 + i] = sum over the block's kHRC rays of d[r][o] a[r][i]; part[blk][64 O + o]
// = sum of d[r][o] (the bias), for ray-major d [R][ldd] (first O columns, O = 64 or 1) and
// a [R][64].  Every sum runs over the block's rays in increasing order.  Thread t owns row
// o = t / 4 and columns 16 (t % 4) .. 16 (t % 4) + 15: one d read and four 16-byte a reads
// per 16 products; the threads with t % 4 == 0 also form the bias sum.
__global__ __launch_bounds__(kHT) void outer_reduce_kernel(const float* d, int ldd, const float* a, int O,
                                                           float* part) {
  static_assert(kHT == 4 * kHW && kHIn == 64 && kHW == 64, "thread t: row t / 4, 16 columns");
  __shared__ float sd[kHRC][kHW + 1];
  __shared__ __attribute__((aligned(16))) float sa[kHRC][kHIn + 4];
  const int64_t r0 = (int64_t)blockIdx.x * kHRC;
  const int t = threadIdx.x;
  {
    // the block's a rows are one contiguous kHRC x 64 slab: 16-byte loads, all issued first
    constexpr int kA = kHRC * kHIn / 4 / kHT;
    f32x4 v[kA];
    const f32x4* src = reinterpret_cast<const f32x4*>(a + r0 * kHIn);
#pragma unroll
    for (int u = 0; u < kA; ++u) v[u] = src[u * kHT + t];
#pragma unroll
    for (int u = 0; u < kA; ++u) {
      const int e = (u * kHT + t) * 4;
      *reinterpret_cast<f32x4*>(&sa[e / kHIn][e % kHIn]) = v[u];
    }
  }
  {
    constexpr int kD = kHRC * kHW / kHT;
    float v[kD];
#pragma unroll
    for (int u = 0; u < kD; ++u) {
      const int e = u * kHT + t, r = e / kHW, o = e % kHW;
      v[u] = o < O ? d[(r0 + r) * ldd + o] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < kD; ++u) {
      const int e = u * kHT + t;
      sd[e / kHW][e % kHW] = v[u];
    }
  }
  __syncthreads();
  const int o = t >> 2, i0 = (t & 3) * 16;
  if (o >= O) return;
  float acc[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.f;
  float bsum = 0.f;
  for (int r = 0; r < kHRC; ++r) {
    const float dv = sd[r][o];
    const f32x4* a4 = reinterpret_cast<const f32x4*>(&sa[r][i0]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f32x4 x = a4[q];
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[4 * q + e] = fmaf(dv, x[e], acc[4 * q + e]);
    }
    bsum += dv;
  }
  float* dst = part + (int64_t)blockIdx.x * (O * kHIn + O);
#pragma unroll
  for (int j = 0; j < 16; ++j) dst[o * kHIn + i0 + j] = acc[j];
  if ((t & 3) == 0) dst[O * kHIn + o] = bsum;
}

// v[k] = sum over blocks b of part[b][k], in a fixed order: eight running sums over
// b = j (mod 8), each in increasing b, then a pairwise tree of the eight.  Thread (j, k) runs
// chain j of output k (its loads independent of one another); a block of 256 threads covers
// 32 outputs x 8 chains.  The sums go straight to the master layout: k = 64 o + i to
// w[o fan_in + i] (the padding columns i >= fan_in are dropped), k = 64 O + o to b[o].
__global__ __launch_bounds__(256) void sum_parts_kernel(const float* part, int nblk, int O, int fan_in, float* w,
                                                        float* b) {
  const int stride = O * kHIn + O;
  __shared__ float s[8][33];
  const int kl = threadIdx.x & 31, j = threadIdx.x >> 5;
  const int k = blockIdx.x * 32 + kl;
  float acc = 0.f;
  if (k < stride) {
#pragma unroll 8
    for (int b = j; b < nblk; b += 8) acc += part[(int64_t)b * stride + k];
  }
  s[j][kl] = acc;
  __syncthreads();
  if (j == 0 && k < stride) {
    const float v = ((s[0][kl] + s[1][kl]) + (s[2][kl] + s[3][kl])) + ((s[4][kl] + s[5][kl]) + (s[6][kl] + s[7][kl]));
    if (k >= O * kHIn)
      b[k - O * kHIn] = v;
    else if (k % kHIn < fan_in)
      w[(k / kHIn) * fan_in + k % kHIn] = v;
  }
}

__global__ void fill_zero_kernel(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0.f;
}

struct HashWs {
  int64_t R;
  int64_t zt, zx, dzt, dzx, lossp, scal, acts, deltas, part, grad, total;
};

HashWs hash_ws(const HashLayout& L, int64_t batch) {
  HashWs w{};
  w.R = (batch + kHRC - 1) / kHRC * kHRC;
  int64_t off = 0;
  auto take = [&](int64_t bytes) { const int64_t o = off; off = align256(off + bytes); return o; };
  w.zt = take(4 * w.R); w.zx = take(4 * w.R); w.dzt = take(4 * w.R); w.dzx = take(4 * w.R);
  w.lossp = take(4ll * loss_scratch_floats());
  w.scal = take(64);
  w.acts = take(4ll * 3 * kHIn * w.R);     // G, H1, H2
  w.deltas = take(4ll * 3 * kHIn * w.R);   // D2, D1, DG
  w.part = take(4ll * (w.R / kHRC) * (kHW * kHIn + kHW));
  w.grad = take(4 * L.params);
  w.total = off;
  return w;
}

// Encodings with a compiled kernel: (levels, direction bands).
bool hash_shape_supported(int nl, int nb, int nh) { return (nl == 16 || nl == 6) && nb == 4 && nh == 2; }

// G == nullptr: the fused one-kernel query; else the two-pass query through G
// (kHGroups x n x 16 bytes).
int run_hash_forward(const HashLayout& L, const float* params, const float* rays, int64_t n, int mode, float* o0,
                     float* o1, float* G, hipStream_t st, const __half* table16 = nullptr) {
  HashArgs a{};
  a.L = L; a.params = params; a.rays = rays; a.n = n; a.mode = mode; a.out0 = o0; a.out1 = o1;
  a.table16 = table16;
  const unsigned blocks = (unsigned)((n + kHT - 1) / kHT);
  if (G == nullptr) {
    if (L.n_levels == 16)
      hash_fwd_kernel<16, 4, 2><<<blocks, kHT, 0, st>>>(a);
    else
      hash_fwd_kernel<6, 4, 2><<<blocks, kHT, 0, st>>>(a);
  } else if (L.n_levels == 16) {
    if (table16)
      hash_pos_kernel<16, __half><<<blocks * kHGroups, kHT, 0, st>>>(a, G);
    else
      hash_pos_kernel<16, float><<<blocks * kHGroups, kHT, 0, st>>>(a, G);
    hash_mlp_kernel<16, 4><<<blocks, kHT, 0, st>>>(a, G);
  } else {
    if (table16)
      hash_pos_kernel<6, __half><<<blocks * kHGroups, kHT, 0, st>>>(a, G);
    else
      hash_pos_kernel<6, float><<<blocks * kHGroups, kHT, 0, st>>>(a, G);
    hash_mlp_kernel<6, 4><<<blocks, kHT, 0, st>>>(a, G);
  }
  return hip_status(hipGetLastError(), "hash forward launch");
}

// The training pass after the forward (stages in memory, [R][64] per layer, R a multiple of
// 64): G = code, H1, H2; D2, D1, DG the deltas and the code gradient.
int run_hash_encode(const HashArgs& a, hipStream_t st) {
  constexpr int rays_per_block = kHT / kESub;
  const unsigned blocks = (unsigned)((a.R + rays_per_block - 1) / rays_per_block);
  if (a.L.n_levels == 16)
    hash_encode_kernel<16, 4><<<blocks, kHT, 0, st>>>(a);
  else
    hash_encode_kernel<6, 4><<<blocks, kHT, 0, st>>>(a);
  return hip_status(hipGetLastError(), "hash encode launch");
}

int run_hash_scatter(const HashArgs& a, const float* dg, hipStream_t st) {
  constexpr int rays_per_block = kHT / kHSub;
  const unsigned blocks = (unsigned)((a.n + rays_per_block - 1) / rays_per_block) * kHGroups;
  if (a.L.n_levels == 16)
    hash_scatter_kernel<16><<<blocks, kHT, 0, st>>>(a, dg);
  else
    hash_scatter_kernel<6><<<blocks, kHT, 0, st>>>(a, dg);
  return hip_status(hipGetLastError(), "hash scatter launch");
}

}  // namespace

}  // namespace ddf

namespace ddf {

// The allocation-free two-pass query's workspace: one array in the library's code object,
// [kHGroups][kHashStaticRays][4] floats (64 MiB), which every GPU the library runs on holds until
// the process ends.  Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address): each device's address comes from hipGetSymbolAddress, taken
// once per device with that device current.
constexpr int64_t kHashStaticRays = 1 << 19;
static __device__ __align__(256) float4 hash_scratch[kHGroups * kHashStaticRays];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];   // per device ordinal; null until first looked up

// The device address of hash_scratch on the current device, looked up on the first call there.
static int hash_scratch_ptr(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(DDF_ERR_UNSUPPORTED, "device ordinal %d beyond 63", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(hash_scratch));
    if (e != hipSuccess) return hip_status(e, "hipGetSymbolAddress(hash_scratch)");
    if (!p) return fail(DDF_ERR_HIP, "hipGetSymbolAddress(hash_scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DDF_OK;
}

}  // namespace ddf

using namespace ddf;

extern "C" {

size_t ddf_hash_param_count(const ddf_hash_desc* d) {
  if (check_hash_desc(d) != DDF_OK) return 0;
  return (size_t)make_hash_layout(*d).params;
}

int ddf_hash_level(const ddf_hash_desc* d, int32_t level, int32_t* resolution, int64_t* entries, int64_t* offset,
                   int32_t* hashed) {
  int rc;
  if ((rc = check_hash_desc(d))) return rc;
  if (level < 0 || level >= d->n_levels) return fail(DDF_ERR_INVALID_ARG, "level %d out of range", level);
  const HashLayout L = make_hash_layout(*d);
  const int64_t T = 1ll << d->log2_table;
  if (resolution) *resolution = L.res[level];
  if (entries) *entries = L.dense[level] ? (int64_t)(L.res[level] + 1) * (L.res[level] + 1) * (L.res[level] + 1) : T;
  if (offset) *offset = L.off[level];
  if (hashed) *hashed = !L.dense[level];
  return DDF_OK;
}

size_t ddf_hash_query_workspace_bytes(const ddf_hash_desc* d, int64_t n) {
  if (check_hash_desc(d) != DDF_OK || n < 0) return 0;
  return (size_t)n * kHGroups * 16;
}

int ddf_hash_query(const ddf_hash_desc* d, const float* params, const float* rays, int64_t n, float* t, float* xi,
                   void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_hash_desc(d))) return rc;
  if (n < 0 || n > (int64_t)INT32_MAX) return fail(DDF_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (n == 0) return DDF_OK;
  if ((rc = check_ptr(params, "params")) || (rc = check_ptr(rays, "rays")) || (rc = check_ptr(t, "t")) ||
      (rc = check_ptr(xi, "xi")))
    return rc;
  if (ws != nullptr) {
    if ((rc = check_ptr(ws, "ws"))) return rc;
    if (ws_bytes < (size_t)n * kHGroups * 16)
      return fail(DDF_ERR_INVALID_ARG, "workspace %zu bytes < %zu", ws_bytes, (size_t)n * kHGroups * 16);
  }
  g_err_clear();
  return run_hash_forward(make_hash_layout(*d), params, rays, n, 0, t, xi, static_cast<float*>(ws),
                          (hipStream_t)stream);
}

int64_t ddf_hash_query_static_max_rays(void) { return kHashStaticRays; }

int ddf_hash_query_static(const ddf_hash_desc* d, const float* params, const float* rays, int64_t n, float* t,
                          float* xi, void* stream) {
  int rc;
  if ((rc = check_hash_desc(d))) return rc;
  if (n < 0 || n > kHashStaticRays)
    return fail(DDF_ERR_INVALID_ARG, "n = %lld outside 0..%lld (the static workspace's capacity)", (long long)n,
                (long long)kHashStaticRays);
  if (n == 0) return DDF_OK;
  if ((rc = check_ptr(params, "params")) || (rc = check_ptr(rays, "rays")) || (rc = check_ptr(t, "t")) ||
      (rc = check_ptr(xi, "xi")))
    return rc;
  void* ws = nullptr;
  if ((rc = hash_scratch_ptr(&ws))) return rc;
  g_err_clear();
  return run_hash_forward(make_hash_layout(*d), params, rays, n, 0, t, xi, static_cast<float*>(ws),
                          (hipStream_t)stream);
}

size_t ddf_hash_table_f16_bytes(const ddf_hash_desc* d) {
  if (check_hash_desc(d) != DDF_OK) return 0;
  const HashLayout L = make_hash_layout(*d);
  return (size_t)L.entries * 2 * sizeof(__half);
}

int ddf_hash_table_to_f16(const ddf_hash_desc* d, const float* params, void* table16, void* stream) {
  int rc;
  if ((rc = check_hash_desc(d))) return rc;
  if ((rc = check_ptr(params, "params")) || (rc = check_ptr(table16, "table16"))) return rc;
  g_err_clear();
  const int64_t n = make_hash_layout(*d).entries * 2;
  table_to_f16_kernel<<<2048, 256, 0, (hipStream_t)stream>>>(params, n, static_cast<__half*>(table16));
  return hip_status(hipGetLastError(), "ddf_hash_table_to_f16 launch");
}

int ddf_hash_query_f16(const ddf_hash_desc* d, const float* params, const void* table16, const float* rays, int64_t n,
                       float* t, float* xi, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_hash_desc(d))) return rc;
  if (n < 0 || n > (int64_t)INT32_MAX) return fail(DDF_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (n == 0) return DDF_OK;
  if ((rc = check_ptr(params, "params")) || (rc = check_ptr(table16, "table16")) || (rc = check_ptr(rays, "rays")) ||
      (rc = check_ptr(t, "t")) || (rc = check_ptr(xi, "xi")) || (rc = check_ptr(ws, "ws")))
    return rc;
  if (ws_bytes < (size_t)n * kHGroups * 16)
    return fail(DDF_ERR_INVALID_ARG, "workspace %zu bytes < %zu", ws_bytes, (size_t)n * kHGroups * 16);
  g_err_clear();
  return run_hash_forward(make_hash_layout(*d), params, rays, n, 0, t, xi, static_cast<float*>(ws),
                          (hipStream_t)stream, static_cast<const __half*>(table16));
}

size_t ddf_hash_train_workspace_bytes(const ddf_hash_desc* d, int64_t batch) {
  if (check_hash_desc(d) != DDF_OK || batch < 0) return 0;
  return (size_t)hash_ws(make_hash_layout(*d), batch).total;
}

int ddf_hash_train_step(const ddf_hash_desc* d, float* params, float* adam_m, float* adam_v, const float* rays,
                        const float* t_gt, const uint8_t* hit_gt, int64_t batch, const ddf_train_hparams* hp,
                        float* loss_out, int32_t* nonfinite_flag, float* grad_out, void* ws, size_t ws_bytes,
                        void* stream) {
  int rc;
  if ((rc = check_hash_desc(d)) || (rc = check_hp_public(hp))) return rc;
  if (!(hp->l1_clamp > 0.f) || !(hp->bce_weight >= 0.f))
    return fail(DDF_ERR_INVALID_ARG, "loss hyper-parameters out of range");
  if (batch < 1 || batch > (int64_t)INT32_MAX / 4) return fail(DDF_ERR_INVALID_ARG, "batch = %lld out of range", (long long)batch);
  if ((rc = check_ptr(params, "params")) || (rc = check_ptr(adam_m, "adam_m")) || (rc = check_ptr(adam_v, "adam_v")) ||
      (rc = check_ptr(rays, "rays")) || (rc = check_ptr(t_gt, "t_gt")) || (rc = check_ptr(hit_gt, "hit_gt")) ||
      (rc = check_ptr(loss_out, "loss_out")) || (rc = check_ptr(nonfinite_flag, "nonfinite_flag")) ||
      (rc = check_ptr(ws, "ws")))
    return rc;
  if (grad_out && (rc = check_ptr(grad_out, "grad_out"))) return rc;
  const HashLayout L = make_hash_layout(*d);
  const HashWs w = hash_ws(L, batch);
  if ((int64_t)ws_bytes < w.total) return fail(DDF_ERR_WORKSPACE, "workspace %zu < %lld bytes", ws_bytes, (long long)w.total);
  hipStream_t st = (hipStream_t)stream;
  uint8_t* wb = static_cast<uint8_t*>(ws);
  float* zt = reinterpret_cast<float*>(wb + w.zt);
  float* zx = reinterpret_cast<float*>(wb + w.zx);
  float* dzt = reinterpret_cast<float*>(wb + w.dzt);
  float* dzx = reinterpret_cast<float*>(wb + w.dzx);
  float* grad = grad_out ? grad_out : reinterpret_cast<float*>(wb + w.grad);
  g_err_clear();
  HashArgs a{};
  a.L = L; a.params = params; a.rays = rays; a.n = batch; a.R = w.R;
  float* acts = reinterpret_cast<float*>(wb + w.acts);
  float* G = acts;
  float* H1 = acts + w.R * kHIn;
  float* H2 = acts + 2 * w.R * kHIn;
  float* dl = reinterpret_cast<float*>(wb + w.deltas);
  float* D2 = dl;
  float* D1 = dl + w.R * kHIn;
  float* DG = dl + 2 * w.R * kHIn;
  a.acts = G;
  a.gtab = grad;
  const unsigned rb = (unsigned)((w.R + kHT - 1) / kHT);
  const float* P = params;
  // forward through memory
  if ((rc = run_hash_encode(a, st))) return rc;
  // hidden layers: 4 lanes per ray (16 outputs each); heads: one lane per ray, two outputs
  constexpr int kDS = 4;
  const unsigned rb4 = (unsigned)((w.R + kHT / kDS - 1) / (kHT / kDS));
  dense_fwd_kernel<kDS, kHW / kDS><<<rb4, kHT, 0, st>>>(G, P + L.w_off[0], P + L.b_off[0], kHW, L.d_in, w.R, 1, H1,
                                                        nullptr, nullptr);
  dense_fwd_kernel<kDS, kHW / kDS><<<rb4, kHT, 0, st>>>(H1, P + L.w_off[1], P + L.b_off[1], kHW, kHW, w.R, 1, H2,
                                                        nullptr, nullptr);
  dense_fwd_kernel<1, 2><<<rb, kHT, 0, st>>>(H2, P + L.wh_off, P + L.bh_off, 2, kHW, w.R, 0, nullptr, zt, zx);
  if ((rc = hip_status(hipGetLastError(), "hash training forward launch"))) return rc;
  if ((rc = launch_ddf_loss(zt, zx, t_gt, hit_gt, batch, w.R, reinterpret_cast<float*>(wb + w.lossp),
                            reinterpret_cast<float*>(wb + w.scal), loss_out, dzt, dzx, hp->bce_weight, hp->l1_clamp, st)))
    return rc;
  // backward: deltas, then the code gradient, its scatter into the table, the weight gradients
  dense_bwd_kernel<kDS, kHIn / kDS><<<rb4, kHT, 0, st>>>(nullptr, dzt, dzx, P + L.wh_off, 2, kHW, w.R, H2, D2);
  dense_bwd_kernel<kDS, kHIn / kDS><<<rb4, kHT, 0, st>>>(D2, nullptr, nullptr, P + L.w_off[1], kHW, kHW, w.R, H1, D1);
  dense_bwd_kernel<kDS, kHIn / kDS><<<rb4, kHT, 0, st>>>(D1, nullptr, nullptr, P + L.w_off[0], kHW, L.d_in, w.R,
                                                         nullptr, DG);
  fill_zero_kernel<<<1024, 256, 0, st>>>(grad, 2 * L.entries);
  if ((rc = hip_status(hipGetLastError(), "hash backward launch"))) return rc;
  if ((rc = run_hash_scatter(a, DG, st))) return rc;
  const unsigned nblk = (unsigned)(w.R / kHRC);
  float* part = reinterpret_cast<float*>(wb + w.part);
  const float* din[2] = {D1, D2};
  const float* ain[2] = {G, H1};
  for (int l = 0; l < 2; ++l) {
    const int fan_in = l == 0 ? L.d_in : kHW;
    outer_reduce_kernel<<<nblk, kHT, 0, st>>>(din[l], kHW, ain[l], kHW, part);
    sum_parts_kernel<<<(unsigned)((kHW * kHIn + kHW + 31) / 32), 256, 0, st>>>(part, (int)nblk, kHW, fan_in,
                                                                                grad + L.w_off[l], grad + L.b_off[l]);
  }
  for (int o = 0; o < 2; ++o) {   // the heads: each logit gradient against H2
    outer_reduce_kernel<<<nblk, kHT, 0, st>>>(o == 0 ? dzt : dzx, 1, H2, 1, part);
    sum_parts_kernel<<<(unsigned)((kHIn + 1 + 31) / 32), 256, 0, st>>>(part, (int)nblk, 1, kHW,
                                                                       grad + L.wh_off + o * kHW, grad + L.bh_off + o);
  }
  if ((rc = hip_status(hipGetLastError(), "hash weight-gradient launch"))) return rc;
  return launch_adam_flat(params, adam_m, adam_v, grad, L.params, hp, nonfinite_flag, st);
}

}  // extern "C"
