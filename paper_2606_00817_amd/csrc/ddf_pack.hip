// Packing of the float32 master into the working copy the query kernels stream.
//
// Block geometry: see ddf_internal.h.  Within a block, lane L feeds
// kblk / 2 consecutive k values: k = kb * kblk + (kblk / 2) * (L / 32) + j.
#include "ddf_internal.h"

namespace ddf {

struct PackArgs {
  const float* master;
  uint8_t* packed;
  Layout lay;
  int64_t w_src[kMaxLayers];   // float offset of W_l in the master
  int64_t b_src[kMaxLayers];   // float offset of b_l
  int64_t head_w_src, head_b_src;
  float act_scale[kMaxLayers]; // FP8: s_A of layer l's input (l >= 1)
  int n_hidden, width, n_out, precision;
};

__device__ inline float fp8_quant(float x) {
  // saturate to the largest finite e4m3 value, then convert (round to nearest even)
  x = fminf(fmaxf(x, -448.f), 448.f);
  return x;
}

// amax |W_l| of the hidden layers l >= 1 (FP8 weight scales), as ordered uint bits.
__global__ void amax_kernel(PackArgs a) {
  const int l = blockIdx.y + 1;
  const int64_t cnt = (int64_t)a.width * a.width;
  const float* w = a.master + a.w_src[l];
  float m = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(w[i]));
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  __shared__ float red[kWaves];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float r = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    unsigned int* slot = reinterpret_cast<unsigned int*>(a.packed + a.lay.scale_off) + 4 * l + kScaleW;
    atomicMax(slot, __float_as_uint(r));
  }
}

__global__ void zero_scales_kernel(PackArgs a) {
  float* s = reinterpret_cast<float*>(a.packed + a.lay.scale_off);
  for (int i = threadIdx.x; i < 4 * a.n_hidden; i += blockDim.x) s[i] = 0.f;
}

// Turns the amax bits into power-of-two scales and fills every scale slot.
__global__ void finish_scales_kernel(PackArgs a) {
  float* s = reinterpret_cast<float*>(a.packed + a.lay.scale_off);
  const int l = threadIdx.x;
  if (l >= a.n_hidden) return;
  float sw = 1.f, sa = 1.f;
  if (a.precision == DDF_FP8_E4M3 && l >= 1) {
    float amax = s[4 * l + kScaleW];   // holds the amax bits written by amax_kernel
    if (amax > 0.f) {
      int e;
      float m = frexpf(amax, &e);      // amax = m 2^e, 0.5 <= m < 1
      sw = ldexpf(1.f, e - 9 + (2.f * m > 1.75f ? 1 : 0));
    }
    sa = a.act_scale[l];
  }
  s[4 * l + kScaleW] = sw;
  s[4 * l + kScaleA] = sa;
  s[4 * l + kDequant] = sw * sa;
  float qn = 1.f;
  if (a.precision == DDF_FP8_E4M3 && l + 1 < a.n_hidden) qn = 1.f / a.act_scale[l + 1];
  s[4 * l + kQuantNext] = qn;
}

// One thread per (block, lane): writes that lane's kblk/2 elements (16 or 32 bytes) of one
// layer.  blockIdx.y selects the job: layer j, or (j >= n_hidden) the transposed copy of layer
// j - n_hidden + 1; every layer of a repack in one launch.
__global__ void pack_layer_kernel(PackArgs a, int with_transposed) {
  const Geo g = geo_of(a.precision);
  const int job = blockIdx.y;
  const int transposed = job >= a.n_hidden ? 1 : 0;
  const int l = transposed ? job - a.n_hidden + 1 : job;
  if (transposed && !with_transposed) return;
  const bool first = (l == 0);
  const int kblk = first ? g.kblk1 : g.kblk;
  const int eb = first ? g.elem1_bytes : g.elem_bytes;
  const int K = first ? a.lay.k1 : a.width;
  const int KB = K / kblk;
  const int per = kblk / 2;
  const int64_t n_lanes = (int64_t)(a.width / 32) * KB * 64;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_lanes) return;
  const int lane = (int)(i % 64);
  const int64_t blk = i / 64;
  const int nt = (int)(blk / KB), kb = (int)(blk % KB);
  const int n = nt * 32 + (lane & 31);
  const int kbase = kb * kblk + per * (lane >> 5);
  const float* W = a.master + a.w_src[l];
  const int fan_in = first ? a.lay.n_feat : a.width;
  uint8_t* dst = a.packed + (transposed ? a.lay.wt_off[l] : a.lay.w_off[l]) + i * per * eb;
  float qs = 1.f;
  if (!first && a.precision == DDF_FP8_E4M3) {
    const float* s = reinterpret_cast<const float*>(a.packed + a.lay.scale_off);
    qs = 1.f / s[4 * l + kScaleW];     // exact: a power of two
  }
  if (!first && !transposed && eb == 2) {
    // bf16 hidden layer in the master's orientation: the lane's 8 consecutive inputs are two
    // 16-byte loads (row n, columns kbase .. kbase + 7), not 8 scalar ones
    const f32x4* src = reinterpret_cast<const f32x4*>(W + (int64_t)n * fan_in + kbase);
    const f32x4 v0 = src[0], v1 = src[1];
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      o[j] = to_bf16(v0[j]);
      o[4 + j] = to_bf16(v1[j]);
    }
    *reinterpret_cast<bf16x8*>(dst) = o;
    return;
  }
  // the lane's bytes are gathered in registers and leave as 16-byte stores (per * eb is 16
  // or 32: fp32 8 x 4, bf16 8 x 2, e4m3 32 x 1, layer-1 bf16 8 x 2)
  i32x4 out[2] = {};
  uint8_t* ob = reinterpret_cast<uint8_t*>(out);
  for (int j = 0; j < per; ++j) {
    int k = kbase + j;
    float w;
    if (first) {
      int kk = (a.precision == DDF_FP32) ? k : k % a.lay.k1_half;
      w = kk < a.lay.n_feat ? W[(int64_t)n * fan_in + kk] : 0.f;
    } else {
      w = transposed ? W[(int64_t)k * fan_in + n] : W[(int64_t)n * fan_in + k];
    }
    if (eb == 4) {
      reinterpret_cast<float*>(ob)[j] = w;
    } else if (eb == 2) {
      reinterpret_cast<__bf16*>(ob)[j] = to_bf16(w);
    } else {
      float q = fp8_quant(w * qs);
      int pk = __builtin_amdgcn_cvt_pk_fp8_f32(q, q, 0, false);
      ob[j] = (uint8_t)(pk & 0xff);
    }
  }
  reinterpret_cast<i32x4*>(dst)[0] = out[0];
  if (per * eb > 16) reinterpret_cast<i32x4*>(dst)[1] = out[1];
}

__global__ void pack_small_kernel(PackArgs a) {
  float* b = reinterpret_cast<float*>(a.packed + a.lay.b_off);
  float* hw = reinterpret_cast<float*>(a.packed + a.lay.head_w_off);
  float* hb = reinterpret_cast<float*>(a.packed + a.lay.head_b_off);
  const int64_t nb = (int64_t)a.n_hidden * a.width;
  const int64_t nh = (int64_t)a.n_out * a.width;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb + nh + a.n_out;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < nb) {
      int l = (int)(i / a.width), n = (int)(i % a.width);
      b[i] = a.master[a.b_src[l] + n];
    } else if (i < nb + nh) {
      hw[i - nb] = a.master[a.head_w_src + (i - nb)];
    } else {
      hb[i - nb - nh] = a.master[a.head_b_src + (i - nb - nh)];
    }
  }
}

hipError_t launch_pack(const ddf_net_desc& d, const float* master, const float* act_scales,
                       void* packed, hipStream_t st, bool with_transposed) {
  PackArgs a{};
  a.master = master;
  a.packed = static_cast<uint8_t*>(packed);
  a.lay = make_layout(d);
  a.n_hidden = d.n_hidden; a.width = d.width; a.n_out = d.n_out; a.precision = d.precision;
  int64_t off = 0;
  for (int l = 0; l < d.n_hidden; ++l) {
    int64_t fi = l == 0 ? a.lay.n_feat : d.width;
    a.w_src[l] = off; off += fi * d.width;
    a.b_src[l] = off; off += d.width;
    a.act_scale[l] = (act_scales && l >= 1) ? act_scales[l - 1] : 1.f;
  }
  a.head_w_src = off; off += (int64_t)d.n_out * d.width;
  a.head_b_src = off;
  zero_scales_kernel<<<1, 64, 0, st>>>(a);
  if (d.precision == DDF_FP8_E4M3 && d.n_hidden > 1)
    amax_kernel<<<dim3(64, d.n_hidden - 1), kThreads, 0, st>>>(a);
  finish_scales_kernel<<<1, 64, 0, st>>>(a);
  {
    // one launch: jobs 0 .. n_hidden - 1 the layers, then the transposed copies of layers 2..n
    const Geo g = geo_of(d.precision);
    int64_t lanes = 0;
    for (int l = 0; l < d.n_hidden; ++l) {
      const int K = l == 0 ? a.lay.k1 : d.width;
      const int kblk = l == 0 ? g.kblk1 : g.kblk;
      const int64_t ll = (int64_t)(d.width / 32) * (K / kblk) * 64;
      lanes = ll > lanes ? ll : lanes;
    }
    const bool tr = with_transposed && d.precision != DDF_FP8_E4M3 && d.n_hidden > 1;
    const dim3 grid((unsigned)((lanes + kThreads - 1) / kThreads), (unsigned)(d.n_hidden + (tr ? d.n_hidden - 1 : 0)));
    pack_layer_kernel<<<grid, kThreads, 0, st>>>(a, tr ? 1 : 0);
  }
  pack_small_kernel<<<256, kThreads, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace ddf
