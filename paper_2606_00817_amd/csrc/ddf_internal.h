// Internal definitions shared by the HIP translation units of libddf.
//
// Packed network layout (the opaque blob of ddf_pack):
//  * every hidden layer l (0-based here) is a grid of operand blocks
//    [n_tiles = width/32][k_blocks][64 lanes][kblk elements]; block (nt, kb)
//    holds, for lane L, exactly the kblk weights that lane feeds to one
//    matrix-core step: output neuron n = 32 nt + (L mod 32) and inputs
//    k = kb * kblk + KMAP(L, j).  A wave therefore streams a layer with
//    contiguous 1 KiB (fp32, bf16) or 2 KiB (fp8) loads.
//  * layer 1 of the reduced precisions reads the encoded input split as
//    bf16 hi and lo halves; its blocks hold W_1 twice along k ([W_1 | W_1]).
//  * biases fp32 [n_hidden][width]; head fp32 [n_out][width] and [n_out].
//  * per-layer scales fp32 [n_hidden][4] (see ScaleSlot).
//  * for training, a transposed copy of hidden layers 2..n (W_l^T in the same
//    block format, used by the backward chain).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ddf.h"

namespace ddf {

constexpr int kMaxLayers = 32;
constexpr int kThreads = 256;   // 4 waves of 64: one per SIMD of a CU
constexpr int kWaves = 4;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x2 __attribute__((ext_vector_type(2)));

enum ScaleSlot { kDequant = 0, kQuantNext = 1, kScaleW = 2, kScaleA = 3 };

// Operand-block geometry per precision.
struct Geo {
  int elem_bytes;   // bytes per hidden-layer weight element (layers >= 2)
  int kblk;         // k elements per block (hidden layers >= 2)
  int elem1_bytes;  // bytes per layer-1 element
  int kblk1;        // k elements per layer-1 block
  int rays_per_wg;  // rays per workgroup of the query kernel
};

inline __host__ __device__ Geo geo_of(int precision) {
  switch (precision) {
    case DDF_FP32: return Geo{4, 8, 4, 8, 32};
    case DDF_BF16: return Geo{2, 16, 2, 16, 64};
    default:       return Geo{1, 64, 2, 16, 128};
  }
}

inline __host__ __device__ int round_up(int x, int m) { return (x + m - 1) / m * m; }

struct Layout {
  int64_t w_off[kMaxLayers];   // byte offset of hidden layer l's operand blocks
  int64_t wt_off[kMaxLayers];  // byte offset of the transposed copy (layers >= 1), training
  int64_t b_off;               // fp32 biases [n_hidden][width]
  int64_t head_w_off;          // fp32 [n_out][width]
  int64_t head_b_off;          // fp32 [n_out]
  int64_t scale_off;           // fp32 [n_hidden][4]
  int64_t total;
  int n_feat;                  // encoded features n_in (1 + 2 L)
  int k1;                      // padded layer-1 k (doubled for the bf16 hi/lo split)
  int k1_half;                 // padded feature count (one half of k1 for reduced precision)
};

inline int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

inline Layout make_layout(const ddf_net_desc& d) {
  Layout L{};
  Geo g = geo_of(d.precision);
  L.n_feat = d.n_in * (1 + 2 * d.n_freq);
  L.k1_half = round_up(L.n_feat, 4 * g.kblk1);   // a multiple of 4 k blocks
  L.k1 = d.precision == DDF_FP32 ? L.k1_half : 2 * L.k1_half;
  int64_t off = 0;
  for (int l = 0; l < d.n_hidden; ++l) {
    int64_t k = l == 0 ? L.k1 : d.width;
    int64_t eb = l == 0 ? g.elem1_bytes : g.elem_bytes;
    L.w_off[l] = off;
    off = align256(off + (int64_t)d.width * k * eb);
  }
  L.b_off = off; off = align256(off + 4ll * d.n_hidden * d.width);
  L.head_w_off = off; off = align256(off + 4ll * d.n_out * d.width);
  L.head_b_off = off; off = align256(off + 4ll * d.n_out);
  L.scale_off = off; off = align256(off + 16ll * d.n_hidden);
  // transposed copies for the backward chain (fp32 / bf16 training only)
  for (int l = 1; l < d.n_hidden; ++l) {
    L.wt_off[l] = off;
    off = align256(off + (int64_t)d.width * d.width * g.elem_bytes);
  }
  L.total = off;
  return L;
}

// ------------------------------------------------------------------ device helpers

__device__ inline float wave_sum32(float v) {
  // sum over the 32 lanes sharing lane / 32 (fixed butterfly order)
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 4);
  v += __shfl_xor(v, 8);
  v += __shfl_xor(v, 16);
  return v;
}

__device__ inline float softplusf_(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }
__device__ inline float sigmoidf_(float z) {
  float e = expf(-fabsf(z));
  return z >= 0.f ? 1.f / (1.f + e) : e / (1.f + e);
}

// float -> bf16, round to nearest even (NaN kept quiet)
__device__ inline __bf16 to_bf16(float x) { return (__bf16)x; }

}  // namespace ddf
