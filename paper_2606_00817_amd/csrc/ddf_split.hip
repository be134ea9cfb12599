// The small-batch DDF query: one launch per layer with the layer's neurons split across
// workgroups.  The fused query gives each workgroup 64 rays and the whole network, so every
// workgroup streams all the weights and a batch below ~16K rays leaves most CUs idle (a 1K-ray
// query takes as long as a 10K-ray one).  Here a workgroup of 8 waves owns 64 rays x 256
// neurons of one layer: a 1K-ray batch fills 16 x (width / 256) workgroups per layer, each
// streaming only its 256 neurons' weights; the activations go through a [rays][width] buffer
// between layers.  Every workgroup of a ray tile reads the tile's whole input, so the
// neuron-group count (width / 256) is also the number of times the activations are re-read,
// the path's bound from a few thousand rays up; 8 waves rather than 4 halve those re-reads
// and give each SIMD two waves (the 128 KiB activation tile allows one workgroup per CU).
// The products are the fused kernel's (same operand blocks, same k order), so the hidden
// activations are bit-identical; the heads' partial sums are added in another order.
#include <math.h>

#include "ddf_chain.h"
#include "ddf_fwd.h"
#include "ddf_internal.h"
#include "ddf_train.h"

namespace ddf {

FwdArgs base_args(const ddf_net_desc& d, const void* packed);

namespace {

constexpr int kSplitWaves = 8;                       // one 32-neuron tile per wave
constexpr int kSplitNeurons = 32 * kSplitWaves;      // neurons per workgroup

struct SplitArgs {
  FwdArgs f;              // network, layout and rays (the first layer's encoding reads them)
  int layer;              // 0-based hidden layer of this launch
  const __bf16* hin;      // [R][width] the layer's input (layer > 0)
  __bf16* hout;           // [R][width] the layer's output (all but the last layer)
  float* part;            // [width / 256][R][2] head partial sums (the last layer)
  int64_t R;              // rows (a multiple of 64)
};

template <int WIDTH>
__global__ __launch_bounds__(64 * kSplitWaves, 1) void split_layer_kernel(SplitArgs a) {
  using P = PBF16;
  using E = __bf16;
  using C = Chain<P, WIDTH, WIDTH / 32>;   // WIDTH / 32 tiles of 32 neurons: one per wave
  constexpr int M = C::M, RT = C::RT, LDX = C::LDX;
  static_assert(C::NT == 1, "one tile per wave");
  __shared__ __attribute__((aligned(16))) E X[C::XSIZE];
  __shared__ float hsum[kSplitWaves][M][2];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // Workgroups go to the 8 XCDs in turn (id mod 8); the neuron groups of one ray tile take
  // consecutive turns on the same XCD, so that they read the tile's input through one L2 at
  // about the same time: the input is fetched past the L2 once, not once per group.
  constexpr int G = WIDTH / kSplitNeurons;            // neuron groups per ray tile
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int64_t tile = (int64_t)(slot / G) * 8 + xcd;
  const int group = slot % G;
  if (tile * M >= a.R) return;                        // the grid is rounded up to 8 tiles
  const int64_t ray0 = tile * M;
  const int l = a.layer;

  if (l == 0) {
    encode_tile<E, M, LDX, kModeQuery>(a.f, ray0, X);
  } else {
    // rows ray0 .. ray0 + 63 of the layer input, 16 bytes per thread and chunk; all of a
    // batch's loads are issued before its LDS writes (one load latency per batch, not per chunk)
    constexpr int kChunks = M * (WIDTH / 8) / (64 * kSplitWaves);   // per thread
    constexpr int kBatch = kChunks < 16 ? kChunks : 16;
#pragma unroll
    for (int b0 = 0; b0 < kChunks; b0 += kBatch) {
      bf16x8 v[kBatch];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        const int idx = (b0 + j) * (64 * kSplitWaves) + threadIdx.x;
        const int r = idx / (WIDTH / 8), c8 = idx % (WIDTH / 8);
        v[j] = *reinterpret_cast<const bf16x8*>(a.hin + (ray0 + r) * WIDTH + c8 * 8);
      }
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        const int idx = (b0 + j) * (64 * kSplitWaves) + threadIdx.x;
        const int r = idx / (WIDTH / 8), c8 = idx % (WIDTH / 8);
        *reinterpret_cast<bf16x8*>(X + r * LDX + c8 * 8) = v[j];
      }
    }
  }
  __syncthreads();

  const int nt0 = group * kSplitWaves + wave;   // this wave's neuron tile
  const int K = l == 0 ? a.f.lay.k1 : WIDTH;
  const void* W = a.f.packed + a.f.lay.w_off[l];
  f32x16 acc[RT][1];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) acc[rt][0] = f32x16{};
  typename C::Ring ring;
  C::preload(ring, W, K / P::KBLK, nt0, lane);
  if (l == 0)
    C::template gemm<0, true>(acc, X, W, K / P::KBLK, nt0, lane, ring);
  else
    C::template gemm<WIDTH / P::KBLK, true>(acc, X, W, K / P::KBLK, nt0, lane, ring);

  // register group q of tile rt: neurons nb + 8 q + i (i < 4) of ray rt 32 + lane % 32
  const float* bias = reinterpret_cast<const float*>(a.f.packed + a.f.lay.b_off) + (int64_t)l * WIDTH;
  const float* hw = reinterpret_cast<const float*>(a.f.packed + a.f.lay.head_w_off);
  const bool last = l + 1 == a.f.n_hidden;
  const int nb = nt0 * 32 + 4 * (lane >> 5);
  float hp0[RT], hp1[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) { hp0[rt] = 0.f; hp1[rt] = 0.f; }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const f32x4 b4 = *reinterpret_cast<const f32x4*>(bias + nb + 8 * q);
    f32x4 w0 = {}, w1 = {};
    if (last) {
      w0 = *reinterpret_cast<const f32x4*>(hw + nb + 8 * q);
      w1 = *reinterpret_cast<const f32x4*>(hw + WIDTH + nb + 8 * q);
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      f32x4 y;
#pragma unroll
      for (int i = 0; i < 4; ++i) y[i] = fmaxf(acc[rt][0][4 * q + i] + b4[i], 0.f);
      if (last) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          hp0[rt] = fmaf(w0[i], y[i], hp0[rt]);
          hp1[rt] = fmaf(w1[i], y[i], hp1[rt]);
        }
      } else {
        V4<E> yv;
#pragma unroll
        for (int i = 0; i < 4; ++i) yv[i] = (E)y[i];
        *reinterpret_cast<V4<E>*>(a.hout + (ray0 + rt * 32 + (lane & 31)) * WIDTH + nb + 8 * q) = yv;
      }
    }
  }
  if (last) {   // uniform over the workgroup
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const float s0 = hp0[rt] + __shfl_xor(hp0[rt], 32);
      const float s1 = hp1[rt] + __shfl_xor(hp1[rt], 32);
      if (lane < 32) {
        hsum[wave][rt * 32 + lane][0] = s0;
        hsum[wave][rt * 32 + lane][1] = s1;
      }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < M; r += blockDim.x) {
      float z0 = 0.f, z1 = 0.f;
#pragma unroll
      for (int w = 0; w < kSplitWaves; ++w) { z0 += hsum[w][r][0]; z1 += hsum[w][r][1]; }
      float* dst = a.part + ((int64_t)group * a.R + ray0 + r) * 2;
      dst[0] = z0;
      dst[1] = z1;
    }
  }
}

// t, xi from the head bias and the slices' partial sums (added in slice order).
__global__ void split_heads_kernel(const float* __restrict__ part, int slices, int64_t R, int64_t n,
                                   const float* __restrict__ hb, float* __restrict__ t, float* __restrict__ xi) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  float z0 = hb[0], z1 = hb[1];
  for (int s = 0; s < slices; ++s) {
    z0 += part[((int64_t)s * R + r) * 2];
    z1 += part[((int64_t)s * R + r) * 2 + 1];
  }
  t[r] = softplusf_(z0);
  xi[r] = sigmoidf_(z1);
}

struct SplitWs {
  int64_t R, h0, h1, part, total;
};

SplitWs split_ws(const ddf_net_desc& d, int64_t n) {
  SplitWs w{};
  w.R = (n + 63) / 64 * 64;
  const int64_t hb = w.R * d.width * 2;
  w.h0 = 0;
  w.h1 = align256(hb);
  w.part = w.h1 + align256(hb);
  w.total = w.part + align256((int64_t)(d.width / kSplitNeurons) * w.R * 2 * 4);
  return w;
}

template <int WIDTH>
hipError_t launch_split(const SplitArgs& a, hipStream_t st) {
  const int64_t tiles8 = (a.R / 64 + 7) / 8 * 8;   // ray tiles rounded up to the 8 XCDs
  const dim3 grid((unsigned)(tiles8 * (WIDTH / kSplitNeurons)));
  hipLaunchKernelGGL((split_layer_kernel<WIDTH>), grid, dim3(64 * kSplitWaves), 0, st, a);
  return hipGetLastError();
}

int check_split(const ddf_net_desc* d) {
  int rc;
  if ((rc = check_desc(d))) return rc;
  if (d->n_in != 6 || d->n_out != 2) return fail(DDF_ERR_INVALID_ARG, "the query needs n_in 6 and n_out 2");
  if (d->precision != DDF_BF16) return fail(DDF_ERR_UNSUPPORTED, "the split query is built for bf16");
  if (d->width != 256 && d->width != 512 && d->width != 1024)
    return fail(DDF_ERR_UNSUPPORTED, "the split query needs width 256, 512 or 1024");
  return DDF_OK;
}

}  // namespace
}  // namespace ddf

using namespace ddf;

extern "C" {

size_t ddf_query_split_workspace_bytes(const ddf_net_desc* d, int64_t n) {
  if (check_split(d) != DDF_OK || n < 0) return 0;
  return (size_t)split_ws(*d, n).total;
}

int ddf_query_split(const ddf_net_desc* d, const void* packed, const float* rays, int64_t n, float* t, float* xi,
                    void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_split(d))) return rc;
  if (n < 0 || n > (int64_t)INT32_MAX / 64) return fail(DDF_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (n == 0) return DDF_OK;
  if ((rc = check_ptr(packed, "packed")) || (rc = check_ptr(rays, "rays")) || (rc = check_ptr(t, "t")) ||
      (rc = check_ptr(xi, "xi")) || (rc = check_ptr(ws, "ws")))
    return rc;
  const SplitWs w = split_ws(*d, n);
  if (ws_bytes < (size_t)w.total)
    return fail(DDF_ERR_WORKSPACE, "workspace %zu bytes < %lld", ws_bytes, (long long)w.total);
  g_err_clear();
  hipStream_t st = (hipStream_t)stream;
  uint8_t* base = static_cast<uint8_t*>(ws);
  SplitArgs a{};
  a.f = base_args(*d, packed);
  a.f.in = rays; a.f.n = n; a.f.stride = n; a.f.mode = kModeQuery;
  a.R = w.R;
  a.part = reinterpret_cast<float*>(base + w.part);
  __bf16* h[2] = {reinterpret_cast<__bf16*>(base + w.h0), reinterpret_cast<__bf16*>(base + w.h1)};
  for (int l = 0; l < d->n_hidden; ++l) {
    a.layer = l;
    a.hin = l > 0 ? h[(l - 1) & 1] : nullptr;
    a.hout = l + 1 < d->n_hidden ? h[l & 1] : nullptr;
    hipError_t e;
    switch (d->width) {
      case 256: e = launch_split<256>(a, st); break;
      case 512: e = launch_split<512>(a, st); break;
      default: e = launch_split<1024>(a, st); break;
    }
    if (e != hipSuccess) return hip_status(e, "split query layer launch");
  }
  const float* hb = reinterpret_cast<const float*>(static_cast<const uint8_t*>(packed) + a.f.lay.head_b_off);
  split_heads_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(a.part, d->width / kSplitNeurons, w.R, n, hb, t,
                                                                  xi);
  return hip_status(hipGetLastError(), "split query heads launch");
}

}  // extern "C"
