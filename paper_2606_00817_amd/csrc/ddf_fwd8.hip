// FP8 (OCP e4m3) forward pass of the DDF / SDF MLP on the gfx950 matrix cores.
//
// Same structure as the fp32/bf16 chain (one workgroup owns a ray tile for the
// whole network: 8 waves, two per SIMD, at width 512 and 1024, 4 at width 256;
// activations resident in LDS, weight blocks streamed from global memory), with
// M = 128 rays per workgroup:
//  * layer 1 reads the encoded input split as bf16 hi + lo
//    (v_mfma_f32_32x32x16_bf16) with bf16 weights;
//  * hidden layers 2..n read e4m3 activations and e4m3 weights
//    (v_mfma_scale_f32_32x32x64_f8f6f4 with unit block scales), accumulate in
//    fp32 and rescale the sum by the layer's power-of-two s_A s_W;
//  * the epilogue adds the bias, applies ReLU and stores e4m3(h / s_A,next)
//    into LDS; the heads read the fp32 output of the last layer.
// A wave owns width/waves output neurons; with 128 rays the accumulators of all of
// them do not fit at once, so each layer runs in two passes over half of the
// wave's neurons, the first pass's e4m3 results waiting in registers until the
// layer's input may be overwritten.
#include "ddf_fwd.h"
#include "ddf_internal.h"

namespace ddf {

namespace {

constexpr int kM8 = 128;                 // rays per workgroup
constexpr int kRT8 = kM8 / 32;           // 32-ray tiles
constexpr int kLDG = 256 + 8;            // bf16 row stride of the layer-1 input (k1 <= 256)

__device__ inline i32x8 lds_a8(const uint8_t* p) {
  const i32x4 lo = *reinterpret_cast<const i32x4*>(p);
  const i32x4 hi = *reinterpret_cast<const i32x4*>(p + 16);
  return i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

__device__ inline i32x8 buf_b8(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
  const i32x4 lo = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0);
  const i32x4 hi = __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 16, soff, 0);
  return i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

// The lane index, recomputed where it is used: the empty asm makes the value opaque, so the
// per-lane addresses derived from it are formed in the epilogue instead of being hoisted to
// the kernel start, kept live across every layer and spilled.
__device__ inline int fresh_lane() {
  int l = (int)(threadIdx.x & 63);
  asm volatile("" : "+v"(l));
  return l;
}

// Four values in [0, 448], already divided by the next layer's scale, as four e4m3 codes in
// one word (element i in byte i), rounded to nearest even.
__device__ inline uint32_t pack_e4m3(float y0, float y1, float y2, float y3) {
  const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(y0, y1, 0, false);
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(y2, y3, lo, true);
}

// The four e4m3 words of one ray and one 32-neuron tile, lane el holding neurons
// 8 q + 4 (el / 32) + i of it in word q, regrouped by two lane-half swaps so that lanes below
// 32 hold neurons 0 .. 15 and the others 16 .. 31, as 16 contiguous bytes each.  One 128-bit
// LDS write per tile then replaces four 32-bit writes: at the row stride of WIDTH + 16 bytes
// the 32 rows of a 32-bit write fall into only 8 banks, while the 128-bit write (like the
// products' 128-bit reads) spreads its rows over all of them.
__device__ inline i32x4 regroup16(const uint32_t (&w)[4]) {
  const auto s02 = __builtin_amdgcn_permlane32_swap(w[0], w[2], false, false);
  const auto s13 = __builtin_amdgcn_permlane32_swap(w[1], w[3], false, false);
  return i32x4{(int)s02[0], (int)s02[1], (int)s13[0], (int)s13[1]};
}

// acc[rt][t] += G[rt rows][0:K1] * W1[tile (tile0 + t)][0:K1]^T   (bf16 operands, 1 KiB
// blocks).  The weight loads run two blocks ahead in a ring of three; the loads past the end
// of the layer are bounds-checked by the buffer resource (zeros, never used).
template <int NTP>
__device__ inline void gemm_l1(f32x16 (&acc)[kRT8][NTP], const __bf16* G, const void* W, int KB,
                               int tile0, int lane, int width) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(W), (short)0, width * KB * 32, 0x00020000);
  const int voff = lane * 16;
  const int base = tile0 * KB * 1024, tstride = KB * 1024;
  const __bf16* xrow = G + (lane & 31) * kLDG + 8 * (lane >> 5);
  bf16x8 b[3][NTP];
#pragma unroll
  for (int st = 0; st < 2; ++st)
#pragma unroll
    for (int t = 0; t < NTP; ++t)
      b[st][t] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, base + t * tstride + st * 1024, 0));
  // three steps per pass of the loop keep the ring's indexing static
  for (int k = 0; k < KB; k += 3) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (k + j < KB) {
#pragma unroll
        for (int t = 0; t < NTP; ++t)
          b[(j + 2) % 3][t] = __builtin_bit_cast(
              bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, base + t * tstride + (k + j + 2) * 1024, 0));
        bf16x8 av[kRT8];
#pragma unroll
        for (int rt = 0; rt < kRT8; ++rt)
          av[rt] = *reinterpret_cast<const bf16x8*>(xrow + rt * 32 * kLDG + (k + j) * 16);
#pragma unroll
        for (int rt = 0; rt < kRT8; ++rt)
#pragma unroll
          for (int t = 0; t < NTP; ++t)
            acc[rt][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[j][t], av[rt], acc[rt][t], 0, 0, 0);
      }
    }
  }
}

// acc[rt][t] += X[rt rows][0:K] * W[tile (tile0 + t)][0:K]^T   (e4m3 operands, 2 KiB blocks).
// K = KB * 64 is a compile-time constant: the k loop is fully unrolled, with the weight
// loads running two blocks ahead in a ring of three (loads past the end of the layer are
// bounds-checked by the buffer resource: they return zeros and are never used).
template <int NTP, int LDX, int KB>
__device__ inline void gemm_f8(f32x16 (&acc)[kRT8][NTP], const uint8_t* X, const void* W, int tile0,
                               int lane, int width) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(W), (short)0, width * KB * 64, 0x00020000);
  const int voff = lane * 32;
  const int base = tile0 * KB * 2048;
  const uint8_t* xrow = X + (lane & 31) * LDX + 32 * (lane >> 5);
  i32x8 b[3][NTP];
  i32x8 av[2][kRT8];
#pragma unroll
  for (int st = 0; st < 2; ++st)
#pragma unroll
    for (int t = 0; t < NTP; ++t) b[st][t] = buf_b8(rs, voff, base + (t * KB + st) * 2048);
#pragma unroll
  for (int rt = 0; rt < kRT8; ++rt) av[0][rt] = lds_a8(xrow + rt * 32 * LDX);
#pragma unroll
  for (int k = 0; k < KB; ++k) {
#pragma unroll
    for (int t = 0; t < NTP; ++t) b[(k + 2) % 3][t] = buf_b8(rs, voff, base + (t * KB + k + 2) * 2048);
    if (k + 1 < KB) {
#pragma unroll
      for (int rt = 0; rt < kRT8; ++rt) av[(k + 1) & 1][rt] = lds_a8(xrow + rt * 32 * LDX + (k + 1) * 64);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int rt = 0; rt < kRT8; ++rt)
#pragma unroll
      for (int t = 0; t < NTP; ++t)
        acc[rt][t] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(b[k % 3][t], av[k & 1][rt], acc[rt][t], 0, 0,
                                                                     0, 127, 0, 127);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Weight block (t, k) of an e4m3 layer for the streamed product below, at byte
// ((tile0 + t) KB + k) 2 KiB + lane 32 of the layer: the per-lane part and (k mod 2) 2 KiB go
// into the vector offset, the wave-uniform tile and k / 2 part into the scalar offset.
template <int KB>
__device__ inline i32x8 ld8(__amdgpu_buffer_rsrc_t rs, int voff, int base, int t, int k) {
  return buf_b8(rs, voff + (k & 1) * 2048, base + t * KB * 2048 + (k >> 1) * 4096);
}

template <int KB>
__device__ inline __amdgpu_buffer_rsrc_t rsrc8(const void* W, int width) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(W), (short)0, width * KB * 64, 0x00020000);
}

// Stages of the streamed product's weight ring.
constexpr int kS8 = 2;

// First kS8 - 1 stages of an e4m3 layer's weight ring (issued ahead of time, before the
// previous pass's epilogue: the weights do not depend on its output).
template <int NTP, int KB>
__device__ inline void preload8(i32x8 (&b)[kS8][NTP], const void* W, int tile0, int lane, int width) {
  const __amdgpu_buffer_rsrc_t rs = rsrc8<KB>(W, width);
#pragma unroll
  for (int st = 0; st < kS8 - 1; ++st)
#pragma unroll
    for (int t = 0; t < NTP; ++t) b[st][t] = ld8<KB>(rs, lane * 32, tile0 * KB * 2048, t, st);
}

// The same product with the activation operand streamed one 32-ray tile at a time (the LDS
// read of the tile two ahead overlaps the current tile's products) and the weight ring one k
// step ahead: fewer registers, for the 8-wave layout where two waves share a SIMD's register
// file.  The ring's first kS8 - 1 stages come from preload8.
template <int NTP, int LDX, int KB>
__device__ inline void gemm_f8_stream(f32x16 (&acc)[kRT8][NTP], const uint8_t* X, const void* W, int tile0,
                                      int lane, int width, i32x8 (&b)[kS8][NTP]) {
  const __amdgpu_buffer_rsrc_t rs = rsrc8<KB>(W, width);
  const int voff = lane * 32;
  const int base = tile0 * KB * 2048;
  const uint8_t* xrow = X + (lane & 31) * LDX + 32 * (lane >> 5);
  // the activation operand two 32-ray tiles ahead, in a rotation of three
  i32x8 av[3];
  av[0] = lds_a8(xrow);
  av[1] = lds_a8(xrow + 32 * LDX);
#pragma unroll
  for (int k = 0; k < KB; ++k) {
#pragma unroll
    for (int t = 0; t < NTP; ++t) b[(k + kS8 - 1) % kS8][t] = ld8<KB>(rs, voff, base, t, k + kS8 - 1);
#pragma unroll
    for (int rt = 0; rt < kRT8; ++rt) {
      const int i = k * kRT8 + rt;            // running tile index: i mod 3 picks the buffer
      const int rt2 = (rt + 2) % kRT8, k2 = k + (rt + 2) / kRT8;
      if (k2 < KB) av[(i + 2) % 3] = lds_a8(xrow + rt2 * 32 * LDX + k2 * 64);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int t = 0; t < NTP; ++t)
        acc[rt][t] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(b[k % kS8][t], av[i % 3], acc[rt][t], 0, 0, 0,
                                                                     127, 0, 127);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

}  // namespace

template <int WIDTH, int MODE, int WAVES>
__global__ __launch_bounds__(WAVES * 64, 1) void fwd8_kernel(FwdArgs a) {
  constexpr int NTW = WIDTH / 32 / WAVES;    // 32-neuron tiles per wave
  constexpr int NTP = NTW / 2;               // tiles per pass
  constexpr int LDX = WIDTH + 16;            // e4m3 row stride (bytes)
  constexpr int XBYTES = kM8 * LDX > kM8 * kLDG * 2 ? kM8 * LDX : kM8 * kLDG * 2;
  __shared__ __attribute__((aligned(16))) uint8_t smem[XBYTES];
  __shared__ float headp[WAVES][kM8][2];
  // the current layer's bias, each wave's own neurons copied in by that wave
  __shared__ __attribute__((aligned(16))) float bsm[WIDTH];
  uint8_t* X = smem;
  __bf16* G = reinterpret_cast<__bf16*>(smem);

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ray0 = (int64_t)blockIdx.x * kM8;
  if (MODE == kModeTrace && ray0 >= *a.count) return;
  const int64_t n_act = MODE == kModeTrace ? (int64_t)*a.count : a.n;
  FwdArgs aa = a;
  aa.n = n_act;

  encode_tile<__bf16, kM8, kLDG, MODE>(aa, ray0, G);
  __syncthreads();

  const float* bias_all = reinterpret_cast<const float*>(a.packed + a.lay.b_off);
  const float* hw = reinterpret_cast<const float*>(a.packed + a.lay.head_w_off);
  const float* hb = reinterpret_cast<const float*>(a.packed + a.lay.head_b_off);
  const float* scales = reinterpret_cast<const float*>(a.packed + a.lay.scale_off);

  i32x8 ring[kS8][NTW / 2];                // e4m3 weight ring (8-wave layout)
  for (int l = 0; l < a.n_hidden; ++l) {
    const bool last = (l + 1 == a.n_hidden);
    const float dq = scales[4 * l + kDequant];
    const float qn = scales[4 * l + kQuantNext];
    const float dqn = dq * qn;
    const void* W = a.packed + a.lay.w_off[l];
    // the bias of the wave's own neurons: fetched before the products, moved to LDS after
    // the first one, so that no epilogue waits on a global load queued behind weight blocks
    constexpr int kNW = WIDTH / WAVES;            // neurons per wave
    constexpr int kBL = (kNW + 63) / 64;          // bias values per lane
    float bv[kBL];
    {
      const float* bl = bias_all + (int64_t)l * WIDTH + wave * kNW;
      const int el = fresh_lane();
#pragma unroll
      for (int j = 0; j < kBL; ++j)
        if (j * 64 + el < kNW) bv[j] = bl[j * 64 + el];
    }
    const float* bias = bsm;
    // Operand roles are swapped (weights as the first matrix-core operand): register group q
    // of tile (rt, t) holds neurons (tile0 + t) 32 + 8 q + 4 (lane / 32) + i, i < 4, of ray
    // rt 32 + lane % 32: 4 consecutive e4m3 results form one word, and regroup16 turns a
    // tile's four words into one 128-bit LDS write.
    // pass-0 e4m3 results, regrouped; kept as separate words, since aligned 4-register
    // tuples live across the second pass make the 1024-wide kernel spill ten times more
    uint32_t hold[kRT8][NTP][4];
    float hp0[kRT8], hp1[kRT8];
#pragma unroll
    for (int rt = 0; rt < kRT8; ++rt) { hp0[rt] = 0.f; hp1[rt] = 0.f; }
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int tile0 = wave * NTW + p * NTP;
      // issue priority: pass 0's products above pass 1's, both above the epilogues.  Of the
      // two waves of a SIMD, the one that takes the matrix cores first (the older) would
      // otherwise also take them back for its pass 1 while the other is still in its pass 0,
      // leaving the other's epilogues with nothing to overlap; this way the waves alternate.
      if (p == 0)
        __builtin_amdgcn_s_setprio(3);
      else
        __builtin_amdgcn_s_setprio(2);
      f32x16 acc[kRT8][NTP];
#pragma unroll
      for (int rt = 0; rt < kRT8; ++rt)
#pragma unroll
        for (int t = 0; t < NTP; ++t) acc[rt][t] = f32x16{};
      if (l == 0) {
        gemm_l1<NTP>(acc, G, W, a.lay.k1 / 16, tile0, lane, WIDTH);
      } else if constexpr (WAVES == 8) {
        // pass 0 finds its first weight blocks already issued (end of the previous layer)
        if (p == 1) preload8<NTP, WIDTH / 64>(ring, W, tile0, lane, WIDTH);
        gemm_f8_stream<NTP, LDX, WIDTH / 64>(acc, X, W, tile0, lane, WIDTH, ring);
      } else {
        gemm_f8<NTP, LDX, WIDTH / 64>(acc, X, W, tile0, lane, WIDTH);
      }
      // the next layer's first weight blocks do not depend on this layer's output: issue them
      // before the epilogue (after the last layer, a harmless re-read of its own blocks)
      if (WAVES == 8 && p == 1)
        preload8<NTP, WIDTH / 64>(ring, a.packed + a.lay.w_off[last ? l : l + 1], wave * NTW, lane, WIDTH);
      __builtin_amdgcn_s_setprio(0);
      if (p == 0) {
        const int el = fresh_lane();
#pragma unroll
        for (int j = 0; j < kBL; ++j)
          if (j * 64 + el < kNW) bsm[wave * kNW + j * 64 + el] = bv[j];
      }
      // the heads read no tile; a layer feeding another writes the tile only after its pass-1
      // outputs are rounded (below), so that a wave waiting for the others has that work done
      if (p == 1 && last) __syncthreads();
      const int el = fresh_lane();
      // the two epilogues are separate uniform branches, so that neither carries the
      // other's tests inside its unrolled loops
      if (last) {
        // heads from the fp32 output of the last hidden layer (a single-output network reads
        // head 0 twice and drops the second sum)
        const float* hw1 = a.n_out > 1 ? hw + WIDTH : hw;
#pragma unroll
        for (int t = 0; t < NTP; ++t) {
          const int nb = (tile0 + t) * 32 + 4 * (el >> 5);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const f32x4 b4 = *reinterpret_cast<const f32x4*>(bias + nb + 8 * q);
            const f32x4 w0 = *reinterpret_cast<const f32x4*>(hw + nb + 8 * q);
            const f32x4 w1 = *reinterpret_cast<const f32x4*>(hw1 + nb + 8 * q);
#pragma unroll
            for (int rt = 0; rt < kRT8; ++rt) {
              f32x4 y;
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                y[i] = fmaxf(fmaf(acc[rt][t][4 * q + i], dq, b4[i]), 0.f);
                hp0[rt] = fmaf(w0[i], y[i], hp0[rt]);
                hp1[rt] = fmaf(w1[i], y[i], hp1[rt]);
              }
              if (MODE == kModeHidden) {
                const int64_t g = ray0 + rt * 32 + (el & 31);
                if (g < n_act) *reinterpret_cast<f32x4*>(a.out0 + g * WIDTH + nb + 8 * q) = y;
              }
            }
          }
        }
      } else {
        uint32_t hold1[kRT8][NTP][4];   // pass 1's rounded outputs, until the barrier
#pragma unroll
        for (int t = 0; t < NTP; ++t) {
          const int nb = (tile0 + t) * 32 + 4 * (el >> 5);
          uint32_t w[kRT8][4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            // relu(acc dq + b) / s_A,next in one rounding: the scales are powers of two, so
            // fma(acc, dq qn, b qn) is exactly qn fma(acc, dq, b)
            const f32x4 b4 = *reinterpret_cast<const f32x4*>(bias + nb + 8 * q);
            f32x4 bq;
#pragma unroll
            for (int i = 0; i < 4; ++i) bq[i] = b4[i] * qn;
#pragma unroll
            for (int rt = 0; rt < kRT8; ++rt) {
              float y[4];
#pragma unroll
              for (int i = 0; i < 4; ++i)   // ReLU and saturation at 448 in one clamp
                y[i] = __builtin_amdgcn_fmed3f(fmaf(acc[rt][t][4 * q + i], dqn, bq[i]), 0.f, 448.f);
              w[rt][q] = pack_e4m3(y[0], y[1], y[2], y[3]);
            }
          }
#pragma unroll
          for (int rt = 0; rt < kRT8; ++rt) {
            const i32x4 v = regroup16(w[rt]);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              if (p == 0)
                hold[rt][t][q] = (uint32_t)v[q];
              else
                hold1[rt][t][q] = (uint32_t)v[q];
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        if (p == 1) {
          __syncthreads();   // every wave is done reading this layer's input
#pragma unroll
          for (int rt = 0; rt < kRT8; ++rt)
#pragma unroll
            for (int t = 0; t < NTP; ++t) {
              uint8_t* row = X + (rt * 32 + (el & 31)) * LDX + 16 * (el >> 5);
              *reinterpret_cast<i32x4*>(row + (wave * NTW + t) * 32) =
                  i32x4{(int)hold[rt][t][0], (int)hold[rt][t][1], (int)hold[rt][t][2], (int)hold[rt][t][3]};
              *reinterpret_cast<i32x4*>(row + (wave * NTW + NTP + t) * 32) =
                  i32x4{(int)hold1[rt][t][0], (int)hold1[rt][t][1], (int)hold1[rt][t][2], (int)hold1[rt][t][3]};
            }
        }
      }
    }
    if (last) {
      const int el = fresh_lane();
#pragma unroll
      for (int rt = 0; rt < kRT8; ++rt) {
        const float s0 = hp0[rt] + __shfl_xor(hp0[rt], 32);
        const float s1 = hp1[rt] + __shfl_xor(hp1[rt], 32);
        if (el < 32) {
          headp[wave][rt * 32 + el][0] = s0;
          headp[wave][rt * 32 + el][1] = s1;
        }
      }
    }
    __syncthreads();
  }

  for (int r = threadIdx.x; r < kM8; r += WAVES * 64) {
    const int64_t g = ray0 + r;
    if (g >= n_act) continue;
    float z0 = hb[0], z1 = a.n_out > 1 ? hb[1] : 0.f;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) { z0 += headp[w][r][0]; z1 += headp[w][r][1]; }
    if (MODE == kModeQuery) {
      a.out0[g] = softplusf_(z0);
      a.out1[g] = sigmoidf_(z1);
    } else if (MODE == kModeSdf) {
      a.out0[g] = z0;
    } else if (MODE == kModeTrace) {
      trace_update(a, a.idx[g], z0);
    }
  }
}

template <int WIDTH>
static hipError_t launch8_t(const FwdArgs& a, int64_t n_tiles, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  constexpr int QW = WIDTH >= 512 ? 8 : 4;   // two waves per SIMD where each keeps >= 2 tiles per pass
  const dim3 grid((unsigned)n_tiles), block(QW * 64);
  switch (a.mode) {
    case kModeQuery: hipLaunchKernelGGL((fwd8_kernel<WIDTH, kModeQuery, QW>), grid, block, 0, st, a); break;
    case kModeSdf: hipLaunchKernelGGL((fwd8_kernel<WIDTH, kModeSdf, QW>), grid, block, 0, st, a); break;
    case kModeTrace: hipLaunchKernelGGL((fwd8_kernel<WIDTH, kModeTrace, QW>), grid, block, 0, st, a); break;
    case kModeHidden: hipLaunchKernelGGL((fwd8_kernel<WIDTH, kModeHidden, QW>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_forward8(const ddf_net_desc& d, const FwdArgs& a, int64_t n_items, hipStream_t st) {
  const int64_t tiles = (n_items + kM8 - 1) / kM8;
  switch (d.width) {
    case 256: return launch8_t<256>(a, tiles, st);
    case 512: return launch8_t<512>(a, tiles, st);
    case 1024: return launch8_t<1024>(a, tiles, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace ddf
