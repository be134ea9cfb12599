// The fused layer-chain building blocks shared by the forward and backward kernels.
#pragma once
#include "ddf_internal.h"

namespace ddf {

struct PF32 {
  using E = float;
  using AFrag = f32x4;
  using BFrag = f32x4;
  static constexpr int M = 32;
  static constexpr int KBLK = 8;
  static __device__ inline void mma(f32x16& c, const AFrag& a, const BFrag& b) {
    // k is permuted inside the block: step s uses k = 4 * (lane / 32) + s
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0], b[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1], b[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[2], b[2], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[3], b[3], c, 0, 0, 0);
  }
};

struct PBF16 {
  using E = __bf16;
  using AFrag = bf16x8;
  using BFrag = bf16x8;
  static constexpr int M = 64;
  static constexpr int KBLK = 16;
  static __device__ inline void mma(f32x16& c, const AFrag& a, const BFrag& b) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

template <class P, int WIDTH, int WAVES = kWaves>
struct Chain {
  using E = typename P::E;
  using AFrag = typename P::AFrag;
  using BFrag = typename P::BFrag;
  static constexpr int M = P::M;
  static constexpr int RT = M / 32;                  // 32-ray tiles per workgroup
  static constexpr int NT = WIDTH / 32 / WAVES;      // 32-neuron tiles per wave
  static constexpr int LDX = WIDTH + 16 / (int)sizeof(E);  // padded LDS row (elements)
  // LDS tile size in elements: M rows of LDX plus one more A block, so the read of the block
  // after the last one (prefetched, never used) stays inside the allocation
  static constexpr int XSIZE = M * LDX + 16;

  static __device__ inline BFrag load_b(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
    return __builtin_bit_cast(BFrag, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
  }

  // The ring of weight blocks a wave keeps in flight: four stages of NT blocks.
  struct Ring {
    BFrag b0[NT], b1[NT], b2[NT], b3[NT];
  };

  static __device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* W, int KB) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(W), (short)0, WIDTH * KB * 32, 0x00020000);
  }

  // Block (t, k) of the wave's tiles, at byte ((nt0 + t) KB + k) * 1 KiB + lane * 16 of the
  // layer: the per-lane part and (k mod 4) KiB go into the vector offset (the constant part
  // folds into the instruction's immediate), the wave-uniform tile and k / 4 part into the
  // scalar offset, so that a fully unrolled k loop needs one scalar offset per four blocks.
  static __device__ inline BFrag ld(__amdgpu_buffer_rsrc_t rs, int voff, int base, int tstride, int t, int k) {
    return load_b(rs, voff + (k & 3) * 1024, base + t * tstride + (k >> 2) * 4096);
  }

  // First three stages of a layer's weight blocks (issued ahead of time, e.g. before the
  // previous layer's epilogue).
  static __device__ inline void preload(Ring& r, const void* W, int KB, int nt0, int lane) {
    const __amdgpu_buffer_rsrc_t rs = rsrc(W, KB);
    const int voff = lane * 16, base = nt0 * KB * 1024, tstride = KB * 1024;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      r.b0[t] = ld(rs, voff, base, tstride, t, 0);
      r.b1[t] = ld(rs, voff, base, tstride, t, 1);
      r.b2[t] = ld(rs, voff, base, tstride, t, 2);
    }
  }

  // One quarter of the k loop, blocks k .. k + 3: before each block's products, the ring
  // load three blocks ahead and the LDS read of the next block's activations.  TAIL = false:
  // on a layer's last quarter these fall past the end (the weight loads are bounds-checked by
  // the buffer resource and return zeros, the LDS read stays in the tile's padding; neither
  // is used); TAIL = true, the layer's last quarter: its ring loads fetch blocks 0..2 of the
  // next layer (resource rsn, offsets basen + t tstriden) instead, and nothing is read past
  // the end.
  template <bool TRANS, bool TAIL>
  static __device__ inline void quarter(f32x16 (&acc)[RT][NT], AFrag (&a0)[RT], AFrag (&a1)[RT], const E* xrow,
                                        __amdgpu_buffer_rsrc_t rs, int voff, int base, int tstride, int k, Ring& r,
                                        __amdgpu_buffer_rsrc_t rsn, int basen, int tstriden) {
#pragma unroll
    for (int t = 0; t < NT; ++t) r.b3[t] = ld(rs, voff, base, tstride, t, k + 3);
    load_a(a1, xrow, k + 1);
    __builtin_amdgcn_sched_barrier(0);
    mma_all<TRANS>(acc, a0, r.b0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < NT; ++t)
      r.b0[t] = TAIL ? ld(rsn, voff, basen, tstriden, t, 0) : ld(rs, voff, base, tstride, t, k + 4);
    load_a(a0, xrow, k + 2);
    __builtin_amdgcn_sched_barrier(0);
    mma_all<TRANS>(acc, a1, r.b1);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < NT; ++t)
      r.b1[t] = TAIL ? ld(rsn, voff, basen, tstriden, t, 1) : ld(rs, voff, base, tstride, t, k + 5);
    load_a(a1, xrow, k + 3);
    __builtin_amdgcn_sched_barrier(0);
    mma_all<TRANS>(acc, a0, r.b2);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < NT; ++t)
      r.b2[t] = TAIL ? ld(rsn, voff, basen, tstriden, t, 2) : ld(rs, voff, base, tstride, t, k + 6);
    if (!TAIL) load_a(a0, xrow, k + 4);
    __builtin_amdgcn_sched_barrier(0);
    mma_all<TRANS>(acc, a1, r.b3);
    __builtin_amdgcn_sched_barrier(0);
  }

  // TRANS = false: acc[rt][t] = X_tile * W_tile^T (rows rays, columns neurons).
  // TRANS = true : acc[rt][t] = W_tile * X_tile^T (rows neurons, columns rays): the same
  //   operand blocks with their matrix-core roles swapped, so that each lane ends up with 4
  //   consecutive neurons of one ray per register group.
  // acc[rt][t] accumulates over the wave's neuron tile (nt0 + t) and all K inputs.  The weight
  // blocks of one layer are read through a buffer resource three blocks ahead in a ring of
  // four (the first three already issued by preload); KB is a multiple of 4.  The last
  // quarter has no blocks of this layer left to fetch: with NEXT its ring loads take blocks
  // 0..2 of the layer Wn (KBn blocks per tile) that follows, leaving the ring as preload(Wn)
  // would, issued during this layer's last products and with no address-unit cycles spent on
  // blocks past the end of the layer.  Without NEXT (the training kernels, whose epilogues
  // have no registers to spare for a ring held across them) the loop stays uniform and its
  // last loads fall past the end.  KBC > 0 fixes KB at compile time (hidden layers): the k
  // loop is then fully unrolled.
  template <int KBC, bool TRANS = false, bool NEXT = false>
  static __device__ inline void gemm(f32x16 (&acc)[RT][NT], const E* X, const void* W, int KB_rt,
                                     int nt0, int lane, Ring& r, const void* Wn = nullptr, int KBn = 0) {
    const int KB = KBC > 0 ? KBC : KB_rt;
    const __amdgpu_buffer_rsrc_t rs = rsrc(W, KB);
    const int voff = lane * 16, base = nt0 * KB * 1024, tstride = KB * 1024;
    const __amdgpu_buffer_rsrc_t rsn = rsrc(NEXT ? Wn : W, NEXT ? KBn : KB);
    const int basen = nt0 * KBn * 1024, tstriden = KBn * 1024;
    const E* xrow = X + (lane & 31) * LDX + (P::KBLK / 2) * (lane >> 5);
    AFrag a0[RT], a1[RT];
    load_a(a0, xrow, 0);
    if constexpr (!NEXT) {
#pragma unroll (KBC > 0 ? KBC / 4 : 1)
      for (int k = 0; k < KB; k += 4)
        quarter<TRANS, false>(acc, a0, a1, xrow, rs, voff, base, tstride, k, r, rsn, basen, tstriden);
    } else {
#pragma unroll (KBC > 4 ? KBC / 4 - 1 : 1)
      for (int k = 0; k < KB - 4; k += 4)
        quarter<TRANS, false>(acc, a0, a1, xrow, rs, voff, base, tstride, k, r, rsn, basen, tstriden);
      quarter<TRANS, true>(acc, a0, a1, xrow, rs, voff, base, tstride, KB - 4, r, rsn, basen, tstriden);
    }
  }

  static __device__ inline void load_a(AFrag (&av)[RT], const E* xrow, int k) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
      av[rt] = *reinterpret_cast<const AFrag*>(xrow + rt * 32 * LDX + k * P::KBLK);
  }

  template <bool TRANS>
  static __device__ inline void mma_all(f32x16 (&acc)[RT][NT], const AFrag (&av)[RT], const BFrag (&b)[NT]) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (TRANS)
          P::mma(acc[rt][t], b[t], av[rt]);
        else
          P::mma(acc[rt][t], av[rt], b[t]);
      }
  }
};

// Four consecutive elements of the operand type as one vector access.
template <class E> struct V4T;
template <> struct V4T<float> { using type = f32x4; };
template <> struct V4T<__bf16> { using type = bf16x4; };
template <class E> using V4 = typename V4T<E>::type;

// Row of the 32x32 accumulator held in register v by `lane`.
__device__ inline int acc_row(int v, int lane) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

// The accumulator layout holds, for one neuron, 4 consecutive rays of an 8-ray block per lane:
// rays 0-3 in lanes below 32, rays 4-7 in the others.  Two such blocks q, q + 1 (4 bf16 each)
// become whole blocks by one lane-half swap per dword: afterwards a lane below 32 holds block
// q's 8 rays and the others block q + 1's, the 16 contiguous bytes of one [rows / 8][cols][8]
// store entry (one full-width store per lane instead of two half-filled ones).
__device__ inline i32x4 pair_blocks(bf16x4 blk_q, bf16x4 blk_q1) {
  const i32x2 a = __builtin_bit_cast(i32x2, blk_q), b = __builtin_bit_cast(i32x2, blk_q1);
  const auto s0 = __builtin_amdgcn_permlane32_swap(a[0], b[0], false, false);
  const auto s1 = __builtin_amdgcn_permlane32_swap(a[1], b[1], false, false);
  return i32x4{(int)s0[0], (int)s1[0], (int)s0[1], (int)s1[1]};
}

// The inverse: a lane below 32 loaded block q's 8 rays, the others block q + 1's; returns the
// lane's 4 rays of block q (first) and of block q + 1 (second) in the accumulator layout.
__device__ inline void unpair_blocks(i32x4 c, bf16x4& blk_q, bf16x4& blk_q1) {
  const auto s0 = __builtin_amdgcn_permlane32_swap(c[0], c[2], false, false);
  const auto s1 = __builtin_amdgcn_permlane32_swap(c[1], c[3], false, false);
  blk_q = __builtin_bit_cast(bf16x4, i32x2{(int)s0[0], (int)s1[0]});
  blk_q1 = __builtin_bit_cast(bf16x4, i32x2{(int)s0[1], (int)s1[1]});
}

// Activation store layout [rows / 8][cols][8]: element (ray g, column c).
__device__ inline int64_t act_index(int64_t g, int c, int cols) { return ((g >> 3) * cols + c) * 8 + (g & 7); }

}  // namespace ddf
