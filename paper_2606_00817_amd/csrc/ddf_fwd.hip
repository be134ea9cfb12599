// Fused forward pass of the DDF / SDF MLP on the gfx950 matrix cores.
//
// One workgroup (4 waves, one per SIMD) owns a tile of M rays for the whole
// network.  The tile's activations stay in LDS ([M][width] in the operand
// type) for all layers; each wave owns width/4 output neurons and streams
// the matching pre-arranged weight blocks straight from global memory into
// registers (every weight element is read once per workgroup and used for
// all M rays).  Products run on MFMA with fp32 accumulation:
//   fp32: v_mfma_f32_32x32x2_f32, M = 32
//   bf16: v_mfma_f32_32x32x16_bf16, M = 64
// The epilogue adds the bias, applies ReLU, rounds to the next layer's
// operand type and writes the tile back into LDS.  The last layer feeds the
// two fp32 heads directly from the accumulators (cross-lane and cross-wave
// reductions in a fixed order), so the heads always read the unrounded last
// hidden layer.  The sinusoidal encoding is computed in registers into LDS
// at the start of the tile; it never touches HBM.
#include "ddf_chain.h"
#include "ddf_fwd.h"
#include "ddf_internal.h"

namespace ddf {

// Epilogue of a layer computed with swapped operand roles (query modes): register group q of
// tile (rt, t) holds neurons (nt0 + t) 32 + 8 q + 4 (lane / 32) + i, i < 4, of ray
// rt 32 + lane % 32.  Bias (read from the wave's LDS copy) + ReLU, then either one vector write of the 4 values into the
// LDS tile, or (last layer) the heads' partial dot products: one value per ray and head per
// lane, the two lane halves added, then written per wave for the fixed-order final sum.
template <class P, int WIDTH, int MODE, int WAVES>
__device__ inline void epilogue_t(const FwdArgs& a,
                                  f32x16 (&acc)[Chain<P, WIDTH, WAVES>::RT][Chain<P, WIDTH, WAVES>::NT],
                                  typename P::E* X, float (*headp)[Chain<P, WIDTH, WAVES>::M][2],
                                  const float* bias, int l, int64_t ray0, int64_t n_act, int nt0, int lane,
                                  int wave) {
  using C = Chain<P, WIDTH, WAVES>;
  using E = typename P::E;
  constexpr int RT = C::RT, NT = C::NT, LDX = C::LDX;
  const float* hw = reinterpret_cast<const float*>(a.packed + a.lay.head_w_off);
  const bool last = (l + 1 == a.n_hidden);
  float hp0[RT], hp1[RT], mx = 0.f;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) { hp0[rt] = 0.f; hp1[rt] = 0.f; }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int nb = (nt0 + t) * 32 + 4 * (lane >> 5);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f32x4 b4 = *reinterpret_cast<const f32x4*>(bias + nb + 8 * q);
      f32x4 w0 = {}, w1 = {};
      if (last) {
        w0 = *reinterpret_cast<const f32x4*>(hw + nb + 8 * q);
        if (a.n_out > 1) w1 = *reinterpret_cast<const f32x4*>(hw + WIDTH + nb + 8 * q);
      }
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        f32x4 y;
#pragma unroll
        for (int i = 0; i < 4; ++i) y[i] = fmaxf(acc[rt][t][4 * q + i] + b4[i], 0.f);
        if (MODE == kModeHidden && last) {
          const int64_t g = ray0 + rt * 32 + (lane & 31);
          if (g < n_act) *reinterpret_cast<f32x4*>(a.out0 + g * WIDTH + nb + 8 * q) = y;
        }
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
          *reinterpret_cast<V4<E>*>(X + (rt * 32 + (lane & 31)) * LDX + nb + 8 * q) = yv;
          if (MODE == kModeCalib && ray0 + rt * 32 + (lane & 31) < n_act)
            mx = fmaxf(mx, fmaxf(fmaxf(y[0], y[1]), fmaxf(y[2], y[3])));
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  if (last) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const float s0 = hp0[rt] + __shfl_xor(hp0[rt], 32);   // the other 128 neurons of this tile
      const float s1 = hp1[rt] + __shfl_xor(hp1[rt], 32);
      if (lane < 32) {
        headp[wave][rt * 32 + lane][0] = s0;
        headp[wave][rt * 32 + lane][1] = s1;
      }
    }
  }
  if (MODE == kModeCalib && !last) {
    for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if (lane == 0) atomicMax(a.amax + l, __float_as_uint(mx));
  }
  __syncthreads();
}

template <class P, int WIDTH, int MODE, int WAVES>
__global__ __launch_bounds__(WAVES * 64, 1) void fwd_kernel(FwdArgs a) {
  using C = Chain<P, WIDTH, WAVES>;
  using E = typename P::E;
  constexpr int M = C::M, RT = C::RT, NT = C::NT, LDX = C::LDX;
  __shared__ __attribute__((aligned(16))) E X[C::XSIZE];
  __shared__ float headp[WAVES][M][2];
  // query modes: the current layer's bias, each wave's own neurons copied in by that wave
  __shared__ __attribute__((aligned(16))) float bsm[WIDTH];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int64_t ray0 = (int64_t)blockIdx.x * M;
  if (MODE == kModeTrace && ray0 >= *a.count) return;   // uniform: no active rays left here
  const int64_t n_act = MODE == kModeTrace ? (int64_t)*a.count : a.n;
  FwdArgs aa = a;
  aa.n = n_act;

  if constexpr (MODE == kModeRecompute)
    load_tile<E, M, LDX, WIDTH>(a, ray0, X);
  else
    encode_tile<E, M, LDX, MODE>(aa, ray0, X);
  __syncthreads();

  const float* bias_all = reinterpret_cast<const float*>(a.packed + a.lay.b_off);
  const float* hw = reinterpret_cast<const float*>(a.packed + a.lay.head_w_off);
  const float* hb = reinterpret_cast<const float*>(a.packed + a.lay.head_b_off);
  const int nt0 = wave * NT;
  typename C::Ring ring;

  for (int l = a.l_begin; l < a.l_end; ++l) {
    const int K = l == 0 ? a.lay.k1 : WIDTH;
    const void* W = a.packed + a.lay.w_off[l];
    f32x16 acc[RT][NT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[rt][t] = f32x16{};
    constexpr bool kTrans = MODE != kModeTrain && MODE != kModeRecompute;
    // query modes: fetch the bias of the wave's own neurons now (into registers, moved to LDS
    // after the product), so that the epilogue never waits on a global load queued behind the
    // next layer's weight blocks
    constexpr int kNW = WIDTH / WAVES;            // neurons per wave
    constexpr int kBL = (kNW + 63) / 64;          // bias values per lane
    float bv[kBL];
    if constexpr (kTrans) {
      const float* bl = bias_all + (int64_t)l * WIDTH + nt0 * 32;
#pragma unroll
      for (int j = 0; j < kBL; ++j)
        if (j * 64 + lane < kNW) bv[j] = bl[j * 64 + lane];
    }
    // query modes fetch a layer's first weight blocks during the previous layer's last
    // products (they do not depend on its output; after the last layer a harmless re-read of
    // its own first blocks); the training epilogue has no registers to spare for them
    const bool more = l + 1 < a.l_end;
    const void* Wn = more ? a.packed + a.lay.w_off[l + 1] : W;
    const int KBn = more ? WIDTH / P::KBLK : K / P::KBLK;
    if (l == 0) {
      C::preload(ring, W, K / P::KBLK, nt0, lane);
      C::template gemm<0, kTrans, kTrans>(acc, X, W, K / P::KBLK, nt0, lane, ring, Wn, KBn);
    } else {
      if (!kTrans) C::preload(ring, W, WIDTH / P::KBLK, nt0, lane);
      C::template gemm<WIDTH / P::KBLK, kTrans, kTrans>(acc, X, W, K / P::KBLK, nt0, lane, ring, Wn, KBn);
    }
    if constexpr (kTrans) {
#pragma unroll
      for (int j = 0; j < kBL; ++j)
        if (j * 64 + lane < kNW) bsm[nt0 * 32 + j * 64 + lane] = bv[j];
    }
    __syncthreads();   // every wave is done reading X
    if constexpr (kTrans) {
      epilogue_t<P, WIDTH, MODE, WAVES>(a, acc, X, headp, bsm, l, ray0, n_act, nt0, lane, wave);
      continue;
    }

    const float* bias = bias_all + (int64_t)l * WIDTH;
    const bool last = (l + 1 == a.n_hidden);
    E* slab = reinterpret_cast<E*>(a.hst[l + 1]);   // H_(l+1) store, or null: not kept
    constexpr int kMD = (RT * NT * 16 + 31) / 32;   // mask-bit dwords per lane
    uint32_t* mw = nullptr;
    if (kSpreadStores<P, WAVES> && a.mbits)
      mw = a.mbits + ((((int64_t)(l + 1) * gridDim.x + blockIdx.x) * WAVES + wave) * kMD) * 64 + lane;
    uint32_t mb[kMD] = {};   // bit (rt NT + t) 16 + v: stored as soon as a dword is complete
    // every global load of the epilogue is issued before its first store (a load queued behind
    // stores waits for them as well)
    float bvs[NT], w0s[NT], w1s[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int n = (nt0 + t) * 32 + (lane & 31);
      bvs[t] = bias[n];
      w0s[t] = last ? hw[n] : 0.f;
      w1s[t] = last && a.n_out > 1 ? hw[WIDTH + n] : 0.f;
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      float hp0[16], hp1[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) { hp0[v] = 0.f; hp1[v] = 0.f; }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int n = (nt0 + t) * 32 + (lane & 31);
        const float bv = bvs[t];
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[rt][t][v] = fmaxf(acc[rt][t][v] + bv, 0.f);
        if constexpr (kSpreadStores<P, WAVES>) {
          uint32_t bits = 0u;
#pragma unroll
          for (int v = 0; v < 16; ++v) bits |= (acc[rt][t][v] > 0.f ? 1u : 0u) << v;
          const int p = (rt * NT + t) * 16;
          mb[p >> 5] |= bits << (p & 31);
        }
        if (last) {
          const float w0 = w0s[t];
          const float w1 = w1s[t];
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            hp0[v] = fmaf(w0, acc[rt][t][v], hp0[v]);
            hp1[v] = fmaf(w1, acc[rt][t][v], hp1[v]);
          }
        } else {
#pragma unroll
          for (int v = 0; v < 16; ++v) X[(rt * 32 + acc_row(v, lane)) * LDX + n] = (E)acc[rt][t][v];
          if (MODE == kModeCalib) {
            float m = 0.f;
#pragma unroll
            for (int v = 0; v < 16; ++v)
              if (ray0 + rt * 32 + acc_row(v, lane) < n_act) m = fmaxf(m, acc[rt][t][v]);
            for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
            if (lane == 0) atomicMax(a.amax + l, __float_as_uint(m));
          }
        }
        if (slab) {
          if constexpr (sizeof(E) == 2) {
            // blocks q, q + 1 paired across the lane halves: one 16-byte store per lane each
#pragma unroll
            for (int q = 0; q < 4; q += 2) {
              bf16x4 h0, h1;
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                h0[i] = (__bf16)acc[rt][t][4 * q + i];
                h1[i] = (__bf16)acc[rt][t][4 * q + 4 + i];
              }
              const i32x4 w = pair_blocks(h0, h1);
              const int64_t g0 = ray0 + rt * 32 + 8 * (q + (lane >> 5));
              __builtin_nontemporal_store(w, reinterpret_cast<i32x4*>(slab + ((g0 >> 3) * WIDTH + n) * 8));
            }
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int64_t g0 = ray0 + rt * 32 + 8 * q;   // 8-ray block of registers 4q..4q+3
              V4<E> hv;
#pragma unroll
              for (int i = 0; i < 4; ++i) hv[i] = (E)acc[rt][t][4 * q + i];
              *reinterpret_cast<V4<E>*>(slab + ((g0 >> 3) * WIDTH + n) * 8 + 4 * (lane >> 5)) = hv;
            }
          }
        }
        __builtin_amdgcn_sched_barrier(0);   // keep the epilogue tile by tile (no hoisting)
      }
      if constexpr (kSpreadStores<P, WAVES>) {
        if (mw) {
          if constexpr (NT >= 2) {
#pragma unroll
            for (int jj = 0; jj < NT / 2; ++jj) mw[(rt * (NT / 2) + jj) * 64] = mb[rt * (NT / 2) + jj];
          } else if (rt == RT - 1) {
#pragma unroll
            for (int jj = 0; jj < kMD; ++jj) mw[jj * 64] = mb[jj];
          }
        }
      }
      if (last) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          hp0[v] = wave_sum32(hp0[v]);
          hp1[v] = wave_sum32(hp1[v]);
        }
        if ((lane & 31) == 0) {
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int r = rt * 32 + acc_row(v, lane);
            headp[wave][r][0] = hp0[v];
            headp[wave][r][1] = hp1[v];
          }
        }
      }
    }
    __syncthreads();
  }

  // a recomputation (a layer range short of the heads) has the kept activations as output
  if (MODE == kModeRecompute || a.l_end != a.n_hidden) return;
  for (int r = threadIdx.x; r < M; r += WAVES * 64) {
    const int64_t g = ray0 + r;
    if (g >= n_act) continue;
    float z0 = hb[0], z1 = a.n_out > 1 ? hb[1] : 0.f;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) { z0 += headp[w][r][0]; z1 += headp[w][r][1]; }
    switch (MODE) {
      case kModeQuery:
      case kModeCalib:
        a.out0[g] = softplusf_(z0);
        a.out1[g] = sigmoidf_(z1);
        break;
      case kModeTrain:
        a.out0[g] = z0;
        if (a.n_out > 1) a.out1[g] = z1;
        break;
      case kModeSdf:
        a.out0[g] = z0;
        break;
      case kModeHidden:
        break;
      default:
        trace_update(a, a.idx[g], z0);
        break;
    }
  }
}

// Persistent sphere tracing (the lane-refill form of the baseline, Sec. IV-D): a grid of one
// workgroup per CU, each owning the M ray slots of one tile for the whole trace.  Per
// iteration a workgroup refills its empty slots from the pool (one atomic per workgroup),
// evaluates the SDF network at p = x + t d for every slot (an empty slot computes on zeros and
// is ignored), and advances each ray by the same rule as the step-synchronous trace: |s| <
// hit_eps is a hit (t kept), else t += s, and the ray leaves its slot once t > t_max or after
// max_steps evaluations.  A ray's evaluation does not depend on which slot or tile holds it,
// so t, hit and steps equal the step-synchronous trace's bit for bit.  Every workgroup leaves
// the loop when the pool is exhausted and its slots are empty, so the grid always drains.
template <class P, int WIDTH, int WAVES>
__global__ __launch_bounds__(WAVES * 64, 1) void pool_trace_kernel(FwdArgs a) {
  using C = Chain<P, WIDTH, WAVES>;
  using E = typename P::E;
  constexpr int M = C::M, NT = C::NT, LDX = C::LDX;
  __shared__ __attribute__((aligned(16))) E X[C::XSIZE];
  __shared__ float headp[WAVES][M][2];
  __shared__ __attribute__((aligned(16))) float bsm[WIDTH];
  __shared__ int32_t slot[M];        // ray held by each slot, -1 = empty
  __shared__ int32_t slot_steps[M];  // evaluations that ray has had
  __shared__ int32_t live;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nt0 = wave * NT;
  const float* bias_all = reinterpret_cast<const float*>(a.packed + a.lay.b_off);
  const float* hb = reinterpret_cast<const float*>(a.packed + a.lay.head_b_off);
  for (int r = threadIdx.x; r < M; r += WAVES * 64) slot[r] = -1;
  FwdArgs aa = a;
  aa.idx = slot;
  aa.n = M;
  typename C::Ring ring;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) {
      int empty = 0;
      for (int r = 0; r < M; ++r) empty += slot[r] < 0;
      // past the end of the pool nothing is claimed, so the counter stays below n + M x grid
      const unsigned long long seen = __hip_atomic_load(a.pool, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int64_t next = (empty && seen < (unsigned long long)a.n) ? (int64_t)atomicAdd(a.pool, (unsigned long long)empty)
                                                              : a.n;
      int n_live = 0;
      for (int r = 0; r < M; ++r) {
        if (slot[r] < 0 && next < a.n) {
          slot[r] = (int32_t)next++;
          slot_steps[r] = 0;
        }
        n_live += slot[r] >= 0;
      }
      live = n_live;
    }
    __syncthreads();
    if (live == 0) break;   // uniform: the pool is exhausted and every slot is empty
    encode_tile<E, M, LDX, kModePool>(aa, 0, X);
    __syncthreads();
    for (int l = 0; l < a.n_hidden; ++l) {
      const int K = l == 0 ? a.lay.k1 : WIDTH;
      const void* W = a.packed + a.lay.w_off[l];
      f32x16 acc[C::RT][NT];
#pragma unroll
      for (int rt = 0; rt < C::RT; ++rt)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[rt][t] = f32x16{};
      constexpr int kNW = WIDTH / WAVES;
      constexpr int kBL = (kNW + 63) / 64;
      float bv[kBL];
      const float* bl = bias_all + (int64_t)l * WIDTH + nt0 * 32;
#pragma unroll
      for (int j = 0; j < kBL; ++j)
        if (j * 64 + lane < kNW) bv[j] = bl[j * 64 + lane];
      // the next layer's first blocks come with this layer's last products (after the last
      // layer a harmless re-read of its own first blocks)
      const bool more = l + 1 < a.n_hidden;
      const void* Wn = more ? a.packed + a.lay.w_off[l + 1] : W;
      const int KBn = more ? WIDTH / P::KBLK : K / P::KBLK;
      if (l == 0) {
        C::preload(ring, W, K / P::KBLK, nt0, lane);
        C::template gemm<0, true, true>(acc, X, W, K / P::KBLK, nt0, lane, ring, Wn, KBn);
      } else {
        C::template gemm<WIDTH / P::KBLK, true, true>(acc, X, W, K / P::KBLK, nt0, lane, ring, Wn, KBn);
      }
#pragma unroll
      for (int j = 0; j < kBL; ++j)
        if (j * 64 + lane < kNW) bsm[nt0 * 32 + j * 64 + lane] = bv[j];
      __syncthreads();
      epilogue_t<P, WIDTH, kModePool, WAVES>(a, acc, X, headp, bsm, l, 0, M, nt0, lane, wave);
    }
    for (int r = threadIdx.x; r < M; r += WAVES * 64) {
      const int32_t id = slot[r];
      if (id < 0) continue;
      float z0 = hb[0];
#pragma unroll
      for (int w = 0; w < WAVES; ++w) z0 += headp[w][r][0];
      const int st = slot_steps[r] + 1;
      slot_steps[r] = st;
      if (a.steps) a.steps[id] = st;
      if (fabsf(z0) < a.hit_eps) {
        a.hit[id] = 1;
        slot[r] = -1;
        continue;
      }
      const float tn = a.t_state[id] + z0;
      a.t_state[id] = tn;
      if (tn > a.t_max || st >= a.max_steps) slot[r] = -1;
    }
  }
}

hipError_t launch_pool_trace(const ddf_net_desc& d, const FwdArgs& a, int n_wg, hipStream_t st) {
  const dim3 grid((unsigned)n_wg), block(8 * 64);
  if (d.precision == DDF_FP32) {
    switch (d.width) {
      case 256: hipLaunchKernelGGL((pool_trace_kernel<PF32, 256, 8>), grid, block, 0, st, a); break;
      case 512: hipLaunchKernelGGL((pool_trace_kernel<PF32, 512, 8>), grid, block, 0, st, a); break;
      case 1024: hipLaunchKernelGGL((pool_trace_kernel<PF32, 1024, 8>), grid, block, 0, st, a); break;
      default: return hipErrorInvalidValue;
    }
  } else if (d.precision == DDF_BF16) {
    switch (d.width) {
      case 256: hipLaunchKernelGGL((pool_trace_kernel<PBF16, 256, 8>), grid, block, 0, st, a); break;
      case 512: hipLaunchKernelGGL((pool_trace_kernel<PBF16, 512, 8>), grid, block, 0, st, a); break;
      case 1024: hipLaunchKernelGGL((pool_trace_kernel<PBF16, 1024, 8>), grid, block, 0, st, a); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// 8 waves (two per SIMD, 128 neurons each) when the width allows it, so that one wave's
// matrix products cover the other's load and LDS latencies.
template <class P, int WIDTH>
static hipError_t launch_t(const FwdArgs& a, int64_t n_tiles, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  constexpr int QW = WIDTH >= 256 ? 8 : 4;
  const dim3 grid((unsigned)n_tiles), bq(QW * 64);
  switch (a.mode) {
    case kModeQuery: hipLaunchKernelGGL((fwd_kernel<P, WIDTH, kModeQuery, QW>), grid, bq, 0, st, a); break;
    case kModeTrain: hipLaunchKernelGGL((fwd_kernel<P, WIDTH, kModeTrain, QW>), grid, bq, 0, st, a); break;
    case kModeSdf: hipLaunchKernelGGL((fwd_kernel<P, WIDTH, kModeSdf, QW>), grid, bq, 0, st, a); break;
    case kModeCalib: hipLaunchKernelGGL((fwd_kernel<P, WIDTH, kModeCalib, QW>), grid, bq, 0, st, a); break;
    case kModeRecompute:
      hipLaunchKernelGGL((fwd_kernel<P, WIDTH, kModeRecompute, QW>), grid, bq, 0, st, a);
      break;
    case kModeHidden: hipLaunchKernelGGL((fwd_kernel<P, WIDTH, kModeHidden, QW>), grid, bq, 0, st, a); break;
    default: hipLaunchKernelGGL((fwd_kernel<P, WIDTH, kModeTrace, QW>), grid, bq, 0, st, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_forward(const ddf_net_desc& d, const FwdArgs& a, int64_t n_items,
                          hipStream_t st) {
  const Geo g = geo_of(d.precision);
  const int64_t tiles = (n_items + g.rays_per_wg - 1) / g.rays_per_wg;
  if (d.precision == DDF_FP32) {
    switch (d.width) {
      case 128: return launch_t<PF32, 128>(a, tiles, st);
      case 256: return launch_t<PF32, 256>(a, tiles, st);
      case 512: return launch_t<PF32, 512>(a, tiles, st);
      case 1024: return launch_t<PF32, 1024>(a, tiles, st);
    }
  } else if (d.precision == DDF_FP8_E4M3) {
    return launch_forward8(d, a, n_items, st);
  } else if (d.precision == DDF_BF16) {
    switch (d.width) {
      case 128: return launch_t<PBF16, 128>(a, tiles, st);
      case 256: return launch_t<PBF16, 256>(a, tiles, st);
      case 512: return launch_t<PBF16, 512>(a, tiles, st);
      case 1024: return launch_t<PBF16, 1024>(a, tiles, st);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace ddf
