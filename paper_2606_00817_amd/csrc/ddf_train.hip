// Training path of libddf: forward with kept activations, distillation loss,
// backward through the fused chain, weight gradients, Adam on the fp32 master.
//
// Workspace (one training batch of n rays, rows padded to R = n rounded up to 128; every
// store below is [R / 8][cols][8], in the operand type):
//   feat   the encoded features (k1_half columns)
//   hkeep  the kept hidden activations (width columns each): all of H_1 .. H_n, or with
//          activation recomputation every k layers only the checkpoints H_k, H_2k, .., H_n
//   hseg   (recomputation) k - 1 slabs for the recomputed layers of one segment
//   delta  dL/da_l: n slabs, or (recomputation) a ring of k + 1
//   z_t, z_xi, dz_t, dz_xi   fp32 [R] each
//   loss partials, scalars, and (when the caller passes none) the gradient buffer.
// Rows n .. R - 1 are computed from zero inputs with zero logit gradients, so they add
// nothing to any sum.
// Everything is deterministic: no floating-point atomics; every reduction has a
// fixed order.
#include "ddf_chain.h"
#include "ddf_fwd.h"
#include "ddf_train.h"

namespace ddf {

constexpr int kLossBlocks = 256;
constexpr int kHeadChunks = 64;   // ray chunks of the head-gradient reduction

struct TrainWs {
  int64_t R;                // padded rows
  int rc;                   // recomputation span k (0: every activation kept)
  int64_t feat, hkeep, hseg, delta;   // byte offsets of the stores
  int64_t zt, zx, dzt, dzx; // fp32 [R]
  int64_t lossp;            // [kLossBlocks][8] floats
  int64_t scal;             // 64 bytes of scalars
  int64_t headp;            // head-gradient partials [kHeadChunks][2][width + 2]
  int64_t grad;             // fp32 [P] (used when the caller passes no gradient buffer)
  int64_t dwpart;           // fp32 [8][P] weight-gradient partial sums of the ray ranges
  int64_t mbits;            // ReLU mask bits [n + 1][R / 64][8][dwords][64] (bf16 8-wave chain), or -1
  int64_t total;
  int esize;
};

// The recomputation span actually used: none when it would not save anything.
inline int recompute_span(const ddf_net_desc& d, int recompute_every) {
  return recompute_every > 0 && recompute_every < d.n_hidden ? recompute_every : 0;
}

inline TrainWs train_ws(const ddf_net_desc& d, int64_t batch, size_t nparams, int recompute_every) {
  const Layout L = make_layout(d);
  TrainWs w{};
  w.esize = d.precision == DDF_FP32 ? 4 : 2;
  w.R = (batch + 127) / 128 * 128;
  w.rc = recompute_span(d, recompute_every);
  const int n = d.n_hidden;
  const int kept = w.rc ? (n + w.rc - 1) / w.rc : n;
  const int64_t S = (int64_t)d.width * w.R * w.esize;
  int64_t off = 0;
  w.feat = off; off = align256(off + (int64_t)L.k1_half * w.R * w.esize);
  w.hkeep = off; off = align256(off + kept * S);
  w.hseg = off; off = align256(off + (w.rc ? w.rc - 1 : 0) * S);
  w.delta = off; off = align256(off + (w.rc ? w.rc + 1 : n) * S);
  w.zt = off; off = align256(off + 4 * w.R);
  w.zx = off; off = align256(off + 4 * w.R);
  w.dzt = off; off = align256(off + 4 * w.R);
  w.dzx = off; off = align256(off + 4 * w.R);
  w.lossp = off; off = align256(off + 32ll * kLossBlocks);
  w.scal = off; off = align256(off + 64);
  w.headp = off; off = align256(off + 4ll * kHeadChunks * 2 * (d.width + 2));
  w.grad = off; off = align256(off + 4 * (int64_t)nparams);
  w.dwpart = off; off = align256(off + 32 * (int64_t)nparams);
  if (d.precision == DDF_BF16 && d.width >= 256) {
    w.mbits = off;
    off = align256(off + 4ll * (n + 1) * (w.R / 64) * 8 * mask_dwords(d.width) * 64);
  } else {
    w.mbits = -1;
  }
  w.total = off;
  return w;
}

// Where each activation and delta lives.  h[0] the features, h[l] H_l (1-based); with
// recomputation H_l of a checkpoint (l a multiple of k, or l = n) has its own kept slab and
// the others share the segment slabs, slot (l - 1) mod k; delta_l sits in ring slot
// l mod (k + 1), so a segment's deltas and the one above it never collide.
struct TrainPtrs {
  uint8_t* h[kMaxLayers + 1];
  uint8_t* dl[kMaxLayers + 1];
  bool kept[kMaxLayers + 1];   // written by the training forward pass
  uint32_t* mbits;             // ReLU mask bits, or null
};

inline TrainPtrs train_ptrs(const ddf_net_desc& d, const TrainWs& w, uint8_t* ws) {
  TrainPtrs p{};
  const int n = d.n_hidden;
  const int64_t S = (int64_t)d.width * w.R * w.esize;
  p.mbits = w.mbits >= 0 ? reinterpret_cast<uint32_t*>(ws + w.mbits) : nullptr;
  p.h[0] = ws + w.feat;
  p.kept[0] = true;
  for (int l = 1; l <= n; ++l) {
    if (w.rc == 0) {
      p.h[l] = ws + w.hkeep + (l - 1) * S;
      p.kept[l] = true;
      p.dl[l] = ws + w.delta + (l - 1) * S;
    } else {
      p.kept[l] = l % w.rc == 0 || l == n;
      p.h[l] = p.kept[l] ? ws + w.hkeep + (int64_t)((l - 1) / w.rc) * S : ws + w.hseg + (int64_t)((l - 1) % w.rc) * S;
      p.dl[l] = ws + w.delta + (int64_t)(l % (w.rc + 1)) * S;
    }
  }
  return p;
}

// Float offsets of every layer's weight and bias in the master vector.
struct MasterOffsets {
  int64_t w[kMaxLayers + 1], b[kMaxLayers + 1];
};

inline MasterOffsets master_offsets(const ddf_net_desc& d) {
  MasterOffsets m{};
  const int64_t nf = (int64_t)d.n_in * (1 + 2 * d.n_freq);
  int64_t off = 0;
  for (int l = 0; l < d.n_hidden; ++l) {
    const int64_t fi = l == 0 ? nf : d.width;
    m.w[l] = off; off += fi * d.width;
    m.b[l] = off; off += d.width;
  }
  m.w[d.n_hidden] = off; off += (int64_t)d.n_out * d.width;
  m.b[d.n_hidden] = off;
  return m;
}

// ------------------------------------------------------------------ loss

// Neumaier compensated accumulation: s + c carries the running sum.
__device__ inline void kahan_add(float& s, float& c, float x) {
  const float t = s + x;
  c += fabsf(s) >= fabsf(x) ? (s - t) + x : (x - t) + s;
  s = t;
}

// Fixed-order reduction of the block's kThreads rows of red: row t absorbs row t + stride for
// stride = kThreads / 2 .. 1.  Column pairs (2j, 2j + 1), j < NP, are (sum, compensation) and
// merge as a compensated sum; the other columns add plainly.  Row 0 ends with the block's
// total.  Called by all kThreads threads of the block, after each has written its row.
template <int NC, int NP>
__device__ inline void tree_sum(float (*red)[NC]) {
  const int t = threadIdx.x;
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    __syncthreads();
    if (t < st) {
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        float sj = red[t][2 * j], cj = red[t][2 * j + 1];
        kahan_add(sj, cj, red[t + st][2 * j]);
        red[t][2 * j] = sj;
        red[t][2 * j + 1] = cj + red[t + st][2 * j + 1];
      }
#pragma unroll
      for (int j = 2 * NP; j < NC; ++j) red[t][j] += red[t + st][j];
    }
  }
  __syncthreads();
}

static_assert(kLossBlocks == kThreads, "the final loss reduction gives each block partial a thread");

struct LossArgs {
  const float* zt; const float* zx; const float* tgt; const uint8_t* hit;
  int64_t n, R;
  float* partial;     // [kLossBlocks][8]
  float* scal;        // [0] 1 / n_hit, [1] n_hit
  float* loss_out;    // [3] total, l1, bce
  float* dzt; float* dzx;
  float bce_weight, clamp;
};

// Per-block compensated sums of the L1 term, the BCE term and the hit count.
__global__ void loss_partial_kernel(LossArgs a) {
  float l1 = 0.f, l1c = 0.f, bce = 0.f, bcec = 0.f, hits = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)kLossBlocks * blockDim.x) {
    const float y = a.hit[i] ? 1.f : 0.f;
    const float z = a.zx[i];
    kahan_add(bce, bcec, softplusf_(z) - y * z);
    if (a.hit[i]) {
      const float u = fabsf(softplusf_(a.zt[i]) - a.tgt[i]);
      kahan_add(l1, l1c, u != u ? u : fminf(u, a.clamp));   // a NaN error stays NaN
      hits += 1.f;
    }
  }
  __shared__ float red[kThreads][5];
  red[threadIdx.x][0] = l1; red[threadIdx.x][1] = l1c;
  red[threadIdx.x][2] = bce; red[threadIdx.x][3] = bcec; red[threadIdx.x][4] = hits;
  tree_sum<5, 2>(red);
  if (threadIdx.x == 0) {
    float* p = a.partial + blockIdx.x * 8;
#pragma unroll
    for (int j = 0; j < 5; ++j) p[j] = red[0][j];
  }
}

// One block of kThreads threads, one per block partial.
__global__ void loss_final_kernel(LossArgs a) {
  __shared__ float red[kThreads][5];
  const float* p = a.partial + threadIdx.x * 8;
#pragma unroll
  for (int j = 0; j < 5; ++j) red[threadIdx.x][j] = p[j];
  tree_sum<5, 2>(red);
  if (threadIdx.x != 0) return;
  const float s0 = red[0][0], c0 = red[0][1], s1 = red[0][2], c1 = red[0][3], h = red[0][4];
  const float l1 = h > 0.f ? (s0 + c0) / h : 0.f;
  const float bce = a.n > 0 ? (s1 + c1) / (float)a.n : 0.f;
  a.scal[0] = h > 0.f ? 1.f / h : 0.f;
  a.scal[1] = h;
  if (a.loss_out) {
    a.loss_out[0] = l1 + a.bce_weight * bce;
    a.loss_out[1] = l1;
    a.loss_out[2] = bce;
  }
}

// Per-ray logit gradients; rows n..R-1 get zeros.
__global__ void loss_grad_kernel(LossArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.R) return;
  float gt = 0.f, gx = 0.f;
  if (i < a.n) {
    const float inv_hit = a.scal[0];
    const float y = a.hit[i] ? 1.f : 0.f;
    if (a.hit[i]) {
      const float u = softplusf_(a.zt[i]) - a.tgt[i];
      const float sgn = u > 0.f ? 1.f : (u < 0.f ? -1.f : 0.f);
      if (u != u) gt = u;                                   // NaN: poison the step
      else if (fabsf(u) <= a.clamp) gt = sgn * sigmoidf_(a.zt[i]) * inv_hit;
    }
    gx = a.bce_weight * (sigmoidf_(a.zx[i]) - y) / (float)a.n;
  }
  a.dzt[i] = gt;
  a.dzx[i] = gx;
}

// SDF fitting: per-block compensated sums of |s - s_gt| (slot 0 of the partials).
__global__ void sdf_loss_partial_kernel(LossArgs a) {
  float l1 = 0.f, l1c = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)kLossBlocks * blockDim.x)
    kahan_add(l1, l1c, fabsf(a.zt[i] - a.tgt[i]));
  __shared__ float red[kThreads][2];
  red[threadIdx.x][0] = l1; red[threadIdx.x][1] = l1c;
  tree_sum<2, 1>(red);
  if (threadIdx.x == 0) {
    float* p = a.partial + blockIdx.x * 8;
    p[0] = red[0][0]; p[1] = red[0][1]; p[2] = 0.f; p[3] = 0.f; p[4] = 0.f;
  }
}

// One block of kThreads threads, one per block partial.
__global__ void sdf_loss_final_kernel(LossArgs a) {
  __shared__ float red[kThreads][2];
  red[threadIdx.x][0] = a.partial[threadIdx.x * 8];
  red[threadIdx.x][1] = a.partial[threadIdx.x * 8 + 1];
  tree_sum<2, 1>(red);
  if (threadIdx.x != 0) return;
  const float s0 = red[0][0], c0 = red[0][1];
  const float l = a.n > 0 ? (s0 + c0) / (float)a.n : 0.f;
  a.loss_out[0] = l; a.loss_out[1] = l; a.loss_out[2] = 0.f;
}

// d|s - s_gt| / ds / n (sign of 0 is 0; a NaN error stays NaN); rows n..R-1 get zeros.
__global__ void sdf_loss_grad_kernel(LossArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.R) return;
  float g = 0.f;
  if (i < a.n) {
    const float u = a.zt[i] - a.tgt[i];
    g = u != u ? u : (u > 0.f ? 1.f : (u < 0.f ? -1.f : 0.f)) / (float)a.n;
  }
  a.dzt[i] = g;
  a.dzx[i] = 0.f;
}

__global__ void copy_grads_kernel(const float* gzt, const float* gzx, float* dzt, float* dzx, int64_t n, int64_t R) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R) return;
  dzt[i] = i < n ? gzt[i] : 0.f;
  dzx[i] = (i < n && gzx) ? gzx[i] : 0.f;
}

// ------------------------------------------------------------------ backward chain

struct BwdArgs {
  const uint8_t* packed;
  Layout lay;
  int n_hidden, n_out;
  int64_t R;
  const void* h[kMaxLayers + 1];   // H_l stores (1-based; the masks)
  void* dl[kMaxLayers + 1];        // delta_l stores
  int lo, hi;                      // this launch computes delta_hi .. delta_lo (1-based)
  const float* dzt;
  const float* dzx;
  const uint32_t* mbits;           // the forward's ReLU mask bits (bf16 8-wave chain)
};

// delta_n = (dz_t w_t + dz_xi w_xi) * 1[H_n > 0]; delta_(l) = (delta_(l+1) W_(l+1)) *
// 1[H_l > 0], the product on the matrix cores with the transposed weight blocks, the running
// delta resident in LDS.  One launch covers layers hi down to lo: from the logit gradients
// when hi = n, else from the stored delta_(hi+1).  Every delta it computes is stored.
template <class P, int WIDTH, int WAVES>
__global__ __launch_bounds__(WAVES * 64, 1) void bwd_chain_kernel(BwdArgs a) {
  using C = Chain<P, WIDTH, WAVES>;
  using E = typename P::E;
  constexpr int M = C::M, RT = C::RT, NT = C::NT, LDX = C::LDX;
  __shared__ __attribute__((aligned(16))) E X[C::XSIZE];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ray0 = (int64_t)blockIdx.x * M;
  const float* hw = reinterpret_cast<const float*>(a.packed + a.lay.head_w_off);

  // The first delta in LDS, one [8 rays] block of one neuron per chunk (vector loads and
  // stores of whole blocks of the [R / 8][WIDTH][8] stores): every load of a thread's chunks
  // is issued before the first is used, the logit gradients of the tile go through LDS.
  constexpr int kChunks = (M / 8) * WIDTH / (WAVES * 64);
  static_assert((M / 8) * WIDTH % (WAVES * 64) == 0, "whole chunks per thread");
  __shared__ float dzs[2][M];
  int top;   // the first delta the loop computes
  if (a.hi == a.n_hidden) {
    const E* Hn = reinterpret_cast<const E*>(a.h[a.n_hidden]);
    E* Dn = reinterpret_cast<E*>(a.dl[a.n_hidden]);
    for (int r = threadIdx.x; r < M; r += WAVES * 64) {
      dzs[0][r] = a.dzt[ray0 + r];
      dzs[1][r] = a.n_out > 1 ? a.dzx[ray0 + r] : 0.f;
    }
    V4<E> h[kChunks][2];
    float w0[kChunks], w1[kChunks];
#pragma unroll
    for (int k = 0; k < kChunks; ++k) {
      const int c = threadIdx.x + k * WAVES * 64, rb = c / WIDTH, j = c % WIDTH;
      const int64_t o = (((ray0 >> 3) + rb) * WIDTH + j) * 8;
      h[k][0] = *reinterpret_cast<const V4<E>*>(Hn + o);
      h[k][1] = *reinterpret_cast<const V4<E>*>(Hn + o + 4);
      w0[k] = hw[j];
      w1[k] = a.n_out > 1 ? hw[WIDTH + j] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kChunks; ++k) {
      const int c = threadIdx.x + k * WAVES * 64, rb = c / WIDTH, j = c % WIDTH;
      const int64_t o = (((ray0 >> 3) + rb) * WIDTH + j) * 8;
      V4<E> dv[2];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        float d = dzs[0][rb * 8 + q] * w0[k];
        if (a.n_out > 1) d = fmaf(dzs[1][rb * 8 + q], w1[k], d);
        d = (float)h[k][q >> 2][q & 3] > 0.f ? d : 0.f;
        X[(rb * 8 + q) * LDX + j] = (E)d;
        dv[q >> 2][q & 3] = (E)d;
      }
      *reinterpret_cast<V4<E>*>(Dn + o) = dv[0];
      *reinterpret_cast<V4<E>*>(Dn + o + 4) = dv[1];
    }
    top = a.n_hidden - 1;
  } else {
    const E* Du = reinterpret_cast<const E*>(a.dl[a.hi + 1]);
    V4<E> u[kChunks][2];
#pragma unroll
    for (int k = 0; k < kChunks; ++k) {
      const int c = threadIdx.x + k * WAVES * 64, rb = c / WIDTH, j = c % WIDTH;
      const int64_t o = (((ray0 >> 3) + rb) * WIDTH + j) * 8;
      u[k][0] = *reinterpret_cast<const V4<E>*>(Du + o);
      u[k][1] = *reinterpret_cast<const V4<E>*>(Du + o + 4);
    }
#pragma unroll
    for (int k = 0; k < kChunks; ++k) {
      const int c = threadIdx.x + k * WAVES * 64, rb = c / WIDTH, j = c % WIDTH;
#pragma unroll
      for (int q = 0; q < 8; ++q) X[(rb * 8 + q) * LDX + j] = u[k][q >> 2][q & 3];
    }
    top = a.hi;
  }
  const int nt0 = wave * NT;
  typename C::Ring ring;
  if (top >= a.lo) C::preload(ring, a.packed + a.lay.wt_off[top], WIDTH / P::KBLK, nt0, lane);
  __syncthreads();
  constexpr int kMD = (RT * NT * 16 + 31) / 32;   // mask-bit dwords per lane
  for (int l = top; l >= a.lo; --l) {
    f32x16 acc[RT][NT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[rt][t] = f32x16{};
    C::template gemm<WIDTH / P::KBLK>(acc, X, a.packed + a.lay.wt_off[l], WIDTH / P::KBLK, nt0, lane, ring);
    // the masks of delta_l as the forward's bits, issued before the barrier
    uint32_t mb[kMD];
    if constexpr (kSpreadStores<P, WAVES>) {
      const uint32_t* mw = a.mbits + ((((int64_t)l * gridDim.x + blockIdx.x) * WAVES + wave) * kMD) * 64 + lane;
#pragma unroll
      for (int j = 0; j < kMD; ++j) mb[j] = mw[j * 64];
    }
    __builtin_amdgcn_sched_barrier(0);
    // the next layer's first weight blocks; the last layer loads its own blocks again, so that
    // the preload is unconditional and the wait for the mask bits above leaves it in flight
    // (behind a branch the wait would also cover the preload)
    C::preload(ring, a.packed + a.lay.wt_off[l > a.lo ? l - 1 : l], WIDTH / P::KBLK, nt0, lane);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    const E* Hm = reinterpret_cast<const E*>(a.h[l]);   // H_l: the mask of delta_l
    E* Dm = reinterpret_cast<E*>(a.dl[l]);
    // this workgroup's 8-ray blocks of the store (uniform) and the lane's place in a block pair
    E* const Dw = Dm + (ray0 >> 3) * WIDTH * 8;
    const uint32_t lane_off = ((uint32_t)(lane >> 5) * WIDTH + nt0 * 32 + (lane & 31)) * 8;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int n = (nt0 + t) * 32 + (lane & 31);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        if constexpr (kSpreadStores<P, WAVES>) {
          const int p = (rt * NT + t) * 16;
          const uint32_t bits = mb[p >> 5] >> (p & 31);
          bf16x4 d[4];
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            d[v >> 2][v & 3] = (__bf16)(((bits >> v) & 1u) ? acc[rt][t][v] : 0.f);
            X[(rt * 32 + acc_row(v, lane)) * LDX + n] = d[v >> 2][v & 3];
          }
          {
#pragma unroll
            for (int q = 0; q < 4; q += 2) {
              // block rt 4 + q (lanes below 32) or rt 4 + q + 1, neuron n: a uniform base plus
              // the lane's offset
              const i32x4 w = pair_blocks(d[q], d[q + 1]);
              E* const blk = Dw + ((rt * 4 + q) * WIDTH + t * 32) * 8;
              __builtin_nontemporal_store(w, reinterpret_cast<i32x4*>(blk + lane_off));
            }
          }
        } else if constexpr (sizeof(E) == 2) {
          // whole 8-ray blocks of the stores, paired across the lane halves: a lane below 32
          // loads / stores block q, the others block q + 1 (16 bytes each)
          i32x4 hc[2];
#pragma unroll
          for (int qq = 0; qq < 2; ++qq) {
            const int64_t g0 = ray0 + rt * 32 + 8 * (2 * qq + (lane >> 5));
            hc[qq] = *reinterpret_cast<const i32x4*>(Hm + ((g0 >> 3) * WIDTH + n) * 8);
          }
#pragma unroll
          for (int qq = 0; qq < 2; ++qq) {
            bf16x4 hm0, hm1, d0, d1;
            unpair_blocks(hc[qq], hm0, hm1);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int v0 = 8 * qq + i, v1 = 8 * qq + 4 + i;
              d0[i] = (__bf16)((float)hm0[i] > 0.f ? acc[rt][t][v0] : 0.f);
              d1[i] = (__bf16)((float)hm1[i] > 0.f ? acc[rt][t][v1] : 0.f);
              X[(rt * 32 + acc_row(v0, lane)) * LDX + n] = d0[i];
              X[(rt * 32 + acc_row(v1, lane)) * LDX + n] = d1[i];
            }
            const i32x4 w = pair_blocks(d0, d1);
            const int64_t g0 = ray0 + rt * 32 + 8 * (2 * qq + (lane >> 5));
            __builtin_nontemporal_store(w, reinterpret_cast<i32x4*>(Dm + ((g0 >> 3) * WIDTH + n) * 8));
          }
        } else {
          // 4 consecutive rays per register group are contiguous in the store: one vector each
          V4<E> hm[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int64_t g0 = ray0 + rt * 32 + 8 * q;
            hm[q] = *reinterpret_cast<const V4<E>*>(Hm + ((g0 >> 3) * WIDTH + n) * 8 + 4 * (lane >> 5));
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int64_t g0 = ray0 + rt * 32 + 8 * q;
            V4<E> dv;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int v = 4 * q + i;
              const float d = (float)hm[q][i] > 0.f ? acc[rt][t][v] : 0.f;
              dv[i] = (E)d;
              X[(rt * 32 + acc_row(v, lane)) * LDX + n] = dv[i];
            }
            *reinterpret_cast<V4<E>*>(Dm + ((g0 >> 3) * WIDTH + n) * 8 + 4 * (lane >> 5)) = dv;
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ weight gradients

struct DwArgs {
  const uint8_t* h[kMaxLayers + 1];    // layer inputs: h[0] the features, h[l] H_l
  const uint8_t* dl[kMaxLayers + 1];   // delta_l stores (1-based)
  float* grad;            // final gradient (one split) or the partials [splits][P]
  MasterOffsets mo;
  int64_t R;              // padded rows
  int64_t P;              // parameters (stride of the partials)
  int first_sq;           // 0-based index of the first square layer of this launch
  int width, k1_half, n_feat;
  int tiles_l0, tiles_l;  // workgroups for layer 1 (0 when it is not in this launch) and
                          // for every other hidden layer
  int tn_l0, tn_l;        // column tiles of layer 1 / of the other layers
  int splits;             // ray ranges, each summed separately
  int items;              // tiles x splits
};

// dW_l = sum_rays delta_l^T H_(l-1) (H_0 = the encoded features) and db_l = sum_rays delta_l,
// for a run of consecutive hidden layers in one launch (all of them without recomputation).  A workgroup owns a TM x TN tile of one layer's
// gradient over one of `splits` equal ray ranges: 4 waves in 2 x 2, each (TM/2) x (TN/2),
// operands read in matrix-core order straight from the [R / 8][cols][8] stores through
// buffer resources, three steps ahead in a ring of four.  Each (tile, range) sum has one
// fixed order; with several ranges the partial sums are added in range order afterwards.
// Work items (range, tile) go out in groups of four that share operand strips (a 2 x 2
// block of tiles of one layer: two row strips of the deltas, two column strips of the
// inputs), and a group's four workgroups get indices equal mod 8, so the dispatcher puts
// them on one XCD, at the same time: the strips come from HBM once per group and the other
// three reads hit that XCD's L2.
template <class P, int TM, int TN>
__global__ __launch_bounds__(kThreads, 1) void dw_kernel(DwArgs a) {
  using Frag = typename P::AFrag;
  constexpr int RTW = TM / 64;   // 32-row tiles per wave
  constexpr int CTW = TN / 64;   // 32-column tiles per wave
  constexpr int KB = P::KBLK;    // rays per step
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // block -> (group, member) -> work item (range, tile)
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int item = 4 * (8 * (slot >> 2) + xcd) + (slot & 3);
  if (item >= a.items) return;   // whole workgroup, before any memory access
  const int tiles = a.items / a.splits;
  const int split = item / tiles;
  int blk = item % tiles;
  int layer, tm, tn, cols;
  if (blk < a.tiles_l0) {
    layer = 0; cols = a.k1_half;
    tm = blk / a.tn_l0; tn = blk % a.tn_l0;
  } else {
    blk -= a.tiles_l0;
    layer = a.first_sq + blk / a.tiles_l; blk %= a.tiles_l;
    cols = a.width;
    if ((a.tn_l & 1) == 0 && ((a.tiles_l / a.tn_l) & 1) == 0) {
      // 2 x 2 blocks of tiles, four consecutive tiles per block
      const int q = blk >> 2, j = blk & 3, half_tn = a.tn_l >> 1;
      tm = 2 * (q / half_tn) + (j >> 1);
      tn = 2 * (q % half_tn) + (j & 1);
    } else {
      tm = blk / a.tn_l; tn = blk % a.tn_l;
    }
  }
  const int W = a.width;
  const int row0 = tm * TM + (wave >> 1) * (TM / 2);
  const int col0 = tn * TN + (wave & 1) * (TN / 2);
  constexpr int es = sizeof(typename P::E);
  const uint8_t* D = a.dl[layer + 1];   // 0-based layer `layer` is hidden layer layer + 1
  const uint8_t* Hb = a.h[layer];
  const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(D), (short)0,
                                                                      (int)(W * a.R * es), 0x00020000);
  const __amdgpu_buffer_rsrc_t rh = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(Hb), (short)0,
                                                                      (int)(cols * a.R * es), 0x00020000);
  // lane's byte offset inside a step: bf16 steps cover 16 rays (two 8-ray blocks, one per
  // lane half), fp32 steps 8 rays (one block, 4 rays per lane half)
  const int half = lane >> 5;
  const int a_step = W * 8 * es * (KB / 8);      // bytes per step in the delta store
  const int b_step = cols * 8 * es * (KB / 8);
  int ao[RTW], bo[CTW];
#pragma unroll
  for (int r = 0; r < RTW; ++r) {
    const int row = row0 + r * 32 + (lane & 31);
    ao[r] = es == 2 ? (half * W + row) * 16 : row * 32 + half * 16;
  }
#pragma unroll
  for (int c = 0; c < CTW; ++c) {
    const int col = col0 + c * 32 + (lane & 31);
    bo[c] = es == 2 ? (half * cols + col) * 16 : col * 32 + half * 16;
  }

  f32x16 acc[RTW][CTW];
#pragma unroll
  for (int r = 0; r < RTW; ++r)
#pragma unroll
    for (int c = 0; c < CTW; ++c) acc[r][c] = f32x16{};
  float rsum[RTW];
#pragma unroll
  for (int r = 0; r < RTW; ++r) rsum[r] = 0.f;
  const bool do_bias = (tn == 0) && ((wave & 1) == 0);

  const int steps = (int)(a.R / KB) / a.splits;   // a multiple of 4
  const int s0 = split * steps;
  Frag A[4][RTW], B[4][CTW];
  auto load = [&](int slot, int s) {
    const int sa = (s0 + s) * a_step, sb = (s0 + s) * b_step;
#pragma unroll
    for (int r = 0; r < RTW; ++r)
      A[slot][r] = __builtin_bit_cast(Frag, __builtin_amdgcn_raw_buffer_load_b128(rd, ao[r], sa, 0));
#pragma unroll
    for (int c = 0; c < CTW; ++c)
      B[slot][c] = __builtin_bit_cast(Frag, __builtin_amdgcn_raw_buffer_load_b128(rh, bo[c], sb, 0));
  };
  auto compute = [&](int slot) {
#pragma unroll
    for (int r = 0; r < RTW; ++r) {
#pragma unroll
      for (int c = 0; c < CTW; ++c) P::mma(acc[r][c], A[slot][r], B[slot][c]);
      if (do_bias)
#pragma unroll
        for (int j = 0; j < KB / 2; ++j) rsum[r] += (float)A[slot][r][j];
    }
  };
  load(0, 0);
  load(1, 1);
  load(2, 2);
  for (int s = 0; s < steps; s += 4) {
    load(3, s + 3);
    __builtin_amdgcn_sched_barrier(0);
    compute(0);
    __builtin_amdgcn_sched_barrier(0);
    load(0, s + 4);
    __builtin_amdgcn_sched_barrier(0);
    compute(1);
    __builtin_amdgcn_sched_barrier(0);
    load(1, s + 5);
    __builtin_amdgcn_sched_barrier(0);
    compute(2);
    __builtin_amdgcn_sched_barrier(0);
    load(2, s + 6);
    __builtin_amdgcn_sched_barrier(0);
    compute(3);
    __builtin_amdgcn_sched_barrier(0);
  }

  const int fan_in = layer == 0 ? a.n_feat : W;
  float* out = a.grad + (a.splits > 1 ? (int64_t)split * a.P : 0);
  float* gw = out + a.mo.w[layer];
#pragma unroll
  for (int r = 0; r < RTW; ++r)
#pragma unroll
    for (int c = 0; c < CTW; ++c) {
      const int col = col0 + c * 32 + (lane & 31);
      if (col < fan_in) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = row0 + r * 32 + acc_row(v, lane);
          gw[(int64_t)row * fan_in + col] = acc[r][c][v];
        }
      }
    }
  if (do_bias) {
    float* gb = out + a.mo.b[layer];
#pragma unroll
    for (int r = 0; r < RTW; ++r) {
      const float tot = rsum[r] + __shfl_xor(rsum[r], 32);   // the two lane halves hold disjoint rays
      if (lane < 32) gb[row0 + r * 32 + lane] = tot;
    }
  }
}

// grad[i] = sum over ray ranges s (in order) of partial[s][i], for the hidden layers' slice
// [0, n) of the parameter vector (the head gradients are written directly); compensated
// (Neumaier), so the ranges' partial sums are added with one rounding at the end.
__global__ void sum_splits_kernel(const float* part, int splits, int64_t P, int64_t n, float* grad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f, c = 0.f;
    for (int k = 0; k < splits; ++k) kahan_add(s, c, part[(int64_t)k * P + i]);
    grad[i] = s + c;
  }
}

// Head gradients: dW_head[o][j] = sum_r dz_o[r] H_n[r][j], db_head[o] = sum_r dz_o[r].
// Phase 1: block (j-block of 32 neurons, ray chunk c) sums its chunk (8 ray groups per
// block, compensated); phase 2 adds the chunks in order.  kHeadChunks chunks of R / 8
// ray blocks each; the last phase-1 column of blocks (j-block == W / 32) does the biases.

template <class E>
__global__ void head_grad_partial_kernel(const E* Hn, const float* dzt, const float* dzx, int64_t R, int W,
                                         float* part /*[kHeadChunks][2][W + 2]*/) {
  __shared__ float red[8][32][2];
  const int jb = blockIdx.x, c = blockIdx.y;
  const int grp = threadIdx.x >> 5, jl = threadIdx.x & 31;
  const int64_t nblk = R / 8;
  const int64_t per = (nblk + kHeadChunks - 1) / kHeadChunks;
  const int64_t b0 = c * per, b1 = min(nblk, b0 + per);
  float s0 = 0.f, c0 = 0.f, s1 = 0.f, c1 = 0.f;
  if (jb * 32 < W) {
    const int j = jb * 32 + jl;
    for (int64_t rb = b0 + grp; rb < b1; rb += 8) {
      const V4<E> h0 = *reinterpret_cast<const V4<E>*>(Hn + (rb * W + j) * 8);
      const V4<E> h1 = *reinterpret_cast<const V4<E>*>(Hn + (rb * W + j) * 8 + 4);
      // the block's 8 logit gradients of each head as two 16-byte loads (the same for every
      // lane: R is a multiple of 64, so rows rb 8 .. rb 8 + 7 exist and are 32-byte aligned)
      const f32x4 t0 = *reinterpret_cast<const f32x4*>(dzt + rb * 8);
      const f32x4 t1 = *reinterpret_cast<const f32x4*>(dzt + rb * 8 + 4);
      const f32x4 x0 = *reinterpret_cast<const f32x4*>(dzx + rb * 8);
      const f32x4 x1 = *reinterpret_cast<const f32x4*>(dzx + rb * 8 + 4);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float hv = (float)(q < 4 ? h0[q] : h1[q - 4]);
        kahan_add(s0, c0, (q < 4 ? t0[q] : t1[q - 4]) * hv);
        kahan_add(s1, c1, (q < 4 ? x0[q] : x1[q - 4]) * hv);
      }
    }
  } else {
    for (int64_t r = b0 * 8 + threadIdx.x; r < b1 * 8; r += kThreads) {
      kahan_add(s0, c0, dzt[r]);
      kahan_add(s1, c1, dzx[r]);
    }
  }
  if (jb * 32 < W) {
    red[grp][jl][0] = s0 + c0;
    red[grp][jl][1] = s1 + c1;
    __syncthreads();
    if (grp == 0) {
      float t0 = 0.f, t1 = 0.f;
      for (int g = 0; g < 8; ++g) { t0 += red[g][jl][0]; t1 += red[g][jl][1]; }
      part[((int64_t)c * 2 + 0) * (W + 2) + jb * 32 + jl] = t0;
      part[((int64_t)c * 2 + 1) * (W + 2) + jb * 32 + jl] = t1;
    }
  } else {
    __shared__ float rb2[kThreads][2];
    rb2[threadIdx.x][0] = s0 + c0;
    rb2[threadIdx.x][1] = s1 + c1;
    __syncthreads();
    if (threadIdx.x == 0) {
      float t0 = 0.f, t1 = 0.f;
      for (int t = 0; t < kThreads; ++t) { t0 += rb2[t][0]; t1 += rb2[t][1]; }
      part[((int64_t)c * 2 + 0) * (W + 2) + W] = t0;
      part[((int64_t)c * 2 + 1) * (W + 2) + W] = t1;
    }
  }
}

__global__ void head_grad_final_kernel(const float* part, int W, int n_out, float* gW, float* gb) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > W) return;
  float t0 = 0.f, c0 = 0.f, t1 = 0.f, c1 = 0.f;
  for (int c = 0; c < kHeadChunks; ++c) {
    kahan_add(t0, c0, part[((int64_t)c * 2 + 0) * (W + 2) + j]);
    kahan_add(t1, c1, part[((int64_t)c * 2 + 1) * (W + 2) + j]);
  }
  if (j < W) {
    gW[j] = t0 + c0;
    if (n_out > 1) gW[W + j] = t1 + c1;
  } else {
    gb[0] = t0 + c0;
    if (n_out > 1) gb[1] = t1 + c1;
  }
}

// ------------------------------------------------------------------ Adam

__global__ void zero_flag_kernel(int32_t* flag) { if (threadIdx.x == 0 && blockIdx.x == 0) *flag = 0; }

// flag |= 1 if any g[i], i < n, is not finite.  16-byte loads over the aligned body (an
// unaligned g takes the 4-byte loop throughout), 4-byte loads over the tail.
__global__ void finite_check_kernel(const float* g, int64_t n, int32_t* flag) {
  bool bad = false;
  const int64_t n4 = (reinterpret_cast<uintptr_t>(g) & 15) ? 0 : n / 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const f32x4* g4 = reinterpret_cast<const f32x4*>(g);
#pragma unroll 4
  for (int64_t i = t; i < n4; i += stride) {
    const f32x4 v = g4[i];
    bad |= !(isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]) && isfinite(v[3]));
  }
  for (int64_t i = 4 * n4 + t; i < n; i += stride) bad |= !isfinite(g[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

__global__ void adam_kernel(float* p, float* m, float* v, const float* g, int64_t n, const int32_t* flag,
                            float lr, float b1, float b2, float eps, float bc1, float bc2) {
  if (*flag) return;                     // a non-finite gradient: the whole update is skipped
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / bc1;
    const float vh = vi / bc2;
    p[i] -= lr * mh / (sqrtf(vh) + eps);
  }
}

// ------------------------------------------------------------------ host side

static int check_train_desc(const ddf_net_desc* d) {
  int rc;
  if ((rc = check_desc(d))) return rc;
  if (d->precision == DDF_FP8_E4M3) return fail(DDF_ERR_UNSUPPORTED, "training runs in fp32 or bf16");
  return DDF_OK;
}

// One activation slab is addressed with 32-bit buffer offsets.
static int check_rows(const ddf_net_desc& d, const TrainWs& w) {
  if ((int64_t)d.width * w.R * w.esize >= (1ll << 31))
    return fail(DDF_ERR_UNSUPPORTED, "batch too large: one activation slab must stay below 2 GiB");
  return DDF_OK;
}

static int check_hp(const ddf_train_hparams* hp) {
  if (!hp) return fail(DDF_ERR_INVALID_ARG, "hp is NULL");
  if (hp->step < 1) return fail(DDF_ERR_INVALID_ARG, "step must be >= 1");
  if (!(hp->lr >= 0.f) || !(hp->beta1 >= 0.f && hp->beta1 < 1.f) || !(hp->beta2 >= 0.f && hp->beta2 < 1.f) ||
      !(hp->eps > 0.f))
    return fail(DDF_ERR_INVALID_ARG, "hyper-parameters out of range");
  return DDF_OK;
}

int check_hp_public(const ddf_train_hparams* hp) { return check_hp(hp); }

// Adam on the fp32 master (skipped as a whole when any gradient is not finite), then the
// repack of the working copy.
static int run_adam(const ddf_net_desc& d, float* master, float* adam_m, float* adam_v, void* packed,
                    const float* grad, size_t P, const ddf_train_hparams* hp, int32_t* flag, hipStream_t st) {
  int rc;
  zero_flag_kernel<<<1, 64, 0, st>>>(flag);
  finite_check_kernel<<<1024, 256, 0, st>>>(grad, (int64_t)P, flag);
  const double bc1 = 1.0 - pow((double)hp->beta1, (double)hp->step);
  const double bc2 = 1.0 - pow((double)hp->beta2, (double)hp->step);
  adam_kernel<<<2048, 256, 0, st>>>(master, adam_m, adam_v, grad, (int64_t)P, flag, hp->lr, hp->beta1,
                                    hp->beta2, hp->eps, (float)bc1, (float)bc2);
  if ((rc = hip_status(hipGetLastError(), "adam launch"))) return rc;
  return hip_status(launch_pack(d, master, nullptr, packed, st, true), "repack launch");
}

static size_t param_count_of(const ddf_net_desc& d) {
  const size_t nf = (size_t)d.n_in * (1 + 2 * d.n_freq);
  const size_t w = d.width;
  return w * nf + w + (size_t)(d.n_hidden - 1) * (w * w + w) + (size_t)d.n_out * w + d.n_out;
}

template <class P>
static hipError_t launch_bwd(const ddf_net_desc& d, const BwdArgs& b, hipStream_t st) {
  const unsigned blocks = (unsigned)(b.R / P::M);
  switch (d.width) {
    case 128: hipLaunchKernelGGL((bwd_chain_kernel<P, 128, 4>), dim3(blocks), dim3(256), 0, st, b); break;
    case 256: hipLaunchKernelGGL((bwd_chain_kernel<P, 256, 8>), dim3(blocks), dim3(512), 0, st, b); break;
    case 512: hipLaunchKernelGGL((bwd_chain_kernel<P, 512, 8>), dim3(blocks), dim3(512), 0, st, b); break;
    default: hipLaunchKernelGGL((bwd_chain_kernel<P, 1024, 8>), dim3(blocks), dim3(512), 0, st, b); break;
  }
  return hipGetLastError();
}

// Ray ranges of the weight-gradient launch: enough workgroups for two per CU, and a step
// count per range that stays a multiple of 4.
static int dw_splits(int tiles, int64_t steps) {
  int s = 1;
  while (s < 8 && tiles * s < 512 && (steps % (4 * 2 * s)) == 0) s *= 2;
  return s;
}

// Weight gradients of the 0-based hidden layers lo0 .. hi0 in one launch.
template <class P>
static hipError_t launch_dw(const ddf_net_desc& d, DwArgs& a, int lo0, int hi0, hipStream_t st) {
  const int T = d.width >= 512 ? 256 : 128;   // square tiles
  a.tn_l0 = (a.k1_half + T - 1) / T;
  a.tn_l = d.width / T;
  a.tiles_l0 = lo0 == 0 ? (d.width / T) * a.tn_l0 : 0;
  a.tiles_l = (d.width / T) * a.tn_l;
  a.first_sq = lo0 == 0 ? 1 : lo0;
  const int tiles = a.tiles_l0 + (hi0 - a.first_sq + 1) * a.tiles_l;
  if (tiles <= 0) return hipSuccess;
  a.items = tiles * a.splits;
  const int groups = (a.items + 3) / 4;
  const dim3 grid((unsigned)(32 * ((groups + 7) / 8)));
  if (T == 256)
    hipLaunchKernelGGL((dw_kernel<P, 256, 256>), grid, dim3(kThreads), 0, st, a);
  else
    hipLaunchKernelGGL((dw_kernel<P, 128, 128>), grid, dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

static int dw_tiles(const ddf_net_desc& d, int k1_half, int lo0, int hi0) {
  const int T = d.width >= 512 ? 256 : 128;
  const int first_sq = lo0 == 0 ? 1 : lo0;
  return (lo0 == 0 ? (d.width / T) * ((k1_half + T - 1) / T) : 0) + (hi0 - first_sq + 1) * (d.width / T) * (d.width / T);
}

// The training forward over all R rows (rows >= n from zero inputs).  Layers [0, n_hidden):
// the logits and the kept activations (features, every H_l or the checkpoints).  A shorter
// range [l_begin, l_end) is the recomputation of one segment's activations: from the inputs
// when l_begin = 0, else from the kept H_(l_begin); no logits.
static int run_forward_rows(const ddf_net_desc& d, const void* packed, const float* in, int64_t n, float* zt,
                            float* zx, const TrainWs& w, const TrainPtrs& p, int l_begin, int l_end,
                            hipStream_t st) {
  FwdArgs a{};
  a.packed = static_cast<const uint8_t*>(packed);
  a.lay = make_layout(d);
  a.n_in = d.n_in; a.n_freq = d.n_freq; a.n_hidden = d.n_hidden; a.n_out = d.n_out;
  a.in = in; a.n = n; a.stride = n;
  a.mode = l_begin == 0 ? kModeTrain : kModeRecompute;
  a.out0 = zt; a.out1 = zx;
  a.l_begin = l_begin; a.l_end = l_end;
  a.act_rows = w.R;
  const bool full = l_begin == 0 && l_end == d.n_hidden;
  a.hst[0] = full ? p.h[0] : nullptr;
  for (int l = 1; l <= d.n_hidden; ++l)
    a.hst[l] = full ? (p.kept[l] ? p.h[l] : nullptr) : (l > l_begin && l <= l_end ? p.h[l] : nullptr);
  if (l_begin > 0) a.hst[l_begin] = p.h[l_begin];   // the recomputation's input
  a.mbits = p.mbits;
  return hip_status(launch_forward(d, a, w.R, st), "training forward launch");
}

// Backward from the logit gradients already in ws (dz_t, dz_xi) into grad: segment by
// segment from the top (one segment of all layers without recomputation), each one
// recomputing its activations from the checkpoint below it, then its delta chain, then its
// weight gradients.
static int run_backward(const ddf_net_desc& d, const void* packed, const float* in, int64_t n, const TrainWs& w,
                        uint8_t* ws, float* grad, hipStream_t st) {
  const Layout L = make_layout(d);
  const TrainPtrs p = train_ptrs(d, w, ws);
  const MasterOffsets mo = master_offsets(d);
  const int nh = d.n_hidden;
  const float* dzt = reinterpret_cast<const float*>(ws + w.dzt);
  const float* dzx = reinterpret_cast<const float*>(ws + w.dzx);
  hipError_t e;
  int rc;
  for (int hi = nh; hi >= 1;) {
    const int lo = w.rc ? (hi - 1) / w.rc * w.rc + 1 : 1;
    if (w.rc && hi - 1 >= lo && (rc = run_forward_rows(d, packed, in, n, nullptr, nullptr, w, p, lo - 1, hi - 1, st)))
      return rc;
    BwdArgs b{};
    b.packed = static_cast<const uint8_t*>(packed);
    b.lay = L;
    b.n_hidden = nh; b.n_out = d.n_out; b.R = w.R;
    for (int l = 0; l <= nh; ++l) { b.h[l] = p.h[l]; b.dl[l] = p.dl[l]; }
    b.lo = lo; b.hi = hi;
    b.dzt = dzt; b.dzx = dzx;
    b.mbits = p.mbits;
    e = d.precision == DDF_FP32 ? launch_bwd<PF32>(d, b, st) : launch_bwd<PBF16>(d, b, st);
    if (e != hipSuccess) return hip_status(e, "backward chain launch");
    DwArgs a{};
    for (int l = 0; l <= nh; ++l) { a.h[l] = p.h[l]; a.dl[l] = p.dl[l]; }
    a.mo = mo;
    a.R = w.R; a.P = (int64_t)param_count_of(d);
    a.width = d.width; a.k1_half = L.k1_half; a.n_feat = L.n_feat;
    // the ray ranges follow from the whole network, so that every tile's sum has the same
    // order with and without recomputation (bit-identical gradients)
    a.splits = dw_splits(dw_tiles(d, L.k1_half, 0, nh - 1), w.R / (d.precision == DDF_FP32 ? 8 : 16));
    a.grad = a.splits > 1 ? reinterpret_cast<float*>(ws + w.dwpart) : grad;
    e = d.precision == DDF_FP32 ? launch_dw<PF32>(d, a, lo - 1, hi - 1, st) : launch_dw<PBF16>(d, a, lo - 1, hi - 1, st);
    if (e != hipSuccess) return hip_status(e, "weight-gradient launch");
    if (a.splits > 1) {
      const int64_t o0 = mo.w[lo - 1], o1 = mo.w[hi];   // this segment's slice of the parameters
      sum_splits_kernel<<<2048, 256, 0, st>>>(a.grad + o0, a.splits, a.P, o1 - o0, grad + o0);
      if ((e = hipGetLastError()) != hipSuccess) return hip_status(e, "weight-gradient sum launch");
    }
    hi = lo - 1;
  }
  const dim3 hb((unsigned)(d.width / 32 + 1), kHeadChunks);
  float* part = reinterpret_cast<float*>(ws + w.headp);
  if (d.precision == DDF_FP32)
    head_grad_partial_kernel<float><<<hb, kThreads, 0, st>>>(reinterpret_cast<const float*>(p.h[nh]), dzt, dzx, w.R,
                                                             d.width, part);
  else
    head_grad_partial_kernel<__bf16><<<hb, kThreads, 0, st>>>(reinterpret_cast<const __bf16*>(p.h[nh]), dzt, dzx,
                                                              w.R, d.width, part);
  head_grad_final_kernel<<<(unsigned)(d.width / 256 + 1), 256, 0, st>>>(part, d.width, d.n_out, grad + mo.w[nh],
                                                                       grad + mo.b[nh]);
  return hip_status(hipGetLastError(), "head-gradient launch");
}

static int run_forward_train(const ddf_net_desc& d, const void* packed, const float* rays, int64_t n, float* zt,
                             float* zx, const TrainWs& w, uint8_t* ws, hipStream_t st) {
  const TrainPtrs p = train_ptrs(d, w, ws);
  return run_forward_rows(d, packed, rays, n, zt, zx, w, p, 0, d.n_hidden, st);
}

// The distillation loss over logits already in device memory: the three terms into loss_out
// and the per-ray logit gradients into dzt / dzx (rows n .. R - 1 zero).  Scratch: partial
// (kLossBlocks x 8 floats) and scal (64 bytes).  Used by the hash-grid field as well.
int launch_ddf_loss(const float* zt, const float* zx, const float* t_gt, const uint8_t* hit, int64_t n, int64_t R,
                    float* partial, float* scal, float* loss_out, float* dzt, float* dzx, float bce_weight,
                    float clamp, hipStream_t st) {
  LossArgs la{};
  la.zt = zt; la.zx = zx; la.tgt = t_gt; la.hit = hit; la.n = n; la.R = R;
  la.partial = partial; la.scal = scal; la.loss_out = loss_out; la.dzt = dzt; la.dzx = dzx;
  la.bce_weight = bce_weight; la.clamp = clamp;
  loss_partial_kernel<<<kLossBlocks, kThreads, 0, st>>>(la);
  loss_final_kernel<<<1, kThreads, 0, st>>>(la);
  loss_grad_kernel<<<(unsigned)((R + 255) / 256), 256, 0, st>>>(la);
  return hip_status(hipGetLastError(), "loss launch");
}

// Adam over a flat fp32 parameter vector (skipped as a whole on a non-finite gradient).
int launch_adam_flat(float* p, float* m, float* v, const float* g, int64_t P, const ddf_train_hparams* hp,
                     int32_t* flag, hipStream_t st) {
  zero_flag_kernel<<<1, 64, 0, st>>>(flag);
  finite_check_kernel<<<1024, 256, 0, st>>>(g, P, flag);
  const double bc1 = 1.0 - pow((double)hp->beta1, (double)hp->step);
  const double bc2 = 1.0 - pow((double)hp->beta2, (double)hp->step);
  adam_kernel<<<2048, 256, 0, st>>>(p, m, v, g, P, flag, hp->lr, hp->beta1, hp->beta2, hp->eps, (float)bc1, (float)bc2);
  return hip_status(hipGetLastError(), "adam launch");
}

int loss_scratch_floats() { return 8 * kLossBlocks; }

// One kept activation slab ([rows / 8][width][8] in the operand type) as float32 [n][width].
template <class E>
__global__ void unpack_slab_kernel(const E* slab, int width, int64_t n, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * width) return;
  const int64_t r = i / width;
  const int c = (int)(i - r * width);
  out[i] = (float)slab[((r >> 3) * width + c) * 8 + (r & 7)];
}

static int check_recompute(int recompute_every) {
  if (recompute_every < 0) return fail(DDF_ERR_INVALID_ARG, "recompute_every = %d must be >= 0", recompute_every);
  return DDF_OK;
}

}  // namespace ddf

using namespace ddf;

extern "C" {

size_t ddf_train_workspace_bytes(const ddf_net_desc* d, int64_t batch, int32_t recompute_every) {
  if (check_train_desc(d) != DDF_OK || batch < 0 || recompute_every < 0) return 0;
  return (size_t)train_ws(*d, batch, param_count_of(*d), recompute_every).total;
}

int ddf_forward_train(const ddf_net_desc* d, const void* packed, const float* rays, int64_t n, float* z_t,
                      float* z_xi, int32_t recompute_every, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_train_desc(d)) || (rc = check_recompute(recompute_every))) return rc;
  if (n < 0 || n > (int64_t)INT32_MAX / 4) return fail(DDF_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (n == 0) return DDF_OK;
  if ((rc = check_ptr(packed, "packed")) || (rc = check_ptr(rays, "rays")) || (rc = check_ptr(z_t, "z_t")) ||
      (rc = check_ptr(ws, "ws")))
    return rc;
  if (d->n_out > 1 && (rc = check_ptr(z_xi, "z_xi"))) return rc;
  const TrainWs w = train_ws(*d, n, param_count_of(*d), recompute_every);
  if ((rc = check_rows(*d, w))) return rc;
  if ((int64_t)ws_bytes < w.total) return fail(DDF_ERR_WORKSPACE, "workspace %zu < %lld bytes", ws_bytes, (long long)w.total);
  return run_forward_train(*d, packed, rays, n, z_t, d->n_out > 1 ? z_xi : z_t, w, static_cast<uint8_t*>(ws),
                           (hipStream_t)stream);
}

int ddf_train_kept_activation(const ddf_net_desc* d, int64_t n, int32_t recompute_every, const void* ws,
                              size_t ws_bytes, int32_t layer, float* h, void* stream) {
  int rc;
  if ((rc = check_train_desc(d)) || (rc = check_recompute(recompute_every))) return rc;
  if (n < 0 || n > (int64_t)INT32_MAX / 4) return fail(DDF_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (layer < 1 || layer > d->n_hidden)
    return fail(DDF_ERR_INVALID_ARG, "layer %d outside 1..%d", layer, d->n_hidden);
  if (n == 0) return DDF_OK;
  if ((rc = check_ptr(ws, "ws")) || (rc = check_ptr(h, "h"))) return rc;
  const TrainWs w = train_ws(*d, n, param_count_of(*d), recompute_every);
  if ((int64_t)ws_bytes < w.total) return fail(DDF_ERR_WORKSPACE, "workspace %zu < %lld bytes", ws_bytes, (long long)w.total);
  const TrainPtrs p = train_ptrs(*d, w, static_cast<uint8_t*>(const_cast<void*>(ws)));
  if (!p.kept[layer])
    return fail(DDF_ERR_INVALID_ARG, "H_%d is not kept with recompute_every = %d", layer, recompute_every);
  hipStream_t st = (hipStream_t)stream;
  const unsigned blocks = (unsigned)((n * d->width + 255) / 256);
  if (d->precision == DDF_FP32)
    unpack_slab_kernel<float><<<blocks, 256, 0, st>>>(reinterpret_cast<const float*>(p.h[layer]), d->width, n, h);
  else
    unpack_slab_kernel<__bf16><<<blocks, 256, 0, st>>>(reinterpret_cast<const __bf16*>(p.h[layer]), d->width, n, h);
  g_err_clear();
  return hip_status(hipGetLastError(), "kept activation unpack");
}

int ddf_backward(const ddf_net_desc* d, const void* packed, const float* rays, int64_t n, const float* grad_z_t,
                 const float* grad_z_xi, float* grad_params, int32_t recompute_every, void* ws, size_t ws_bytes,
                 void* stream) {
  int rc;
  if ((rc = check_train_desc(d)) || (rc = check_recompute(recompute_every))) return rc;
  if (n < 0 || n > (int64_t)INT32_MAX / 4) return fail(DDF_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (n == 0) return DDF_OK;
  if ((rc = check_ptr(packed, "packed")) || (rc = check_ptr(rays, "rays")) || (rc = check_ptr(grad_z_t, "grad_z_t")) ||
      (rc = check_ptr(grad_params, "grad_params")) || (rc = check_ptr(ws, "ws")))
    return rc;
  if (d->n_out > 1 && (rc = check_ptr(grad_z_xi, "grad_z_xi"))) return rc;
  const TrainWs w = train_ws(*d, n, param_count_of(*d), recompute_every);
  if ((rc = check_rows(*d, w))) return rc;
  if ((int64_t)ws_bytes < w.total) return fail(DDF_ERR_WORKSPACE, "workspace %zu < %lld bytes", ws_bytes, (long long)w.total);
  hipStream_t st = (hipStream_t)stream;
  uint8_t* wb = static_cast<uint8_t*>(ws);
  copy_grads_kernel<<<(unsigned)((w.R + 255) / 256), 256, 0, st>>>(grad_z_t, d->n_out > 1 ? grad_z_xi : nullptr,
                                                                  reinterpret_cast<float*>(wb + w.dzt),
                                                                  reinterpret_cast<float*>(wb + w.dzx), n, w.R);
  if ((rc = hip_status(hipGetLastError(), "gradient copy"))) return rc;
  g_err_clear();
  return run_backward(*d, packed, rays, n, w, wb, grad_params, st);
}

int ddf_train_step(const ddf_net_desc* d, float* master, float* adam_m, float* adam_v, void* packed,
                   const float* rays, const float* t_gt, const uint8_t* hit_gt, int64_t batch,
                   const ddf_train_hparams* hp, float* loss_out, int32_t* nonfinite_flag, float* grad_out, void* ws,
                   size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_train_desc(d))) return rc;
  if (d->n_in != 6 || d->n_out != 2) return fail(DDF_ERR_INVALID_ARG, "ddf_train_step needs a DDF net (n_in 6, n_out 2)");
  if ((rc = check_hp(hp)) || (rc = check_recompute(hp->recompute_every))) return rc;
  if (!(hp->l1_clamp > 0.f) || !(hp->bce_weight >= 0.f))
    return fail(DDF_ERR_INVALID_ARG, "loss hyper-parameters out of range");
  if (batch < 1 || batch > (int64_t)INT32_MAX / 4) return fail(DDF_ERR_INVALID_ARG, "batch = %lld out of range", (long long)batch);
  if ((rc = check_ptr(master, "master")) || (rc = check_ptr(adam_m, "adam_m")) || (rc = check_ptr(adam_v, "adam_v")) ||
      (rc = check_ptr(packed, "packed")) || (rc = check_ptr(rays, "rays")) || (rc = check_ptr(t_gt, "t_gt")) ||
      (rc = check_ptr(hit_gt, "hit_gt")) || (rc = check_ptr(loss_out, "loss_out")) ||
      (rc = check_ptr(nonfinite_flag, "nonfinite_flag")) || (rc = check_ptr(ws, "ws")))
    return rc;
  if (grad_out && (rc = check_ptr(grad_out, "grad_out"))) return rc;
  const size_t P = param_count_of(*d);
  const TrainWs w = train_ws(*d, batch, P, hp->recompute_every);
  if ((rc = check_rows(*d, w))) return rc;
  if ((int64_t)ws_bytes < w.total) return fail(DDF_ERR_WORKSPACE, "workspace %zu < %lld bytes", ws_bytes, (long long)w.total);
  hipStream_t st = (hipStream_t)stream;
  uint8_t* wb = static_cast<uint8_t*>(ws);
  float* zt = reinterpret_cast<float*>(wb + w.zt);
  float* zx = reinterpret_cast<float*>(wb + w.zx);
  g_err_clear();
  if ((rc = run_forward_train(*d, packed, rays, batch, zt, zx, w, wb, st))) return rc;
  LossArgs la{};
  la.zt = zt; la.zx = zx; la.tgt = t_gt; la.hit = hit_gt; la.n = batch; la.R = w.R;
  la.partial = reinterpret_cast<float*>(wb + w.lossp);
  la.scal = reinterpret_cast<float*>(wb + w.scal);
  la.loss_out = loss_out;
  la.dzt = reinterpret_cast<float*>(wb + w.dzt);
  la.dzx = reinterpret_cast<float*>(wb + w.dzx);
  la.bce_weight = hp->bce_weight; la.clamp = hp->l1_clamp;
  loss_partial_kernel<<<kLossBlocks, kThreads, 0, st>>>(la);
  loss_final_kernel<<<1, kThreads, 0, st>>>(la);
  loss_grad_kernel<<<(unsigned)((w.R + 255) / 256), 256, 0, st>>>(la);
  if ((rc = hip_status(hipGetLastError(), "loss launch"))) return rc;
  float* grad = grad_out ? grad_out : reinterpret_cast<float*>(wb + w.grad);
  if ((rc = run_backward(*d, packed, rays, batch, w, wb, grad, st))) return rc;
  return run_adam(*d, master, adam_m, adam_v, packed, grad, P, hp, nonfinite_flag, st);
}

int sdf_train_step(const ddf_net_desc* d, float* master, float* adam_m, float* adam_v, void* packed,
                   const float* points, const float* sdf_gt, int64_t n, const ddf_train_hparams* hp,
                   float* loss_out, int32_t* nonfinite_flag, float* grad_out, void* ws, size_t ws_bytes,
                   void* stream) {
  int rc;
  if ((rc = check_train_desc(d))) return rc;
  if (d->n_in != 3 || d->n_out != 1) return fail(DDF_ERR_INVALID_ARG, "sdf_train_step needs an SDF net (n_in 3, n_out 1)");
  if ((rc = check_hp(hp)) || (rc = check_recompute(hp->recompute_every))) return rc;
  if (n < 1 || n > (int64_t)INT32_MAX / 4) return fail(DDF_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if ((rc = check_ptr(master, "master")) || (rc = check_ptr(adam_m, "adam_m")) || (rc = check_ptr(adam_v, "adam_v")) ||
      (rc = check_ptr(packed, "packed")) || (rc = check_ptr(points, "points")) || (rc = check_ptr(sdf_gt, "sdf_gt")) ||
      (rc = check_ptr(loss_out, "loss_out")) || (rc = check_ptr(nonfinite_flag, "nonfinite_flag")) ||
      (rc = check_ptr(ws, "ws")))
    return rc;
  if (grad_out && (rc = check_ptr(grad_out, "grad_out"))) return rc;
  const size_t P = param_count_of(*d);
  const TrainWs w = train_ws(*d, n, P, hp->recompute_every);
  if ((rc = check_rows(*d, w))) return rc;
  if ((int64_t)ws_bytes < w.total) return fail(DDF_ERR_WORKSPACE, "workspace %zu < %lld bytes", ws_bytes, (long long)w.total);
  hipStream_t st = (hipStream_t)stream;
  uint8_t* wb = static_cast<uint8_t*>(ws);
  float* zt = reinterpret_cast<float*>(wb + w.zt);
  g_err_clear();
  if ((rc = run_forward_train(*d, packed, points, n, zt, zt, w, wb, st))) return rc;
  LossArgs la{};
  la.zt = zt; la.tgt = sdf_gt; la.n = n; la.R = w.R;
  la.partial = reinterpret_cast<float*>(wb + w.lossp);
  la.loss_out = loss_out;
  la.dzt = reinterpret_cast<float*>(wb + w.dzt);
  la.dzx = reinterpret_cast<float*>(wb + w.dzx);
  sdf_loss_partial_kernel<<<kLossBlocks, kThreads, 0, st>>>(la);
  sdf_loss_final_kernel<<<1, kThreads, 0, st>>>(la);
  sdf_loss_grad_kernel<<<(unsigned)((w.R + 255) / 256), 256, 0, st>>>(la);
  if ((rc = hip_status(hipGetLastError(), "sdf loss launch"))) return rc;
  float* grad = grad_out ? grad_out : reinterpret_cast<float*>(wb + w.grad);
  if ((rc = run_backward(*d, packed, points, n, w, wb, grad, st))) return rc;
  return run_adam(*d, master, adam_m, adam_v, packed, grad, P, hp, nonfinite_flag, st);
}

}  // extern "C"
