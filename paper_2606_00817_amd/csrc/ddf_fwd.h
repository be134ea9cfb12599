// Arguments of the fused forward kernel and its per-mode hooks.
#pragma once
#include "ddf_chain.h"
#include "ddf_internal.h"

namespace ddf {

// The bf16 chain with 8 waves writes the ReLU masks of its training forward as bits, which the
// backward chain's epilogue reads instead of the kept activations.
template <class P, int WAVES>
constexpr bool kSpreadStores = sizeof(typename P::E) == 2 && WAVES == 8;

// Mask-bit dwords per lane and layer of the bf16 8-wave chain (RT x NT x 16 bits).
inline __host__ __device__ int mask_dwords(int width) { return 2 * (width / 32 / 8) * 16 / 32; }

enum FwdMode {
  kModeQuery = 0,   // t = softplus(z_t), xi = sigmoid(z_xi)
  kModeTrain = 1,   // raw logits + activations kept for the backward pass
  kModeSdf = 2,     // signed distance z_0 at points
  kModeTrace = 3,   // one sphere-tracing step over the active-ray list
  kModeCalib = 4,   // query that records max h_l of hidden layers 1..n-1 (FP8 scales)
  kModeRecompute = 5,  // training: rerun hidden layers from a kept activation, keeping theirs
  kModeHidden = 6,     // the last hidden layer's float32 output h_n per ray, [n][width] in out0
  kModePool = 7        // persistent sphere tracing: a workgroup's ray slots refilled from a pool
};

struct FwdArgs {
  const float* in;        // SoA inputs [n_in][stride]; trace mode: rays [6][stride]
  int64_t n;              // items (trace mode: capacity of the active list)
  int64_t stride;         // row stride of `in`
  const uint8_t* packed;
  Layout lay;
  int n_in, n_freq, n_hidden, n_out;
  int mode;
  float* out0;            // query: t; train: z_t; sdf: s; hidden: h_n [n][width]
  float* out1;            // query: xi; train: z_xi
  // 0-based hidden layers this launch runs: [l_begin, l_end) (queries: all of them)
  int l_begin, l_end;
  // train / recompute modes: activation stores of `act_rows` rows, [rows / 8][cols][8]
  // layout: hst[0] the encoded features (k1_half columns), hst[l] H_l, the output of
  // hidden layer l (1-based, width columns); a null entry is not kept.  The recompute
  // mode reads its input tile from hst[l_begin].
  void* hst[kMaxLayers + 1];
  int64_t act_rows;
  // train / recompute modes of the bf16 8-wave chain: the ReLU masks of H_1..H_n as bits,
  // [n + 1][tiles][waves][dwords][64 lanes] (slot l for H_l), in the backward epilogue's
  // register order; null = not written
  uint32_t* mbits;
  // trace mode
  const int32_t* idx;     // active rays of this step
  const int32_t* count;   // number of active rays
  int32_t* next_idx;      // rays still active after this step
  int32_t* next_count;
  float* t_state;         // per-ray t (the output t)
  uint8_t* hit;
  int32_t* steps;         // may be null
  int step;               // 0-based step index
  float hit_eps, t_max;
  int max_steps;          // pool mode: evaluations per ray at most
  unsigned long long* pool;  // pool mode: rays handed out so far (starts at 0)
  // calib mode: per hidden layer, the max post-ReLU value as ordered uint bits
  unsigned int* amax;
};

__device__ inline void trace_update(const FwdArgs& a, int32_t src, float s) {
  if (a.steps) a.steps[src] = a.step + 1;
  if (fabsf(s) < a.hit_eps) {
    a.hit[src] = 1;
    return;
  }
  const float tn = a.t_state[src] + s;
  a.t_state[src] = tn;
  if (!(tn > a.t_max)) {
    const int32_t slot = atomicAdd(a.next_count, 1);
    a.next_idx[slot] = src;
  }
}

// Encoded inputs of rays [ray0, ray0 + M) into X[:, 0:k1]; padding columns are zero.
// Reduced precisions store the bf16 hi part in columns [0, k1_half) and the lo part
// in [k1_half, k1).  Train mode also writes the features (fp32, or bf16 hi) to the
// feature store hst[0] when there is one, layout [rows / 8][k1_half][8].
template <class E, int M, int LDX, int MODE>
__device__ void encode_tile(const FwdArgs& a, int64_t ray0, E* X) {
  const int n_in = a.n_in, nf = a.n_freq;
  const int khalf = a.lay.k1_half;
  const bool split = sizeof(E) == 2;
  const int items = M * n_in * (1 + nf);
  for (int idx = threadIdx.x; idx < items; idx += blockDim.x) {
    const int r = idx % M;
    const int rest = idx / M;
    const int j = rest % n_in;
    const int kk = rest / n_in;
    const int64_t g = ray0 + r;
    float v = 0.f;
    if (g < a.n) {
      if (MODE == kModeTrace || MODE == kModePool) {
        // the active list (trace) or the workgroup's slots (pool; -1 = empty slot, zeros)
        const int32_t src = a.idx[g];
        if (MODE == kModeTrace || src >= 0) {
          const float tt = a.t_state[src];
          v = fmaf(tt, a.in[(int64_t)(3 + j) * a.stride + src], a.in[(int64_t)j * a.stride + src]);
        }
      } else {
        v = a.in[(int64_t)j * a.stride + g];
      }
    }
    float f0, f1 = 0.f;
    int c0, c1 = -1;
    if (kk == 0) {
      f0 = v; c0 = j;
    } else {
      sincospif(ldexpf(v, kk - 1), &f0, &f1);
      c0 = (2 * kk - 1) * n_in + j;
      c1 = c0 + n_in;
    }
    for (int w = 0; w < 2; ++w) {
      const int c = w == 0 ? c0 : c1;
      if (c < 0) break;
      const float f = w == 0 ? f0 : f1;
      if (split) {
        const E hi = (E)f;
        const E lo = (E)(f - (float)hi);
        X[r * LDX + c] = hi;
        X[r * LDX + khalf + c] = lo;
      } else {
        X[r * LDX + c] = (E)f;
      }
      if (MODE == kModeTrain && a.hst[0])
        reinterpret_cast<E*>(a.hst[0])[((g >> 3) * khalf + c) * 8 + (g & 7)] = (E)f;
    }
  }
  const int pad = khalf - a.lay.n_feat;
  for (int idx = threadIdx.x; idx < M * pad; idx += blockDim.x) {
    const int r = idx % M, c = a.lay.n_feat + idx / M;
    X[r * LDX + c] = (E)0.f;
    if (split) X[r * LDX + khalf + c] = (E)0.f;
    if (MODE == kModeTrain && a.hst[0]) {
      const int64_t g = ray0 + r;
      reinterpret_cast<E*>(a.hst[0])[((g >> 3) * khalf + c) * 8 + (g & 7)] = (E)0.f;
    }
  }
}

// Recompute mode: the kept activation H_(l_begin) of rays [ray0, ray0 + M) into X[:, 0:W]
// (exactly the operand tile the forward pass had in LDS).
template <class E, int M, int LDX, int WIDTH>
__device__ void load_tile(const FwdArgs& a, int64_t ray0, E* X) {
  const E* H = reinterpret_cast<const E*>(a.hst[a.l_begin]);
  for (int idx = threadIdx.x; idx < M * WIDTH; idx += blockDim.x) {
    const int q = idx & 7;
    const int c = (idx >> 3) % WIDTH;
    const int rb = (idx >> 3) / WIDTH;
    X[(rb * 8 + q) * LDX + c] = H[(((ray0 >> 3) + rb) * WIDTH + c) * 8 + q];
  }
}

hipError_t launch_forward(const ddf_net_desc& d, const FwdArgs& a, int64_t n_items,
                          hipStream_t st);
hipError_t launch_pool_trace(const ddf_net_desc& d, const FwdArgs& a, int n_wg, hipStream_t st);
hipError_t launch_forward8(const ddf_net_desc& d, const FwdArgs& a, int64_t n_items,
                           hipStream_t st);

hipError_t launch_pack(const ddf_net_desc& d, const float* master, const float* act_scales,
                       void* packed, hipStream_t st, bool with_transposed);

}  // namespace ddf
