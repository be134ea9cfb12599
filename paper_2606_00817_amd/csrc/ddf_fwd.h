// Arguments of the fused forward kernel and its per-mode hooks.
#pragma once
#include "ddf_internal.h"

namespace ddf {

enum FwdMode {
  kModeQuery = 0,   // t = softplus(z_t), xi = sigmoid(z_xi)
  kModeTrain = 1,   // raw logits + activations kept for the backward pass
  kModeSdf = 2,     // signed distance z_0 at points
  kModeTrace = 3    // one sphere-tracing step over the active-ray list
};

struct FwdArgs {
  const float* in;        // SoA inputs [n_in][stride]; trace mode: rays [6][stride]
  int64_t n;              // items (trace mode: capacity of the active list)
  int64_t stride;         // row stride of `in`
  const uint8_t* packed;
  Layout lay;
  int n_in, n_freq, n_hidden, n_out;
  int mode;
  float* out0;            // query: t; train: z_t; sdf: s
  float* out1;            // query: xi; train: z_xi
  // train mode: activation store, slabs of `act_rows` rows in [rows / 8][cols][8] layout:
  // the encoded features (k1_half columns) then H_1 .. H_n (width columns each).
  void* act;
  int64_t act_rows;
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

hipError_t launch_forward(const ddf_net_desc& d, const FwdArgs& a, int64_t n_items,
                          hipStream_t st);

hipError_t launch_pack(const ddf_net_desc& d, const float* master, const float* act_scales,
                       void* packed, hipStream_t st, bool with_transposed);

}  // namespace ddf
