// Training path of libddf: kept activations, distillation loss, backward, Adam.
#include "ddf_fwd.h"
#include "ddf_train.h"

using namespace ddf;

extern "C" {

size_t ddf_train_workspace_bytes(const ddf_net_desc* d, int64_t batch) { return 0; }

int ddf_forward_train(const ddf_net_desc* d, const void* packed, const float* rays, int64_t n,
                      float* z_t, float* z_xi, void* ws, size_t ws_bytes, void* stream) {
  return fail(DDF_ERR_UNSUPPORTED, "training not built yet");
}

int ddf_backward(const ddf_net_desc* d, const void* packed, const float* rays, int64_t n,
                 const float* grad_z_t, const float* grad_z_xi, float* grad_params, void* ws,
                 size_t ws_bytes, void* stream) {
  return fail(DDF_ERR_UNSUPPORTED, "training not built yet");
}

int ddf_train_step(const ddf_net_desc* d, float* master, float* adam_m, float* adam_v, void* packed,
                   const float* rays, const float* t_gt, const uint8_t* hit_gt, int64_t batch,
                   const ddf_train_hparams* hp, float* loss_out, int32_t* nonfinite_flag,
                   float* grad_out, void* ws, size_t ws_bytes, void* stream) {
  return fail(DDF_ERR_UNSUPPORTED, "training not built yet");
}

}  // extern "C"
