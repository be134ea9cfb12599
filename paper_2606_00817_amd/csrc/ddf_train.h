// Training-path declarations (forward with kept activations, loss, backward, Adam).
#pragma once
#include "ddf_internal.h"

namespace ddf {
int fail(int code, const char* fmt, ...);
int hip_status(hipError_t e, const char* what);
int check_desc(const ddf_net_desc* d);
int check_ptr(const void* p, const char* name);
void g_err_clear();
int check_hp_public(const ddf_train_hparams* hp);
int launch_ddf_loss(const float* zt, const float* zx, const float* t_gt, const uint8_t* hit, int64_t n, int64_t R,
                    float* partial, float* scal, float* loss_out, float* dzt, float* dzx, float bce_weight,
                    float clamp, hipStream_t st);
int launch_adam_flat(float* p, float* m, float* v, const float* g, int64_t P, const ddf_train_hparams* hp,
                     int32_t* flag, hipStream_t st);
int loss_scratch_floats();
}  // namespace ddf
