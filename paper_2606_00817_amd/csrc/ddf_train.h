// Training-path declarations (forward with kept activations, loss, backward, Adam).
#pragma once
#include "ddf_internal.h"

namespace ddf {
int fail(int code, const char* fmt, ...);
int hip_status(hipError_t e, const char* what);
int check_desc(const ddf_net_desc* d);
int check_ptr(const void* p, const char* name);
void g_err_clear();
}  // namespace ddf
