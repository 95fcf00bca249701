// Learned warm start (placeholder until the network kernels land).
#include "ws.h"

extern "C" {
CPPPL_API int64_t cpppl_ws_in_dim(const cpppl_dims* d) { return d ? 2 * (2 * d->o + 2 * d->v) : 0; }
CPPPL_API int64_t cpppl_ws_out_dim(const cpppl_dims* d) { return d ? (2 * d->o + 2 * d->v) : 0; }
CPPPL_API cpppl_status cpppl_mlp_create(int, int, int, int, int64_t, uint64_t, int, cpppl_mlp** out) {
  if (out) *out = nullptr;
  return CPPPL_E_UNSUPPORTED;
}
CPPPL_API cpppl_status cpppl_mlp_destroy(cpppl_mlp*) { return CPPPL_E_UNSUPPORTED; }
CPPPL_API cpppl_status cpppl_mlp_num_params(const cpppl_mlp*, int64_t*) { return CPPPL_E_UNSUPPORTED; }
CPPPL_API cpppl_status cpppl_mlp_get_params(cpppl_mlp*, float*, int) { return CPPPL_E_UNSUPPORTED; }
CPPPL_API cpppl_status cpppl_mlp_set_params(cpppl_mlp*, const float*, int) { return CPPPL_E_UNSUPPORTED; }
CPPPL_API cpppl_status cpppl_mlp_forward(cpppl_mlp*, const float*, int64_t, float*, int) { return CPPPL_E_UNSUPPORTED; }
CPPPL_API cpppl_status cpppl_mlp_grad(cpppl_mlp*, const float*, const float*, int64_t, float*, float*, int) { return CPPPL_E_UNSUPPORTED; }
CPPPL_API cpppl_status cpppl_mlp_add_rows(cpppl_mlp*, const float*, const float*, int64_t, int) { return CPPPL_E_UNSUPPORTED; }
CPPPL_API cpppl_status cpppl_mlp_clear_rows(cpppl_mlp*) { return CPPPL_E_UNSUPPORTED; }
CPPPL_API cpppl_status cpppl_mlp_train(cpppl_mlp*, int, float, int64_t, uint64_t, float*) { return CPPPL_E_UNSUPPORTED; }
CPPPL_API cpppl_status cpppl_mlp_save(cpppl_mlp*, const char*) { return CPPPL_E_UNSUPPORTED; }
CPPPL_API cpppl_status cpppl_mlp_load(cpppl_mlp*, const char*) { return CPPPL_E_UNSUPPORTED; }
CPPPL_API cpppl_status cpppl_warm_start(cpppl_ctx*, const double*, int, int, cpppl_mlp*, int*) { return CPPPL_E_UNSUPPORTED; }
CPPPL_API cpppl_status cpppl_ws_training_rows(cpppl_ctx*, cpppl_mlp*) { return CPPPL_E_UNSUPPORTED; }
}
