// Per-rank-column warm-start network: a ReLU MLP in FP32 with hand-written
// forward, backward and Adam kernels (internal interface).
#pragma once

#include <string>
#include <vector>

#include "../../include/cpppl.h"
#include "common.h"

struct cpppl_mlp {
  int device = 0;
  std::vector<int> sizes;  // in, hidden..., out
  int nl = 0;              // linear layers
  int64_t nparams = 0;
  std::vector<int64_t> woff, boff;
  float* params = nullptr;
  float* grads = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  int64_t adam_step = 0;
  // stored training rows
  int64_t cap = 0, nrows = 0;
  float* xs = nullptr;
  float* ys = nullptr;
  // per-batch work: activations of every layer, gradient buffers, batch copies
  int64_t work_rows = 0;
  float* work = nullptr;
  float* scal = nullptr;      // device scalars (loss partials)
  float* host_scal = nullptr; // pinned
  // standardisation of the warm-start rows (cpppl_mlp_standardize): inputs
  // x' = (x - x_mu) x_inv per column, targets y' = y / y_sc per column
  bool standardized = false;
  float* x_mu = nullptr;
  float* x_inv = nullptr;
  float* y_sc = nullptr;
  std::string err;
};

namespace cpppl {

// Forward pass on n rows of x (device) into y (device, n x out); keeps activations.
void mlp_forward_dev(cpppl_mlp* m, const float* x, int64_t n, float* y, hipStream_t s);
// Loss (device scalar in m->scal[0]) and gradients (m->grads) for rows x, targets y.
void mlp_loss_grad_dev(cpppl_mlp* m, const float* x, const float* y, int64_t n, hipStream_t s);
void mlp_ensure_work(cpppl_mlp* m, int64_t rows);
// In place: x[r][:] = (x[r][:] - x_mu) x_inv (row stride ldx), a no-op unless standardised.
void mlp_std_x_dev(cpppl_mlp* m, float* x, int64_t ldx, int64_t n, hipStream_t s);
// In place: y[r][:] *= y_sc (row stride ldy), a no-op unless standardised.
void mlp_unscale_y_dev(cpppl_mlp* m, float* y, int64_t ldy, int64_t n, hipStream_t s);
// Append device rows to the training set (standardised on the way in once the
// network is).
void mlp_append_dev(cpppl_mlp* m, const float* x, int64_t ldx, const float* y, int64_t ldy,
                    int64_t n, hipStream_t s);

}  // namespace cpppl
