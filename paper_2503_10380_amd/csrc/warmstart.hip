// Warm starts across amplitude iterations.
//
// The paper's "optimal guess" restarts ALS from the previous converged
// factors (Section "An improved initial guess strategy").  This file adds two
// candidates computed from the change of the amplitudes dt:
//  * first order: the PPL tensor is linear in t, so one matrix-free MTTKRP of
//    dR (the chain evaluated on dt) at the previous factors, solved with the
//    previous W, gives the first-order change of each factor column
//    D_m = M_m(dR) W_m^{-1} / lambda;
//  * learned: the first-order candidate plus a per-column network's correction:
//    the network maps [previous columns, D columns, log10 of the relative step
//    ||dt|| / ||t||] of the four factors to the part of the change of the
//    columns that the first-order change misses (an untrained network leaves
//    the first-order candidate).
// Features and targets are stored raw; cpppl_mlp_standardize fits per-column
// centring and scaling on the stored rows (so the network sees O(1) numbers
// whatever the step and mode sizes), and the learned candidate applies it on
// the way in and undoes it on the way out.  The judge keeps, of the plain
// warm start and the candidates formed, the one with the lowest
// ||CP||^2 - 2 <R, CP> for the new t.
#include <cmath>
#include <limits>
#include <stdexcept>

#include "mlp.h"
#include "ops.h"
#include "ws.h"

using namespace cpppl;

namespace {

constexpr int TPB = 256;
unsigned nb(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + TPB - 1) / TPB, 1 << 16)); }

// D[r][n] /= lam[r] (zero rows stay zero)
__global__ void div_rows_kernel(double* D, const double* lam, int64_t R, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < R * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double l = lam[e / n];
    D[e] = l > 0.0 ? D[e] / l : 0.0;
  }
}

// acc[0] += sum x^2 (single block, fixed order)
__global__ __launch_bounds__(TPB) void sumsq_kernel(const double* x, int64_t n, double* acc) {
  __shared__ double sh[TPB];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += TPB) s += x[i] * x[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = TPB / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[0] += sh[0];
}

// out[0] = log10(sqrt(acc[0] / acc[1])), the relative step size; -30 for a zero step
__global__ void log_ratio_kernel(const double* acc, double* out) {
  const double r = sqrt(acc[0] / acc[1]);
  out[0] = (r > 0.0 && isfinite(r)) ? log10(r) : -30.0;
}

// y[r][col] = (float)value[0] for every row r
__global__ void fill_col_kernel(float* y, int64_t R, int64_t ldy, int64_t col, const double* value) {
  const float v = (float)value[0];
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < R;
       r += (int64_t)gridDim.x * blockDim.x)
    y[r * ldy + col] = v;
}

// y[r][off + i] = (float)(x[r][i] * (scale ? *scale : 1))
__global__ void pack_kernel(const double* x, int64_t R, int64_t n, const double* scale, float* y,
                            int64_t ldy, int64_t off) {
  const double s = scale ? scale[0] : 1.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < R * n;
       e += (int64_t)gridDim.x * blockDim.x)
    y[(e / n) * ldy + off + e % n] = (float)(x[e] * s);
}

// y[r][off + i] -= (float)D[r][i]
__global__ void sub_rows_kernel(float* y, int64_t ldy, int64_t off, const double* D, int64_t R,
                                int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < R * n;
       e += (int64_t)gridDim.x * blockDim.x)
    y[(e / n) * ldy + off + e % n] -= (float)D[e];
}

// F[r][i] = F0[r][i] + (D ? D[r][i] : 0) + (Y ? Y[r][off + i] : 0)
__global__ void candidate_kernel(const double* F0, const double* D, const float* Y, int64_t ldy,
                                 int64_t off, int64_t R, int64_t n, double* F) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < R * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double v = F0[e];
    if (D) v += D[e];
    if (Y) v += (double)Y[(e / n) * ldy + off + e % n];
    F[e] = v;
  }
}

void set_candidate(cpppl_ctx* c, const double* const D[4], const float* Y, int64_t ldy) {
  const Plan& p = c->plan;
  const int64_t R = c->d.rank;
  int64_t off = 0;
  for (int m = 0; m < 4; ++m) {
    const int64_t n = ws_nmode(c->d, m);
    hipLaunchKernelGGL(candidate_kernel, dim3(nb(R * n)), dim3(TPB), 0, c->stream,
                       c->at<double>(p.wsF[m]), D ? D[m] : nullptr, Y, ldy, off, R, n,
                       c->at<double>(p.FT[m]));
    CPPPL_LAUNCH_CHECK("candidate");
    off += n;
  }
  ws_copy(c, p.lam, p.wsLam, (size_t)R * 8);
  ws_init_after_factors(c);
}

}  // namespace

#define WS_TRY(c)                                      \
  if (!(c)) return CPPPL_E_ARG;                        \
  if ((c)->hip_failed) return CPPPL_E_HIP;             \
  try {                                                \
    CPPPL_HIP(hipSetDevice((c)->device));
#define WS_CATCH(c)                                                      \
  }                                                                      \
  catch (const StatusError& e) {                                         \
    (c)->err = e.msg;                                                    \
    return e.st;                                                         \
  }                                                                      \
  catch (const HipError& e) {                                            \
    (c)->hip_failed = true;                                              \
    (c)->err = std::string(e.where) + ": " + hipGetErrorString(e.err);   \
    return CPPPL_E_HIP;                                                  \
  }                                                                      \
  catch (const std::invalid_argument& e) {                               \
    (c)->err = e.what();                                                 \
    return CPPPL_E_ARG;                                                  \
  }                                                                      \
  catch (const std::exception& e) {                                      \
    (c)->err = e.what();                                                 \
    return CPPPL_E_STATE;                                                \
  }                                                                      \
  (c)->err.clear();                                                      \
  return CPPPL_OK;

extern "C" {

CPPPL_API int64_t cpppl_ws_in_dim(const cpppl_dims* d) { return d ? 2 * (2 * d->o + 2 * d->v) + 1 : 0; }
CPPPL_API int64_t cpppl_ws_out_dim(const cpppl_dims* d) { return d ? (2 * d->o + 2 * d->v) : 0; }

CPPPL_API cpppl_status cpppl_warm_start(cpppl_ctx* c, const double* dt, int on_device,
                                        int strategy, cpppl_mlp* mlp, int* chosen) {
  WS_TRY(c)
  if (!dt) throw std::invalid_argument("dt is NULL");
  if (strategy < CPPPL_WS_PLAIN || strategy > CPPPL_WS_NEAR_OPTIMAL)
    throw std::invalid_argument("unknown warm-start strategy");
  if (!c->ws) throw StatusError(CPPPL_E_STATE, "no workspace bound");
  if (c->planted || !c->have_t || !c->have_b || !c->have_factors)
    throw StatusError(CPPPL_E_STATE, "warm start needs t, B and factors");
  const int64_t in_dim = cpppl_ws_in_dim(&c->d), out_dim = cpppl_ws_out_dim(&c->d);
  if (strategy == CPPPL_WS_LEARNED) {
    if (!mlp) throw std::invalid_argument("the learned warm start needs a network");
    if (mlp->sizes.front() != in_dim || mlp->sizes.back() != out_dim)
      throw std::invalid_argument("network shape does not match these dims");
  }
  const Plan& p = c->plan;
  const int64_t R = c->d.rank;
  double* sc = c->at<double>(p.scal);

  if (strategy == CPPPL_WS_NEAR_OPTIMAL) {  // the cached (n-5)th iterate, no features
    ws_load_dt(c, dt, on_device);
    ws_add_dt(c);
    ws_derive_t(c);
    const bool used = ws_install_near_cache(c);
    c->ws_valid = false;
    ws_sync(c);
    if (chosen) *chosen = used ? CPPPL_WS_NEAR_OPTIMAL : CPPPL_WS_PLAIN;
    return CPPPL_OK;
  }

  // previous (converged) factors
  for (int m = 0; m < 4; ++m) ws_copy(c, p.wsF[m], p.FT[m], (size_t)(ws_nmode(c->d, m) * R) * 8);
  ws_copy(c, p.wsLam, p.lam, (size_t)R * 8);

  // first-order change from the MTTKRP of dR at the previous factors
  ws_load_dt(c, dt, on_device);
  for (int m = 0; m < 4; ++m) {
    const int64_t n = ws_nmode(c->d, m);
    ws_mttkrp_dt(c, m);
    ws_solve_no_update(c, m, p.wsD[m]);
    hipLaunchKernelGGL(div_rows_kernel, dim3(nb(R * n)), dim3(TPB), 0, c->stream,
                       c->at<double>(p.wsD[m]), c->at<double>(p.wsLam), R, n);
    CPPPL_LAUNCH_CHECK("div_rows");
  }
  // the relative step size ||dt|| / ||t|| (t before the step), as log10
  const int64_t nt = c->d.o * c->d.o * c->d.v * c->d.v;
  zero_doubles(sc + S_WS_SUMSQ, 2, c->stream);
  hipLaunchKernelGGL(sumsq_kernel, dim3(1), dim3(TPB), 0, c->stream, c->at<double>(p.dt64), nt,
                     sc + S_WS_SUMSQ);
  hipLaunchKernelGGL(sumsq_kernel, dim3(1), dim3(TPB), 0, c->stream, ws_t_doubles(c), nt,
                     sc + S_WS_SUMSQ + 1);
  CPPPL_LAUNCH_CHECK("sumsq");
  hipLaunchKernelGGL(log_ratio_kernel, dim3(1), dim3(1), 0, c->stream, sc + S_WS_SUMSQ,
                     sc + S_WS_SCALE);
  CPPPL_LAUNCH_CHECK("log_ratio");

  // features [F_gamma, F_rho, F_alpha, F_beta, D_gamma, D_rho, D_alpha, D_beta, log10 step]
  float* feat = c->at<float>(p.wsFeat);
  int64_t off = 0;
  for (int m = 0; m < 4; ++m) {
    const int64_t n = ws_nmode(c->d, m);
    hipLaunchKernelGGL(pack_kernel, dim3(nb(R * n)), dim3(TPB), 0, c->stream,
                       c->at<double>(p.wsF[m]), R, n, (const double*)nullptr, feat, in_dim, off);
    hipLaunchKernelGGL(pack_kernel, dim3(nb(R * n)), dim3(TPB), 0, c->stream,
                       c->at<double>(p.wsD[m]), R, n, (const double*)nullptr, feat, in_dim,
                       out_dim + off);
    CPPPL_LAUNCH_CHECK("pack");
    off += n;
  }
  hipLaunchKernelGGL(fill_col_kernel, dim3(nb(R)), dim3(TPB), 0, c->stream, feat, R, in_dim,
                     in_dim - 1, (const double*)(sc + S_WS_SCALE));
  CPPPL_LAUNCH_CHECK("fill_col");
  if (strategy == CPPPL_WS_LEARNED) {
    // the network sees the features standardised as its training rows were,
    // on a copy (the raw features stay for cpppl_ws_training_rows)
    float* xin = c->at<float>(p.wsFeatStd);
    CPPPL_HIP(hipMemcpyAsync(xin, feat, (size_t)(R * in_dim) * 4, hipMemcpyDeviceToDevice,
                             c->stream));
    mlp_std_x_dev(mlp, xin, in_dim, R, c->stream);
    mlp_forward_dev(mlp, xin, R, c->at<float>(p.wsOut), c->stream);
    mlp_unscale_y_dev(mlp, c->at<float>(p.wsOut), out_dim, R, c->stream);
  }

  // the new amplitudes: t <- t + dt
  ws_add_dt(c);
  ws_derive_t(c);

  // the judge: the lowest ||CP||^2 - 2 <R, CP> at the new t among the plain
  // start, the first-order candidate and (LEARNED) the network's
  int pick = CPPPL_WS_PLAIN;
  if (strategy != CPPPL_WS_PLAIN) {
    double best = ws_judge_loss(c);  // factors are still the previous ones
    const double* D[4];
    for (int m = 0; m < 4; ++m) D[m] = c->at<double>(p.wsD[m]);
    set_candidate(c, D, nullptr, 0);
    const double l_fo = ws_judge_loss(c);
    if (std::isfinite(l_fo) && l_fo < best) {
      best = l_fo;
      pick = CPPPL_WS_FIRST_ORDER;
    }
    if (strategy == CPPPL_WS_LEARNED) {
      set_candidate(c, D, c->at<float>(p.wsOut), out_dim);
      const double l_learn = ws_judge_loss(c);
      if (std::isfinite(l_learn) && l_learn < best) {
        best = l_learn;
        pick = CPPPL_WS_LEARNED;
      }
    }
    if (pick == CPPPL_WS_PLAIN) set_candidate(c, nullptr, nullptr, 0);
    else if (pick == CPPPL_WS_FIRST_ORDER && strategy == CPPPL_WS_LEARNED) set_candidate(c, D, nullptr, 0);
  }
  c->ws_valid = true;
  ws_sync(c);
  if (chosen) *chosen = pick;
  WS_CATCH(c)
}

CPPPL_API cpppl_status cpppl_ws_training_rows(cpppl_ctx* c, cpppl_mlp* mlp) {
  WS_TRY(c)
  if (!mlp) throw std::invalid_argument("mlp is NULL");
  if (!c->ws_valid) throw StatusError(CPPPL_E_STATE, "no warm start to learn from");
  const int64_t in_dim = cpppl_ws_in_dim(&c->d), out_dim = cpppl_ws_out_dim(&c->d);
  if (mlp->sizes.front() != in_dim || mlp->sizes.back() != out_dim)
    throw std::invalid_argument("network shape does not match these dims");
  const Plan& p = c->plan;
  const int64_t R = c->d.rank;
  float* y = c->at<float>(p.wsOut);
  int64_t off = 0;
  // target = aligned converged column - previous column - first-order change
  for (int m = 0; m < 4; ++m) {
    const int64_t n = ws_nmode(c->d, m);
    aligned_delta_f32(c->at<double>(p.FT[m]), c->at<double>(p.wsF[m]), R, n, y + off, out_dim,
                      c->stream);
    hipLaunchKernelGGL(sub_rows_kernel, dim3(nb(R * n)), dim3(TPB), 0, c->stream, y, out_dim, off,
                       (const double*)c->at<double>(p.wsD[m]), R, n);
    CPPPL_LAUNCH_CHECK("sub_rows");
    off += n;
  }
  mlp_append_dev(mlp, c->at<float>(p.wsFeat), in_dim, y, out_dim, R, c->stream);
  ws_sync(c);
  WS_CATCH(c)
}

}  // extern "C"
