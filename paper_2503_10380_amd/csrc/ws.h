// Internal helpers shared between the ALS driver and the warm-start code.
#pragma once

#include <string>

#include "ctx.h"

namespace cpppl {

struct StatusError {
  cpppl_status st;
  std::string msg;
  StatusError(cpppl_status s, std::string m);
};

// MTTKRP of `mode` at the current factors into the MT buffer (R x n, FP64).
void ws_mttkrp_into_MT(cpppl_ctx* c, DType dt, int mode);
// buffer at out_off (R x n) <- W_mode^{-1} MT with the current Grams.
void ws_solve_no_update(cpppl_ctx* c, int mode, size_t out_off);
// Grams, low-precision copies and the eta reference after the factors changed.
void ws_init_after_factors(cpppl_ctx* c);
// t <- t + dt (the loaded dt; with singles the raw doubles follow, tau = t2 + t1 t1).
void ws_add_dt(cpppl_ctx* c);
// Re-derive the operand layouts of t from the FP64 master.
void ws_derive_t(cpppl_ctx* c);
void ws_ensure_norm(cpppl_ctx* c);
bool ws_install_near_cache(cpppl_ctx* c);
void ws_copy(cpppl_ctx* c, size_t dst, size_t src, size_t bytes);
void ws_sync(cpppl_ctx* c);
// The doubles amplitudes (the raw t2 when a singles dressing is on).
const double* ws_t_doubles(cpppl_ctx* c);
int64_t ws_nmode(const cpppl_dims& d, int m);
// MTTKRP of `mode` with dt (loaded by ws_load_dt) in place of t, into MT.
void ws_mttkrp_dt(cpppl_ctx* c, int mode);
void ws_load_dt(cpppl_ctx* c, const double* dt, int on_device);
// ||CP||^2 - 2 <R, CP> at the current factors (synchronises).
double ws_judge_loss(cpppl_ctx* c);

}  // namespace cpppl
