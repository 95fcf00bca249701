// Internal state of a CP-PPL context (not part of the C ABI).
#pragma once

#include <string>
#include <vector>

#include "../../include/cpppl.h"
#include "common.h"
#include "gemm.h"

namespace cpppl {

// Offsets of every device buffer inside the caller-bound workspace.
struct Plan {
  size_t total = 0;
  // inputs, FP64 masters and layouts
  size_t t64, t64T, tdc, b64, b64T, b64P;
  // bfloat16 operand copies (BF16 contexts)
  size_t t16, t16T, b16T, b16P;
  // e4m3 operand copies and their power-of-two scales (FP8 contexts): sT per ij,
  // sB per X, sBx[X*v + q] = sB[X]
  size_t t8, t8T, b8T, b8P, sT, sB, sBx;
  // singles (dims.singles): raw doubles t2 (t64 then holds tau), t1, D_vo, and
  // Dbar with the same layouts and copies as B
  size_t t2raw, t1, bvo, bb64, bb64T, bb64P, bb16T, bb16P, bb8T, bb8P, sBb, sBbx;
  // factors (transposed, R x n), weights, snapshots, Grams
  size_t FT[4], F16T[4], lam;
  size_t FTprev[2][4], lamprev[2];  // two snapshot slots: the states before the last two sweeps
  size_t gram[4], cross[4], invA, invB, invD, MT, stage, nearRing, nearCache;
  // intermediates: one region [tau | Ya | Yb | Z]; G aliases Z
  size_t big, tau, Ya, Yb, Z;
  size_t big_bytes;
  size_t Kt, HT, partial, partial_elems;
  size_t rowbuf, sums, scal, status;
  // planted CP tensor
  size_t FpT[4], lamp, Cp;
  // warm start: previous factors, first-order change, features / targets, dt layouts
  size_t wsF[4], wsLam, wsFeat, wsFeatStd, wsOut, wsD[4];
  size_t dt64, dt64T, dt16, dt16T;
  // orbital energies of the Jacobi step: e_occ (o) then e_vir (v)
  size_t eorb;
};

enum Scal {  // slots of the device scalar block
  S_NORM_R2 = 0,
  S_E_EXACT = 1,
  S_FIT = 8,     // 8..12: inner, cp2, res2, fit, loss
  S_ETA = 16,    // 16..19: nn, np, pp, eta
  S_ENERGY = 20,
  S_CP2_PREV = 21,
  S_JUDGE = 24,  // 24..28 judge fit scalars
  S_WS_SCALE = 30,  // log10 of the relative step ||dt|| / ||t|| (a warm-start feature)
  S_WS_SUMSQ = 32,  // 32..33: ||dt||^2 and ||t||^2
  S_COUNT = 64
};

struct Path {
  DType dt;
  size_t esz;
  bool fp8 = false;          // T2, T2T, BnT, Bp hold e4m3 codes
  const float* sT = nullptr;   // scale of t row ij
  const float* sBx = nullptr;  // scale of B^X, repeated per (X, q)
  const void* T2;   // t[ij][cd]   (o^2 x v^2)
  const void* T2T;  // t[cd][ij]   (v^2 x o^2)
  const void* BnT;  // B[X][q][p]  = B^X_pq       (alpha side)
  const void* Bp;   // B[p][X][q]  = B^X_pq
  const void* BnT_b;  // the same layouts of the b-side operand: Dbar with singles, else B
  const void* Bp_b;
  const float* sBx_b = nullptr;  // its e4m3 scales
  const void* FTop[4];
};

}  // namespace cpppl

struct cpppl_ctx {
  cpppl_dims d{};
  cpppl_precision prec = CPPPL_FP64;
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  bool hip_failed = false;

  char* ws = nullptr;
  size_t ws_bytes = 0;
  cpppl::Plan plan;

  bool have_t = false, have_b = false, have_factors = false, planted = false;
  bool singles_on = false;  // t64 holds tau and the b side uses Dbar
  int64_t rank_p = 0;
  bool norm_valid = false;
  bool ybeta_valid = false;
  // tau holds KR(gamma, rho)^T t at the current gamma, rho in tau_dt: formed at
  // the end of a sweep that evaluates E_CP, and reused by the next sweep
  bool tau_valid = false;
  cpppl::DType tau_dt = cpppl::DType::F64;
  bool want_energy = false;  // sweeps evaluate E_CP (per-sweep energy history / energy stop)
  // test hook: the W_alpha inverse forked early for sweep `inject_alpha_fault`
  // of the next cpppl_als call reports a failed pivot (-1: off)
  int inject_alpha_fault = -1;
  bool inject_now = false;
  bool want_eta = true;  // sweeps evaluate eta (eq. N3_stopping)
  bool near_valid = false;  // the near-optimal cache holds an iterate
  cpppl::DType ybeta_dt = cpppl::DType::F64;
  bool ws_valid = false;      // warm-start snapshot (wsF) holds the factors before the last warm start

  hipStream_t side = nullptr;     // inverse of W overlapped with the MTTKRP chain
  hipEvent_t ev_main = nullptr, ev_side = nullptr;
  hipEvent_t ev_done[2] = {nullptr, nullptr};  // a sweep's results reached host_scal slot k
  int launch_chunks = 1;  // launches per unsplit BF16 product (more while a side inverse is pending)
  int snap = 0;  // snapshot slot holding the state before the most recently issued sweep
  // -W_alpha^{-1} of the next sweep is queued on the side stream (forked at the
  // end of the previous sweep); cleared by that sweep, or by waiting for it
  bool alpha_forked = false;
  double* inv = nullptr;          // buffer holding -W^{-1} of the last prepared mode

  double* host_scal = nullptr;  // pinned, two slots of S_COUNT doubles + 16 status ints
  int* host_status = nullptr;   // = (int*)(host_scal + S_COUNT)

  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  // timed spans of a class; `calls` is 1 for the span that counts the call
  // (a product cut into several launches gives one span per launch, the first
  // counting the call)
  struct Seg { int cls; hipEvent_t a, b; int calls; };
  std::vector<Seg> segs;
  struct SpanState { int cls; bool has_sub; };
  SpanState* span = nullptr;  // innermost open class span

  template <typename T = void>
  T* at(size_t off) { return (T*)(ws + off); }
};
