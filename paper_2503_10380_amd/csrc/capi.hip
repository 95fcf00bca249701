// C ABI, workspace plan and ALS driver of the CP-PPL library.
//
// One sweep updates alpha, beta, gamma, rho in that order.  The MTTKRP of each
// factor is evaluated matrix-free (eq. distribute / eq. foreachr and the same
// idea for the occupied factors):
//   tau[r][c][d] = sum_ij gamma_ir rho_jr t_ijcd                     (shared by a, b)
//   Y_F[r][X][q] = sum_p F_pr B^X_pq                                  (F = alpha or beta)
//   alpha: Z[r][X][c] = sum_d Y_beta[r][X][d] tau[r][c][d],  M[r][a] = sum_Xc B^X_ac Z[r][X][c]
//   beta:  Z[r][X][d] = sum_c Y_alpha[r][X][c] tau[r][c][d], M[r][b] = sum_Xd B^X_bd Z[r][X][d]
//   G[r][c][d] = sum_X Y_alpha[r][X][c] Y_beta[r][X][d],  H[r][ij] = sum_cd G[r][cd] t_ijcd
//   gamma: M[r][i] = sum_j H[r][ij] rho_jr;  rho: M[r][j] = sum_i H[r][ij] gamma_ir
// then F^T = W^{-1} M^T with W the Hadamard product of the other three Grams,
// inverted in FP64 by the block sweep (Gauss-Jordan) operator where the paper
// takes a Cholesky factorisation, and the rows of F^T are scaled to unit 2-norm
// (the norms are lambda).  Y_beta of the updated beta is kept for the next
// sweep's alpha update (caching of intermediates across gradient evaluations).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <stdexcept>
#include <string>

#include "../../include/cpppl_testing.h"
#include "ctx.h"
#include "linalg.h"
#include "ops.h"
#include "ws.h"

using namespace cpppl;

namespace cpppl {

StatusError::StatusError(cpppl_status s, std::string m) : st(s), msg(std::move(m)) {}

namespace {

constexpr size_t ALIGN = 256;
constexpr int MAX_RANK = 4096;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

int64_t nmode(const cpppl_dims& d, int m) { return m < 2 ? d.o : d.v; }

Plan build_plan(const cpppl_dims& d, cpppl_precision prec) {
  Plan p;
  size_t off = 0;
  auto add = [&](size_t bytes) {
    size_t o = off;
    off += align_up(std::max<size_t>(bytes, 8));
    return o;
  };
  const int64_t o = d.o, v = d.v, X = d.nx, R = d.rank;
  const size_t o2v2 = (size_t)(o * o * v * v), xv2 = (size_t)(X * v * v);
  const bool lp = prec != CPPPL_FP64;   // bfloat16 factors and intermediates
  const bool bf = prec == CPPPL_BF16;   // bfloat16 t and B
  const bool f8 = prec == CPPPL_FP8_E4M3;  // e4m3 t and B with scales
  p.t64 = add(o2v2 * 8);
  p.t64T = add(o2v2 * 8);
  p.b64 = add(xv2 * 8);
  p.b64T = add(xv2 * 8);
  p.b64P = add(xv2 * 8);
  p.t16 = bf ? add(o2v2 * 2) : 0;
  p.t16T = bf ? add(o2v2 * 2) : 0;
  p.b16T = bf ? add(xv2 * 2) : 0;
  p.b16P = bf ? add(xv2 * 2) : 0;
  p.t8 = f8 ? add(o2v2) : 0;
  p.t8T = f8 ? add(o2v2) : 0;
  p.b8T = f8 ? add(xv2) : 0;
  p.b8P = f8 ? add(xv2) : 0;
  p.sT = f8 ? add((size_t)(o * o) * 4) : 0;
  p.sB = f8 ? add((size_t)X * 4) : 0;
  p.sBx = f8 ? add((size_t)(X * v) * 4) : 0;
  const bool sg = d.singles != 0;
  p.t2raw = sg ? add(o2v2 * 8) : 0;
  p.t1 = sg ? add((size_t)(o * v) * 8) : 0;
  p.bvo = sg ? add((size_t)(X * v * o) * 8) : 0;
  p.bb64 = sg ? add(xv2 * 8) : 0;
  p.bb64T = sg ? add(xv2 * 8) : 0;
  p.bb64P = sg ? add(xv2 * 8) : 0;
  p.bb16T = (sg && bf) ? add(xv2 * 2) : 0;
  p.bb16P = (sg && bf) ? add(xv2 * 2) : 0;
  p.bb8T = (sg && f8) ? add(xv2) : 0;
  p.bb8P = (sg && f8) ? add(xv2) : 0;
  p.sBb = (sg && f8) ? add((size_t)X * 4) : 0;
  p.sBbx = (sg && f8) ? add((size_t)(X * v) * 4) : 0;
  for (int m = 0; m < 4; ++m) {
    const size_t n = (size_t)nmode(d, m);
    p.FT[m] = add(n * R * 8);
    p.FTprev[0][m] = add(n * R * 8);
    p.FTprev[1][m] = add(n * R * 8);
    p.F16T[m] = lp ? add(n * R * 2) : 0;
    p.gram[m] = add((size_t)R * R * 8);
    p.cross[m] = add((size_t)R * R * 8);
    p.FpT[m] = add(n * R * 8);
    p.wsF[m] = add(n * R * 8);
    p.wsD[m] = add(n * R * 8);
  }
  p.lam = add(R * 8);
  p.lamprev[0] = add(R * 8);
  p.lamprev[1] = add(R * 8);
  p.lamp = add(R * 8);
  p.wsLam = add(R * 8);
  p.Cp = add((size_t)R * R * 8);
  p.invA = add((size_t)R * R * 8);
  p.invB = add((size_t)R * R * 8);
  p.invD = add((size_t)INV_DBUF * 8);
  // near-optimal cache: one factor set = (2o + 2v) R + R doubles; a ring of six plus the cache
  const size_t set_e = (size_t)((2 * o + 2 * v) * R + R);
  p.nearRing = add(6 * set_e * 8);
  p.nearCache = add(set_e * 8);
  const int64_t nmax = std::max(o, v);
  p.MT = add((size_t)nmax * R * 8);
  p.stage = add((size_t)std::max<int64_t>(nmax * R, R * R) * 8);
  p.wsFeat = add((size_t)R * (2 * (2 * o + 2 * v) + 1) * 4);
  p.wsFeatStd = add((size_t)R * (2 * (2 * o + 2 * v) + 1) * 4);
  p.wsOut = add((size_t)R * (2 * o + 2 * v) * 4);
  p.dt64 = add(o2v2 * 8);
  p.dt64T = add(o2v2 * 8);
  p.dt16 = bf ? add(o2v2 * 2) : 0;
  p.dt16T = bf ? add(o2v2 * 2) : 0;
  p.eorb = add((size_t)(o + v) * 8);
  // intermediates, sized for FP64 and shared by the BF16 path
  const size_t tau_e = (size_t)(R * v * v), y_e = (size_t)(R * X * v);
  const size_t z_e = (size_t)(R * std::max(X, v) * v);  // Z, and G (R v^2) aliased on it
  size_t big_e = tau_e + 2 * y_e + z_e;
  // the one-time ||R||^2 pass reuses this region: t with (c, d) swapped plus
  // at least one a-block of (ac|bd) and of R
  big_e = std::max(big_e, o2v2 + (size_t)(v * v * v) + (size_t)(o * o * v) + 64);
  p.big = add(big_e * 8);
  p.big_bytes = big_e * 8;
  p.tau = p.big;
  p.Ya = p.tau + tau_e * 8;
  p.Yb = p.Ya + y_e * 8;
  p.Z = p.Yb + y_e * 8;
  p.Kt = add((size_t)(R * o * o) * 8);
  p.HT = add((size_t)(R * o * o) * 8);
  p.partial_elems = (size_t)std::max({64 * R * v, 16 * R * o * o, 4 * R * R, (int64_t)1 << 16});
  p.partial = add(p.partial_elems * 8);
  p.rowbuf = add((size_t)std::max<int64_t>(2 * R, 4096) * 8);
  p.sums = add(2 * 1024 * 8);
  p.scal = add(S_COUNT * 8);
  p.status = add(16 * 4);  // directly after scal (S_COUNT * 8 is a multiple of ALIGN): one copy reads both
  static_assert((S_COUNT * 8) % ALIGN == 0, "status must follow the scalar block");
  p.tdc = 0;
  p.total = off;
  return p;
}

void validate_dims(const cpppl_dims* d) {
  if (!d) throw std::invalid_argument("dims is NULL");
  if (d->o <= 0 || d->v <= 0 || d->nx <= 0 || d->rank <= 0)
    throw std::invalid_argument("all dims must be positive");
  if (d->rank > MAX_RANK) throw std::invalid_argument("rank exceeds 4096");
  if (d->o > 4096 || d->v > 65536 || d->nx > (1 << 20)) throw std::invalid_argument("dims too large");
}

void need_ws(cpppl_ctx* c) {
  if (!c->ws) throw StatusError(CPPPL_E_STATE, "no workspace bound (cpppl_bind_workspace)");
}

// ------------------------------------------------------------------ timing
hipEvent_t next_event(cpppl_ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    CPPPL_HIP(hipEventCreate(&e));
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}
struct Span {
  cpppl_ctx* c;
  int cls;
  hipStream_t st;
  hipEvent_t a = nullptr;
  cpppl_ctx::SpanState state{0, false};
  cpppl_ctx::SpanState* outer = nullptr;
  Span(cpppl_ctx* c_, int cls_, hipStream_t s_ = nullptr) : c(c_), cls(cls_), st(s_ ? s_ : c_->stream) {
    if (c->timing) {
      a = next_event(c);
      CPPPL_HIP(hipEventRecord(a, st));
      state.cls = cls;
      outer = c->span;
      c->span = &state;
    }
  }
  ~Span() noexcept(false) {
    if (c->timing && a) {
      c->span = outer;
      if (state.has_sub) return;  // the launches of a cut product were timed one by one
      hipEvent_t b = next_event(c);
      CPPPL_HIP(hipEventRecord(b, st));
      c->segs.push_back({cls, a, b, 1});
    }
  }
};

// Times one launch of a product cut into several (inside a class span), so
// that side-stream work dispatched between the launches is not counted.
struct LaunchSpan {
  cpppl_ctx* c;
  hipEvent_t a = nullptr;
  int calls;
  LaunchSpan(cpppl_ctx* c_, bool first) : c(c_), calls(first ? 1 : 0) {
    if (c->timing && c->span) {
      a = next_event(c);
      CPPPL_HIP(hipEventRecord(a, c->stream));
    }
  }
  ~LaunchSpan() noexcept(false) {
    if (a) {
      hipEvent_t b = next_event(c);
      CPPPL_HIP(hipEventRecord(b, c->stream));
      c->segs.push_back({c->span->cls, a, b, calls});
      c->span->has_sub = true;
    }
  }
};

// ------------------------------------------------------------------ paths
Path path_for(cpppl_ctx* c, DType dt) {
  const Plan& p = c->plan;
  Path P;
  P.dt = dt;
  if (dt == DType::F64) {
    P.esz = 8;
    P.T2 = c->at(p.t64);
    P.T2T = c->at(p.t64T);
    P.BnT = c->at(p.b64T);
    P.Bp = c->at(p.b64P);
    P.BnT_b = c->singles_on ? c->at(p.bb64T) : P.BnT;
    P.Bp_b = c->singles_on ? c->at(p.bb64P) : P.Bp;
    for (int m = 0; m < 4; ++m) P.FTop[m] = c->at(p.FT[m]);
  } else if (c->prec == CPPPL_BF16) {
    P.esz = 2;
    P.T2 = c->at(p.t16);
    P.T2T = c->at(p.t16T);
    P.BnT = c->at(p.b16T);
    P.Bp = c->at(p.b16P);
    P.BnT_b = c->singles_on ? c->at(p.bb16T) : P.BnT;
    P.Bp_b = c->singles_on ? c->at(p.bb16P) : P.Bp;
    for (int m = 0; m < 4; ++m) P.FTop[m] = c->at(p.F16T[m]);
  } else if (c->prec == CPPPL_FP8_E4M3) {
    // e4m3 t and B (scaled per ij row and per X slice), bfloat16 everything else
    P.esz = 2;
    P.fp8 = true;
    P.T2 = c->at(p.t8);
    P.T2T = c->at(p.t8T);
    P.BnT = c->at(p.b8T);
    P.Bp = c->at(p.b8P);
    P.sT = c->at<float>(p.sT);
    P.sBx = c->at<float>(p.sBx);
    P.BnT_b = c->singles_on ? c->at(p.bb8T) : P.BnT;
    P.Bp_b = c->singles_on ? c->at(p.bb8P) : P.Bp;
    P.sBx_b = c->singles_on ? c->at<float>(p.sBbx) : P.sBx;
    for (int m = 0; m < 4; ++m) P.FTop[m] = c->at(p.F16T[m]);
  } else {
    throw StatusError(CPPPL_E_UNSUPPORTED, "the low-precision path needs a BF16 or FP8 context");
  }
  return P;
}

// Inverse steps queued on the side stream are dispatched only between
// main-stream launches (a grid with work-groups still to place keeps the CUs),
// so while a side inverse is pending an unsplit BF16 product is cut into
// c->launch_chunks launches along its batch, else along N in whole tiles.
// Measured at o=32, v=256, X=768, R=1024: four launches per product raise the
// sweep rate by 4 %, because the inverse then waits less at its join.
void run_gemm(cpppl_ctx* c, const Path& P, const Gemm& g, int max_chunks = 4) {
  hipStream_t s = c->stream;
  const int k = std::min(c->launch_chunks, max_chunks);
  if (P.dt == DType::F64) {
    gemm_f64(g, s);
    return;
  }
  if (k <= 1 || g.splits > 1) {
    gemm_bf16(g, s);
    return;
  }
  const int64_t ea = 2, eb = g.b_fp8 ? 1 : 2;
  const int64_t ec = g.ctype == DType::BF16 ? 2 : (g.ctype == DType::F32 ? 4 : 8);
  if (g.batch >= k && !g.b_fp8) {
    const int64_t per = (g.batch + k - 1) / k;
    for (int64_t b0 = 0; b0 < g.batch; b0 += per) {
      Gemm h = g;
      h.batch = std::min(per, g.batch - b0);
      h.A = (const char*)g.A + b0 * g.sab * ea;
      h.B = (const char*)g.B + b0 * g.sbb * eb;
      h.C = (char*)g.C + b0 * g.scb * ec;
      LaunchSpan ls(c, b0 == 0);
      gemm_bf16(h, s);
    }
  } else if (g.batch == 1 && g.N >= 128 * k) {
    const int64_t per = ((g.N + k - 1) / k + 127) / 128 * 128;
    for (int64_t n0 = 0; n0 < g.N; n0 += per) {
      Gemm h = g;
      h.N = std::min(per, g.N - n0);
      h.B = (const char*)g.B + n0 * g.sbn * eb;
      h.C = (char*)g.C + n0 * ec;
      if (g.b_fp8 && g.bscale_mode == 1) h.bscale = g.bscale + n0;
      LaunchSpan ls(c, n0 == 0);
      gemm_bf16(h, s);
    }
  } else {
    gemm_bf16(g, s);
  }
}

int splits_for(cpppl_ctx* c, const Path& P, int64_t M, int64_t N, int64_t K, int64_t batch) {
  const int64_t tiles = (P.dt == DType::F64 ? gemm_tiles_f64(M, N) : gemm_tiles_bf16(M, N)) * batch;
  const int64_t bk = P.dt == DType::F64 ? 16 : 64;
  int s = choose_splits(tiles, K, 1024, 4 * bk, 256);
  const int64_t cap = (int64_t)(c->plan.partial_elems / (size_t)std::max<int64_t>(1, M * N * batch));
  if (s > cap) s = (int)std::max<int64_t>(1, cap);
  return s;
}

// ------------------------------------------------------------------ chain steps
// Launches per Y and Z product while a side inverse is pending.  Both go to
// the B-resident kernel, whose work-groups load a v x 256 block of B each, so
// fewer, larger launches pay: measured at o = 32, v = 256, X = 768, R = 1024
// alternating on one box, 391 sweeps/s with Y whole and Z in two launches,
// 390 with Z whole, 385 with Z in four (Y in four: 6 % slower than whole).
constexpr int Y_LAUNCHES = 1, Z_LAUNCHES = 2;
// tau keeps four launches (one measured the same sweep rate).  G, 1024 batches
// of 256 x 256 from K = X, in two launches of two rounds of work-groups each:
// 396.5 sweeps/s on average against 394.1 with four one-round launches and
// 390.4 with one launch (three alternating runs each), G 230 against 265 us
// per call.
constexpr int TAU_LAUNCHES = 4, G_LAUNCHES = 2;

// tau[r][cd] = sum_ij Kt[r][ij] t[ij][cd], Kt = KR(gamma, rho)   (path dtype)
void compute_tau(cpppl_ctx* c, const Path& P) {
  Span sp(c, CPPPL_T_KR_T2);
  const int64_t o = c->d.o, v = c->d.v, R = c->d.rank;
  // e4m3 t: its per-ij scale runs along k here and is folded into Kt
  khatri_rao_t(c->at<double>(c->plan.FT[0]), c->at<double>(c->plan.FT[1]), o, R, c->at(c->plan.Kt),
               P.dt, c->stream, P.fp8 ? P.sT : nullptr);
  Gemm g;
  g.M = R; g.N = v * v; g.K = o * o;
  g.A = c->at(c->plan.Kt); g.sam = o * o; g.sak = 1;
  g.B = P.T2T; g.sbn = o * o; g.sbk = 1; g.b_fp8 = P.fp8;
  g.C = c->at(c->plan.tau); g.scm = v * v; g.ctype = P.dt;
  run_gemm(c, P, g, TAU_LAUNCHES);
}


// Y[r][X][q] = sum_p F[r][p] B^X_pq for F = factor `mode` (2 alpha with B,
// 3 beta with the b-side operand: Dbar with singles, eq. dfB)
void compute_Y(cpppl_ctx* c, const Path& P, int mode, size_t out) {
  Span sp(c, CPPPL_T_Y);
  const int64_t v = c->d.v, X = c->d.nx, R = c->d.rank;
  const bool bside = mode == 3;
  Gemm g;
  g.M = R; g.N = X * v; g.K = v;
  g.A = P.FTop[mode]; g.sam = v; g.sak = 1;
  g.B = bside ? P.BnT_b : P.BnT; g.sbn = v; g.sbk = 1;
  g.b_fp8 = P.fp8; g.bscale = bside ? P.sBx_b : P.sBx; g.bscale_mode = 1;  // n = (X, q)
  g.C = c->at(out); g.scm = X * v; g.ctype = P.dt;
  run_gemm(c, P, g, Y_LAUNCHES);
}

// Z for mode a (contract d with tau[r][c][d]) or b (contract c).
void compute_Z(cpppl_ctx* c, const Path& P, int mode) {
  Span sp(c, CPPPL_T_Z);
  const int64_t v = c->d.v, X = c->d.nx, R = c->d.rank;
  Gemm g;
  g.batch = R; g.M = X; g.N = v; g.K = v;
  g.A = c->at(mode == 2 ? c->plan.Yb : c->plan.Ya); g.sam = v; g.sak = 1; g.sab = X * v;
  g.B = c->at(c->plan.tau); g.sbb = v * v;
  if (mode == 2) { g.sbn = v; g.sbk = 1; } else { g.sbk = v; g.sbn = 1; }
  g.C = c->at(c->plan.Z); g.scm = v; g.scb = X * v; g.ctype = P.dt;
  run_gemm(c, P, g, Z_LAUNCHES);
}

// M^T[r][p] = sum_{X,q} Z[r][X][q] B^X_pq  -> MT (FP64); mode 3 (beta)
// contracts the b-side operand (Dbar with singles)
void compute_M(cpppl_ctx* c, const Path& P, int mode) {
  Span sp(c, CPPPL_T_M);
  const int64_t v = c->d.v, X = c->d.nx, R = c->d.rank;
  const bool bside = mode == 3;
  Gemm g;
  g.M = R; g.N = v; g.K = X * v;
  g.A = c->at(c->plan.Z); g.sam = X * v; g.sak = 1;
  g.B = bside ? P.Bp_b : P.Bp; g.sbn = X * v; g.sbk = 1;
  g.b_fp8 = P.fp8; g.bscale = bside ? P.sBx_b : P.sBx; g.bscale_mode = 2;  // k = (X, q), v % 8 == 0
  g.C = c->at(c->plan.MT); g.scm = v; g.ctype = DType::F64;
  g.splits = splits_for(c, P, g.M, g.N, g.K, 1);
  g.partial = c->at(c->plan.partial);
  run_gemm(c, P, g);
}

// G[r][c][d] = sum_X Ya[r][X][c] Yb[r][X][d]   (stored in the Z buffer)
void compute_G(cpppl_ctx* c, const Path& P) {
  Span sp(c, CPPPL_T_G);
  const int64_t v = c->d.v, X = c->d.nx, R = c->d.rank;
  Gemm g;
  g.batch = R; g.M = v; g.N = v; g.K = X;
  g.A = c->at(c->plan.Ya); g.sam = 1; g.sak = v; g.sab = X * v;
  g.B = c->at(c->plan.Yb); g.sbk = v; g.sbn = 1; g.sbb = X * v;
  g.C = c->at(c->plan.Z); g.scm = v; g.scb = v * v; g.ctype = P.dt;
  run_gemm(c, P, g, G_LAUNCHES);
}

// H^T[r][ij] = sum_cd G[r][cd] t[ij][cd]  -> HT (FP64)
void compute_H(cpppl_ctx* c, const Path& P) {
  Span sp(c, CPPPL_T_H);
  const int64_t o = c->d.o, v = c->d.v, R = c->d.rank;
  Gemm g;
  g.M = R; g.N = o * o; g.K = v * v;
  g.A = c->at(c->plan.Z); g.sam = v * v; g.sak = 1;
  g.B = P.T2; g.sbn = v * v; g.sbk = 1;
  g.b_fp8 = P.fp8; g.bscale = P.sT; g.bscale_mode = 1;  // n = ij
  g.C = c->at(c->plan.HT); g.scm = o * o; g.ctype = DType::F64;
  g.splits = splits_for(c, P, g.M, g.N, g.K, 1);
  g.partial = c->at(c->plan.partial);
  run_gemm(c, P, g);
}

void compute_occ(cpppl_ctx* c, int mode, hipStream_t st = nullptr) {
  if (!st) st = c->stream;
  Span sp(c, CPPPL_T_SOLVE, st);
  const int64_t o = c->d.o, R = c->d.rank;
  const double* other = c->at<double>(c->plan.FT[mode == 0 ? 1 : 0]);
  occ_reduce(c->at<double>(c->plan.HT), other, c->at<double>(c->plan.MT), o, R, mode == 0 ? 0 : 1,
             st);
}

// MTTKRP of a planted CP tensor via cross Grams.
void planted_mttkrp(cpppl_ctx* c, int mode) {
  Span sp(c, CPPPL_T_M);
  const int64_t R = c->d.rank, P = c->rank_p;
  const Plan& p = c->plan;
  int ks[3], nk = 0;
  for (int k = 0; k < 4; ++k)
    if (k != mode) ks[nk++] = k;
  for (int q = 0; q < 3; ++q) {
    const int k = ks[q];
    const int64_t n = nmode(c->d, k);
    Gemm g;
    g.M = R; g.N = P; g.K = n;
    g.A = c->at(p.FT[k]); g.sam = n; g.sak = 1;
    g.B = c->at(p.FpT[k]); g.sbn = n; g.sbk = 1;
    g.C = c->at(p.cross[q]); g.scm = P; g.ctype = DType::F64;
    gemm_f64(g, c->stream);
  }
  hadamard_scale_cols(c->at<double>(p.cross[0]), c->at<double>(p.cross[1]),
                      c->at<double>(p.cross[2]), c->at<double>(p.lamp), c->at<double>(p.Cp), R, P,
                      c->stream);
  const int64_t n = nmode(c->d, mode);
  Gemm g;
  g.M = R; g.N = n; g.K = P;
  g.A = c->at(p.Cp); g.sam = P; g.sak = 1;
  g.B = c->at(p.FpT[mode]); g.sbk = n; g.sbn = 1;
  g.C = c->at(p.MT); g.scm = n; g.ctype = DType::F64;
  gemm_f64(g, c->stream);
}

// Gram_m = F_m^T F_m (R x R) from FT_m (R x n).
void compute_gram(cpppl_ctx* c, int m) {
  const int64_t n = nmode(c->d, m), R = c->d.rank;
  Gemm g;
  g.M = R; g.N = R; g.K = n;
  g.A = c->at(c->plan.FT[m]); g.sam = n; g.sak = 1;
  g.B = c->at(c->plan.FT[m]); g.sbn = n; g.sbk = 1;
  g.C = c->at(c->plan.gram[m]); g.scm = R; g.ctype = DType::F64;
  gemm_f64(g, c->stream);
}

void refresh_lowp(cpppl_ctx* c, int m) {
  if (c->prec == CPPPL_FP64) return;
  const int64_t n = nmode(c->d, m), R = c->d.rank;
  convert(c->at<double>(c->plan.FT[m]), c->at(c->plan.F16T[m]), DType::BF16, n * R, c->stream);
}

void copy_d2d(cpppl_ctx* c, size_t dst, size_t src, size_t bytes) {
  CPPPL_HIP(hipMemcpyAsync(c->at(dst), c->at(src), bytes, hipMemcpyDeviceToDevice, c->stream));
}

void sync(cpppl_ctx* c) {
  CPPPL_HIP(hipStreamSynchronize(c->stream));
  CPPPL_HIP(hipStreamSynchronize(c->side));
}

int read_status(cpppl_ctx* c) {
  CPPPL_HIP(hipMemcpyAsync(c->host_status, c->at(c->plan.status), 16 * sizeof(int),
                           hipMemcpyDeviceToHost, c->stream));
  sync(c);
  return c->host_status[0];
}

// Waits for an inverse forked ahead for the next sweep, before the inverse
// buffers are used for anything else.
void drop_early_fork(cpppl_ctx* c) {
  if (!c->alpha_forked) return;
  CPPPL_HIP(hipStreamSynchronize(c->side));
  c->alpha_forked = false;
}

// -W_m^{-1}, W_m = *_{k != m} Gram_k, on stream `st` into c->inv; a failed
// pivot sets status word `word`.  careful: synchronise and retry with a ridge
// shift while a pivot fails.  Returns retries.
int prepare_inverse(cpppl_ctx* c, int m, hipStream_t st, bool careful, int word = 0) {
  drop_early_fork(c);
  Span sp(c, CPPPL_T_INV, st);
  const int64_t R = c->d.rank;
  const Plan& p = c->plan;
  const double* G[3];
  int q = 0;
  for (int k = 0; k < 4; ++k)
    if (k != m) G[q++] = c->at<double>(p.gram[k]);
  int retries = 0;
  for (int attempt = 0; attempt < 6; ++attempt) {
    hadamard(G[0], G[1], G[2], c->at<double>(p.invA), R * R, st);
    if (attempt > 0) add_ridge(c->at<double>(p.invA), R, 1e-14 * std::pow(100.0, attempt - 1), st);
    if (careful) zero_ints(c->at<int>(p.status), 1, st);
    c->inv = spd_inverse_neg(c->at<double>(p.invA), c->at<double>(p.invB), c->at<double>(p.invD), R,
                             c->at<int>(p.status) + word, st);
    if (!careful) break;
    CPPPL_HIP(hipStreamSynchronize(st));
    if (read_status(c) == 0) break;
    retries = attempt + 1;
    if (attempt == 5) throw StatusError(CPPPL_E_NOT_SPD, "W is not positive definite after 5 ridge retries");
  }
  return retries;
}

// F_m^T = W^{-1} M^T (one GEMM), normalise the rows into lambda, refresh Gram_m.
void apply_inverse(cpppl_ctx* c, int m) {
  Span sp(c, CPPPL_T_SOLVE);
  const int64_t n = nmode(c->d, m), R = c->d.rank;
  const Plan& p = c->plan;
  Gemm g;
  g.M = R; g.N = n; g.K = R;
  g.A = c->inv; g.sam = R; g.sak = 1;
  g.B = c->at(p.MT); g.sbk = n; g.sbn = 1;
  g.C = c->at(p.FT[m]); g.scm = n; g.ctype = DType::F64; g.alpha = -1.0;
  // few output tiles (R x n): split K so that the launch fills the chip
  int s = choose_splits(gemm_tiles_f64(R, n), R, 256, 64, 16);
  const int64_t cap = (int64_t)(p.partial_elems / (size_t)(R * n));
  g.splits = (int)std::max<int64_t>(1, std::min<int64_t>(s, cap));
  g.partial = c->at(p.partial);
  g.keep_partials = true;  // summed below, unless K was not split
  const int used = gemm_f64(g, c->stream);
  if (used > 1) {
    // the split sum, the normalisation and the BF16 copy in one launch
    finish_factor(c->at<double>(p.partial), used, R, n, g.alpha, c->at<double>(p.FT[m]),
                  c->at<double>(p.lam), c->prec != CPPPL_FP64 ? c->at(p.F16T[m]) : nullptr,
                  c->stream);
  } else {
    row_normalize(c->at<double>(p.FT[m]), R, n, c->at<double>(p.lam), c->stream);
    refresh_lowp(c, m);
  }
  compute_gram(c, m);
}

int solve_mode(cpppl_ctx* c, int m, bool careful) {
  const int r = prepare_inverse(c, m, c->stream, careful);
  apply_inverse(c, m);
  return r;
}

// Marks the point of the main stream after which the Grams W_m needs are ready.
void mark_fork(cpppl_ctx* c) { CPPPL_HIP(hipEventRecord(c->ev_main, c->stream)); }

__global__ void set_flag_kernel(int* flag) { *flag = 1; }

// Start -W_m^{-1} on the side stream from the point marked by mark_fork.
// fault: the test hook's injected failure, a flag raised after the inverse
// (before the join event, so the sweep's status readback sees it).
void fork_inverse(cpppl_ctx* c, int m, int word = 0, bool fault = false) {
  CPPPL_HIP(hipStreamWaitEvent(c->side, c->ev_main, 0));
  prepare_inverse(c, m, c->side, false, word);
  if (fault) {
    hipLaunchKernelGGL(set_flag_kernel, dim3(1), dim3(1), 0, c->side, c->at<int>(c->plan.status) + word);
    CPPPL_LAUNCH_CHECK("set_flag");
  }
  CPPPL_HIP(hipEventRecord(c->ev_side, c->side));
}
void join_inverse(cpppl_ctx* c) { CPPPL_HIP(hipStreamWaitEvent(c->stream, c->ev_side, 0)); }

// The MTTKRP of `mode` at the current factors into MT (R x n).
void mttkrp_into_MT(cpppl_ctx* c, const Path& P, int mode) {
  if (c->planted) {
    planted_mttkrp(c, mode);
    return;
  }
  if (mode >= 2) {
    compute_tau(c, P);
    if (mode == 2) compute_Y(c, P, 3, c->plan.Yb);
    else compute_Y(c, P, 2, c->plan.Ya);
    compute_Z(c, P, mode);
    compute_M(c, P, mode);
  } else {
    compute_Y(c, P, 2, c->plan.Ya);
    compute_Y(c, P, 3, c->plan.Yb);
    compute_G(c, P);
    compute_H(c, P);
    compute_occ(c, mode);
  }
  c->ybeta_valid = c->tau_valid = false;
}

// eta terms: nn = cp2 (this sweep), np = lam^T (* F_k^T Fprev_k) lamprev, pp = previous cp2.
void compute_eta(cpppl_ctx* c) {
  Span sp(c, CPPPL_T_FIT);
  const int64_t R = c->d.rank;
  const Plan& p = c->plan;
  const double* X[4];
  for (int m = 0; m < 4; ++m) {
    const int64_t n = nmode(c->d, m);
    Gemm g;
    g.M = R; g.N = R; g.K = n;
    g.A = c->at(p.FT[m]); g.sam = n; g.sak = 1;
    g.B = c->at(p.FTprev[c->snap][m]); g.sbn = n; g.sbk = 1;
    g.C = c->at(p.cross[m]); g.scm = R; g.ctype = DType::F64;
    gemm_f64(g, c->stream);
    X[m] = c->at<double>(p.cross[m]);
  }
  double* sc = c->at<double>(p.scal);
  weighted_hadamard_sum(X, c->at<double>(p.lam), c->at<double>(p.lamprev[c->snap]), R,
                        c->at<double>(p.rowbuf), sc + S_ETA + 1, c->stream);
  // sc[S_ETA] = nn = cp2 of this sweep, sc[S_ETA+2] = pp = cp2 of the previous state
  CPPPL_HIP(hipMemcpyAsync(sc + S_ETA, sc + S_FIT + 1, 8, hipMemcpyDeviceToDevice, c->stream));
  CPPPL_HIP(hipMemcpyAsync(sc + S_ETA + 2, sc + S_CP2_PREV, 8, hipMemcpyDeviceToDevice, c->stream));
  finish_eta(sc + S_ETA, c->stream);
  CPPPL_HIP(hipMemcpyAsync(sc + S_CP2_PREV, sc + S_FIT + 1, 8, hipMemcpyDeviceToDevice, c->stream));
}

// The factors (FT[0..3], lambda) as one contiguous set at `base`.
void copy_factor_set(cpppl_ctx* c, size_t base, bool to_set) {
  const Plan& p = c->plan;
  const int64_t R = c->d.rank;
  const double* src[5];
  double* dst[5];
  int64_t n[5];
  size_t off = base;
  for (int m = 0; m < 5; ++m) {
    const int64_t e = m < 4 ? nmode(c->d, m) * R : R;
    double* live = c->at<double>(m < 4 ? p.FT[m] : p.lam);
    double* set = c->at<double>(off);
    src[m] = to_set ? live : set;
    dst[m] = to_set ? set : live;
    n[m] = e;
    off += (size_t)e * 8;
  }
  copy_doubles(src, dst, n, 5, c->stream);
}
size_t factor_set_bytes(const cpppl_ctx* c) {
  return (size_t)((2 * c->d.o + 2 * c->d.v) * c->d.rank + c->d.rank) * 8;
}

// Factors and weights into snapshot slot `slot`, which becomes the eta
// reference of the next sweep.
void snapshot(cpppl_ctx* c, int slot) {
  const Plan& p = c->plan;
  c->snap = slot;
  const int64_t R = c->d.rank;
  const double* src[5];
  double* dst[5];
  int64_t n[5];
  for (int m = 0; m < 4; ++m) {
    src[m] = c->at<double>(p.FT[m]);
    dst[m] = c->at<double>(p.FTprev[slot][m]);
    n[m] = nmode(c->d, m) * R;
  }
  src[4] = c->at<double>(p.lam);
  dst[4] = c->at<double>(p.lamprev[slot]);
  n[4] = R;
  copy_doubles(src, dst, n, 5, c->stream);
}

void restore_snapshot(cpppl_ctx* c, int slot) {
  const Plan& p = c->plan;
  c->snap = slot;
  const int64_t R = c->d.rank;
  for (int m = 0; m < 4; ++m) {
    copy_d2d(c, p.FT[m], p.FTprev[slot][m], (size_t)(nmode(c->d, m) * R) * 8);
    compute_gram(c, m);
    refresh_lowp(c, m);
  }
  copy_d2d(c, p.lam, p.lamprev[slot], (size_t)R * 8);
  c->ybeta_valid = c->tau_valid = false;
}

// cp2 of the current factors into sc[S_CP2_PREV] (eta reference for the first sweep).
void cp2_current(cpppl_ctx* c, double* out) {
  const double* G[4];
  for (int m = 0; m < 4; ++m) G[m] = c->at<double>(c->plan.gram[m]);
  weighted_hadamard_sum(G, c->at<double>(c->plan.lam), c->at<double>(c->plan.lam), c->d.rank,
                        c->at<double>(c->plan.rowbuf), out, c->stream);
}

// One ALS sweep on path P; returns ridge retries.  Outside careful mode the
// inverse of W for alpha, beta and gamma runs on the side stream while the
// main stream evaluates that factor's MTTKRP.  early_word >= 0: once rho is
// updated, W_alpha of the next sweep is final, and its inverse is forked on
// the side stream at once (a failed pivot sets status word early_word), to
// run beside this sweep's fit and the next sweep's first products.
int sweep(cpppl_ctx* c, const Path& P, bool careful, int early_word = -1) {
  const Plan& p = c->plan;
  int retries = 0;
  // tau of this sweep's gamma and rho, left by the previous sweep's energy
  bool have_tau = c->tau_valid && c->tau_dt == P.dt;
  c->tau_valid = false;
  if (c->planted || careful) {
    drop_early_fork(c);
    have_tau = have_tau && !c->planted;
    if (c->planted) {
      for (int m : {2, 3, 0, 1}) {
        planted_mttkrp(c, m);
        retries += solve_mode(c, m, careful);
      }
    } else {
      if (!have_tau) compute_tau(c, P);
      if (!c->ybeta_valid || c->ybeta_dt != P.dt) compute_Y(c, P, 3, p.Yb);
      compute_Z(c, P, 2);
      compute_M(c, P, 2);
      retries += solve_mode(c, 2, true);
      compute_Y(c, P, 2, p.Ya);
      compute_Z(c, P, 3);
      compute_M(c, P, 3);
      retries += solve_mode(c, 3, true);
      compute_Y(c, P, 3, p.Yb);
      compute_G(c, P);
      compute_H(c, P);
      compute_occ(c, 0);
      retries += solve_mode(c, 0, true);
      compute_occ(c, 1);
      retries += solve_mode(c, 1, true);
      c->ybeta_valid = true;
      c->ybeta_dt = P.dt;
    }
  } else {
    // The inverse may start with the mode's first main-stream kernel (the
    // fork mark), but its ~20 launches are issued by the host only after the
    // mode's first two main-stream kernels are queued, so the main queue does
    // not wait on the host issuing them.
    struct Chunked {
      cpppl_ctx* c;
      explicit Chunked(cpppl_ctx* x) : c(x) { c->launch_chunks = 4; }
      ~Chunked() { c->launch_chunks = 1; }
    } chunked(c);
    const bool pre = c->alpha_forked;  // W_alpha^{-1} already queued by the previous sweep
    c->alpha_forked = false;
    if (!pre) mark_fork(c);
    if (!have_tau) compute_tau(c, P);
    if (!c->ybeta_valid || c->ybeta_dt != P.dt) compute_Y(c, P, 3, p.Yb);
    compute_Z(c, P, 2);
    if (!pre) fork_inverse(c, 2);
    compute_M(c, P, 2);
    join_inverse(c);
    apply_inverse(c, 2);
    mark_fork(c);
    compute_Y(c, P, 2, p.Ya);
    compute_Z(c, P, 3);
    fork_inverse(c, 3);
    compute_M(c, P, 3);
    join_inverse(c);
    apply_inverse(c, 3);
    mark_fork(c);
    compute_Y(c, P, 3, p.Yb);
    c->ybeta_valid = true;
    c->ybeta_dt = P.dt;
    compute_G(c, P);
    fork_inverse(c, 0);
    compute_H(c, P);
    compute_occ(c, 0);
    join_inverse(c);
    apply_inverse(c, 0);
    // M_rho (H against the new gamma) on the side stream beside rho's inverse
    mark_fork(c);
    CPPPL_HIP(hipStreamWaitEvent(c->side, c->ev_main, 0));
    compute_occ(c, 1, c->side);
    CPPPL_HIP(hipEventRecord(c->ev_side, c->side));
    prepare_inverse(c, 1, c->stream, false);
    join_inverse(c);
    apply_inverse(c, 1);
    if (early_word >= 0) {
      zero_ints(c->at<int>(p.status) + early_word, 1, c->stream);
      mark_fork(c);
      fork_inverse(c, 2, early_word, c->inject_now);
      c->alpha_forked = true;
    }
  }
  {
    Span sp(c, CPPPL_T_FIT);
    const double* G[4];
    for (int m = 0; m < 4; ++m) G[m] = c->at<double>(p.gram[m]);
    fit_scalars(c->at<double>(p.MT), c->at<double>(p.FT[1]), c->d.o, c->at<double>(p.lam), G,
                c->d.rank, c->at<double>(p.scal) + S_NORM_R2, c->at<double>(p.rowbuf),
                c->at<double>(p.scal) + S_FIT, c->stream);
  }
  if (c->want_energy && !c->planted) {
    // E_CP at the updated factors: tau' = KR(gamma', rho')^T t is exactly the
    // tau the next sweep starts from, so it is kept for it (no extra product)
    compute_tau(c, P);
    Span sp(c, CPPPL_T_FIT);
    energy_from_tau(c->at(p.tau), P.dt, c->at<double>(p.FT[2]), c->at<double>(p.FT[3]),
                    c->at<double>(p.lam), c->d.rank, c->d.v, c->at<double>(p.rowbuf),
                    c->at<double>(p.scal) + S_ENERGY, c->stream);
    c->tau_valid = true;
    c->tau_dt = P.dt;
  }
  if (c->want_eta) {
    compute_eta(c);
  } else {  // keep ||CP||^2 as the reference of a later eta
    double* sc = c->at<double>(p.scal);
    CPPPL_HIP(hipMemcpyAsync(sc + S_CP2_PREV, sc + S_FIT + 1, 8, hipMemcpyDeviceToDevice, c->stream));
  }
  return retries;
}

// ||R||^2 and sum R t, FP64, streaming R in a-blocks through the intermediate region.
void compute_norm_r2(cpppl_ctx* c) {
  const Plan& p = c->plan;
  double* sc = c->at<double>(p.scal);
  if (c->planted) {
    const int64_t P = c->rank_p;
    const double* G[4];
    for (int m = 0; m < 4; ++m) {
      const int64_t n = nmode(c->d, m);
      Gemm g;
      g.M = P; g.N = P; g.K = n;
      g.A = c->at(p.FpT[m]); g.sam = n; g.sak = 1;
      g.B = c->at(p.FpT[m]); g.sbn = n; g.sbk = 1;
      g.C = c->at(p.cross[m]); g.scm = P; g.ctype = DType::F64;
      gemm_f64(g, c->stream);
      G[m] = c->at<double>(p.cross[m]);
    }
    weighted_hadamard_sum(G, c->at<double>(p.lamp), c->at<double>(p.lamp), P,
                          c->at<double>(p.rowbuf), sc + S_NORM_R2, c->stream);
    set_scalar(sc + S_E_EXACT, std::numeric_limits<double>::quiet_NaN(), c->stream);
    c->norm_valid = true;
    return;
  }
  const int64_t o = c->d.o, v = c->d.v, X = c->d.nx;
  const int64_t o2 = o * o, v2 = v * v;
  double* region = c->at<double>(p.big);
  const int64_t cap = (int64_t)(p.big_bytes / 8);
  double* tdc = region;                         // t[ij][d][c]
  transpose_batched(c->at<double>(p.t64), tdc, DType::F64, o2, v, v, c->stream);
  int64_t ab = (cap - o2 * v2 - 64) / (v * v2 + o2 * v);
  ab = std::max<int64_t>(1, std::min<int64_t>(ab, v));
  double* gblk = tdc + o2 * v2;                 // [a][b][d][c] for a in the block
  double* rblk = gblk + ab * v * v2;            // [ij][a][b]
  zero_doubles(sc + S_NORM_R2, 2, c->stream);
  for (int64_t a0 = 0; a0 < v; a0 += ab) {
    const int64_t nb = std::min(ab, v - a0);
    Gemm g1;  // g_a[(b,d)][c] = sum_X Dbar[X][(b,d)] B[X][a][c]   (Dbar = B without singles)
    g1.batch = nb; g1.M = v2; g1.N = v; g1.K = X;
    g1.A = c->at(c->singles_on ? p.bb64 : p.b64); g1.sam = 1; g1.sak = v2; g1.sab = 0;
    g1.B = c->at<double>(p.b64) + a0 * v; g1.sbk = v2; g1.sbn = 1; g1.sbb = v;
    g1.C = gblk; g1.scm = v; g1.scb = v * v2; g1.ctype = DType::F64;
    gemm_f64(g1, c->stream);
    Gemm g2;  // R[ij][(a,b)] = sum_(d,c) t[ij][d][c] g[(a,b)][(d,c)]
    g2.M = o2; g2.N = nb * v; g2.K = v2;
    g2.A = tdc; g2.sam = v2; g2.sak = 1;
    g2.B = gblk; g2.sbn = v2; g2.sbk = 1;
    g2.C = rblk; g2.scm = nb * v; g2.ctype = DType::F64;
    gemm_f64(g2, c->stream);
    sumsq_dot_accumulate(rblk, c->at<double>(p.t64) + a0 * v, o2, nb * v, nb * v, v2,
                         c->at<double>(p.sums), sc + S_NORM_R2, c->stream);
  }
  c->norm_valid = true;
  c->ybeta_valid = c->tau_valid = false;  // the region holding Y_beta was overwritten
}

void ensure_norm(cpppl_ctx* c) {
  if (!c->norm_valid) compute_norm_r2(c);
}

void compute_energy(cpppl_ctx* c, double* out) {
  Span sp(c, CPPPL_T_FIT);
  if (c->planted) {
    set_scalar(out, std::numeric_limits<double>::quiet_NaN(), c->stream);
    return;
  }
  const Path P = path_for(c, DType::F64);
  compute_tau(c, P);
  energy_from_tau(c->at(c->plan.tau), DType::F64, c->at<double>(c->plan.FT[2]),
                  c->at<double>(c->plan.FT[3]), c->at<double>(c->plan.lam), c->d.rank, c->d.v,
                  c->at<double>(c->plan.rowbuf), out, c->stream);
  c->tau_valid = true;
  c->tau_dt = DType::F64;
}

void require_inputs(cpppl_ctx* c) {
  need_ws(c);
  if (!c->planted && !(c->have_t && c->have_b))
    throw StatusError(CPPPL_E_STATE, "load t2 and the DF tensor (or a planted tensor) first");
  if (!c->have_factors) throw StatusError(CPPPL_E_STATE, "set the factors first");
}

void load_device_or_host(cpppl_ctx* c, void* dst, const void* src, size_t bytes, int on_device) {
  CPPPL_HIP(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           c->stream));
  if (!on_device) sync(c);
}

void check_finite_input(cpppl_ctx* c, const double* x, int64_t n, const char* what) {
  zero_ints(c->at<int>(c->plan.status) + 1, 1, c->stream);
  nonfinite_check(x, n, c->at<int>(c->plan.status) + 1, c->stream);
  CPPPL_HIP(hipMemcpyAsync(c->host_status, c->at(c->plan.status), 16 * sizeof(int),
                           hipMemcpyDeviceToHost, c->stream));
  sync(c);
  if (c->host_status[1]) throw StatusError(CPPPL_E_NONFINITE, std::string("non-finite values in ") + what);
}

// Derive the operand layouts of t from the FP64 master.
void derive_t(cpppl_ctx* c) {
  const Plan& p = c->plan;
  const int64_t o2 = c->d.o * c->d.o, v2 = c->d.v * c->d.v;
  transpose_batched(c->at<double>(p.t64), c->at(p.t64T), DType::F64, 1, o2, v2, c->stream);
  if (c->prec == CPPPL_BF16) {
    convert(c->at<double>(p.t64), c->at(p.t16), DType::BF16, o2 * v2, c->stream);
    transpose_batched(c->at<double>(p.t64), c->at(p.t16T), DType::BF16, 1, o2, v2, c->stream);
  } else if (c->prec == CPPPL_FP8_E4M3) {
    float* sT = c->at<float>(p.sT);
    e4m3_row_scales(c->at<double>(p.t64), o2, v2, sT, c->stream);
    quantize_e4m3(c->at<double>(p.t64), c->at<uint8_t>(p.t8), o2 * v2, sT, v2, o2, 1, c->stream);
    quantize_e4m3(c->at<double>(p.t64T), c->at<uint8_t>(p.t8T), o2 * v2, sT, 1, o2, 1, c->stream);
  }
}

// Layouts of a DF-type operand (B, or Dbar with singles) from its FP64 master
// src[X][p][q]: B^X transposed per X and the (p, X, q) permutation, in FP64 and
// in the context's low precision (e4m3 with one power-of-two scale per X).
struct BLayouts {
  size_t f64T, f64P, bf16T, bf16P, e4T, e4P, scale, scale_x;
};
void derive_b(cpppl_ctx* c, size_t src, const BLayouts& L) {
  const int64_t v = c->d.v, X = c->d.nx, n = X * v * v;
  const double* b = c->at<double>(src);
  transpose_batched(b, c->at(L.f64T), DType::F64, X, v, v, c->stream);
  permute_pxq(b, c->at(L.f64P), DType::F64, X, v, c->stream);
  if (c->prec == CPPPL_BF16) {
    transpose_batched(b, c->at(L.bf16T), DType::BF16, X, v, v, c->stream);
    permute_pxq(b, c->at(L.bf16P), DType::BF16, X, v, c->stream);
  } else if (c->prec == CPPPL_FP8_E4M3) {
    float* sc = c->at<float>(L.scale);
    e4m3_row_scales(b, X, v * v, sc, c->stream);
    quantize_e4m3(c->at<double>(L.f64T), c->at<uint8_t>(L.e4T), n, sc, v * v, X, 1, c->stream);
    quantize_e4m3(c->at<double>(L.f64P), c->at<uint8_t>(L.e4P), n, sc, 1, X * v, v, c->stream);
    expand_scales(sc, c->at<float>(L.scale_x), X, v, c->stream);
  }
}

// t64 from the raw doubles: tau = t2 + t1 t1 with singles (eq. B), else t2.
void dress_t(cpppl_ctx* c) {
  const Plan& p = c->plan;
  const int64_t o = c->d.o, v = c->d.v;
  if (c->singles_on)
    dress_tau(c->at<double>(p.t2raw), c->at<double>(p.t1), c->at<double>(p.t64), o, v, c->stream);
  else
    CPPPL_HIP(hipMemcpyAsync(c->at(p.t64), c->at(p.t2raw), (size_t)(o * o * v * v) * 8,
                             hipMemcpyDeviceToDevice, c->stream));
  derive_t(c);
}

// Dbar^X_bd = D^X_bd - 2 sum_k D^X_bk t1[k][d] (the intermediate before eq. dfB)
// and its layouts.
void derive_dbar(cpppl_ctx* c) {
  const Plan& p = c->plan;
  const int64_t o = c->d.o, v = c->d.v, X = c->d.nx;
  CPPPL_HIP(hipMemcpyAsync(c->at(p.bb64), c->at(p.b64), (size_t)(X * v * v) * 8,
                           hipMemcpyDeviceToDevice, c->stream));
  Gemm g;  // per X: Dbar[b][d] += -2 sum_k bvo[b][k] t1[k][d]
  g.batch = X; g.M = v; g.N = v; g.K = o;
  g.A = c->at(p.bvo); g.sam = o; g.sak = 1; g.sab = v * o;
  g.B = c->at(p.t1); g.sbk = v; g.sbn = 1; g.sbb = 0;
  g.C = c->at(p.bb64); g.scm = v; g.scb = v * v; g.ctype = DType::F64;
  g.alpha = -2.0; g.beta = 1.0;
  gemm_f64(g, c->stream);
  derive_b(c, p.bb64, BLayouts{p.bb64T, p.bb64P, p.bb16T, p.bb16P, p.bb8T, p.bb8P, p.sBb, p.sBbx});
}

void init_after_factors(cpppl_ctx* c) {
  for (int m = 0; m < 4; ++m) {
    compute_gram(c, m);
    refresh_lowp(c, m);
  }
  cp2_current(c, c->at<double>(c->plan.scal) + S_CP2_PREV);
  c->have_factors = true;
  c->ybeta_valid = c->tau_valid = false;
}

}  // namespace

// ---- helpers shared with the warm-start code (ws.h) ----
void ws_mttkrp_into_MT(cpppl_ctx* c, DType dt, int mode) { mttkrp_into_MT(c, path_for(c, dt), mode); }
void ws_solve_no_update(cpppl_ctx* c, int mode, size_t out_off) {
  // out = MT W^{-1} with the current Grams (no normalisation, no state change)
  const int64_t n = nmode(c->d, mode), R = c->d.rank;
  prepare_inverse(c, mode, c->stream, false);
  Gemm g;
  g.M = R; g.N = n; g.K = R;
  g.A = c->inv; g.sam = R; g.sak = 1;
  g.B = c->at(c->plan.MT); g.sbk = n; g.sbn = 1;
  g.C = c->at(out_off); g.scm = n; g.ctype = DType::F64; g.alpha = -1.0;
  gemm_f64(g, c->stream);
}
void ws_init_after_factors(cpppl_ctx* c) { init_after_factors(c); }
void ws_mttkrp_dt(cpppl_ctx* c, int mode) {
  // the MTTKRP chain with dt in place of t (the PPL tensor is linear in t)
  // BF16 contexts use a bfloat16 copy of dt; FP64 and FP8 contexts the FP64 one
  const DType dt = c->prec == CPPPL_BF16 ? DType::BF16 : DType::F64;
  Path P = path_for(c, dt);
  if (dt == DType::F64) {
    P.T2 = c->at(c->plan.dt64);
    P.T2T = c->at(c->plan.dt64T);
  } else {
    P.T2 = c->at(c->plan.dt16);
    P.T2T = c->at(c->plan.dt16T);
  }
  mttkrp_into_MT(c, P, mode);
}
void ws_load_dt(cpppl_ctx* c, const double* dt, int on_device) {
  const Plan& p = c->plan;
  const int64_t o2 = c->d.o * c->d.o, v2 = c->d.v * c->d.v;
  load_device_or_host(c, c->at(p.dt64), dt, (size_t)(o2 * v2) * 8, on_device);
  check_finite_input(c, c->at<double>(p.dt64), o2 * v2, "dt");
  transpose_batched(c->at<double>(p.dt64), c->at(p.dt64T), DType::F64, 1, o2, v2, c->stream);
  if (c->prec == CPPPL_BF16) {
    convert(c->at<double>(p.dt64), c->at(p.dt16), DType::BF16, o2 * v2, c->stream);
    transpose_batched(c->at<double>(p.dt64), c->at(p.dt16T), DType::BF16, 1, o2, v2, c->stream);
  }
}
// L = ||CP||^2 - 2 <R, CP> at the current factors (FP64 MTTKRP of alpha).
double ws_judge_loss(cpppl_ctx* c) {
  const Plan& p = c->plan;
  mttkrp_into_MT(c, path_for(c, DType::F64), 2);
  const double* G[4];
  for (int m = 0; m < 4; ++m) G[m] = c->at<double>(p.gram[m]);
  fit_scalars(c->at<double>(p.MT), c->at<double>(p.FT[2]), c->d.v, c->at<double>(p.lam), G,
              c->d.rank, c->at<double>(p.scal) + S_NORM_R2, c->at<double>(p.rowbuf),
              c->at<double>(p.scal) + S_JUDGE, c->stream);
  CPPPL_HIP(hipMemcpyAsync(c->host_scal, c->at(p.scal), S_COUNT * 8, hipMemcpyDeviceToHost, c->stream));
  sync(c);
  return c->host_scal[S_JUDGE + 1] - 2.0 * c->host_scal[S_JUDGE];
}
void ws_add_dt(cpppl_ctx* c) {
  const Plan& p = c->plan;
  const int64_t n = c->d.o * c->d.o * c->d.v * c->d.v;
  axpy1(c->at<double>(p.dt64), c->at<double>(p.t64), n, c->stream);
  if (c->d.singles) axpy1(c->at<double>(p.dt64), c->at<double>(p.t2raw), n, c->stream);
}
void ws_derive_t(cpppl_ctx* c) {
  derive_t(c);
  c->norm_valid = false;
  c->ybeta_valid = c->tau_valid = false;
}
void ws_ensure_norm(cpppl_ctx* c) { ensure_norm(c); }
void ws_copy(cpppl_ctx* c, size_t dst, size_t src, size_t bytes) { copy_d2d(c, dst, src, bytes); }
bool ws_install_near_cache(cpppl_ctx* c) {
  if (!c->near_valid) return false;
  copy_factor_set(c, c->plan.nearCache, false);
  init_after_factors(c);
  return true;
}
void ws_sync(cpppl_ctx* c) { sync(c); }
const double* ws_t_doubles(cpppl_ctx* c) {
  return c->at<double>(c->singles_on ? c->plan.t2raw : c->plan.t64);
}
int64_t ws_nmode(const cpppl_dims& d, int m) { return nmode(d, m); }

}  // namespace cpppl

// =================================================================== C ABI
#define API_TRY(c)                                                            \
  if (!(c)) return CPPPL_E_ARG;                                               \
  if ((c)->hip_failed) {                                                      \
    (c)->err = "context unusable after a HIP error";                          \
    return CPPPL_E_HIP;                                                       \
  }                                                                           \
  try {                                                                       \
    CPPPL_HIP(hipSetDevice((c)->device));

#define API_CATCH(c)                                                          \
  }                                                                           \
  catch (const cpppl::StatusError& e) {                                       \
    (c)->err = e.msg;                                                         \
    return e.st;                                                              \
  }                                                                           \
  catch (const cpppl::HipError& e) {                                          \
    (c)->hip_failed = true;                                                   \
    (c)->err = std::string(e.where) + ": " + hipGetErrorString(e.err);        \
    return CPPPL_E_HIP;                                                       \
  }                                                                           \
  catch (const std::invalid_argument& e) {                                    \
    (c)->err = e.what();                                                      \
    return CPPPL_E_ARG;                                                       \
  }                                                                           \
  catch (const std::bad_alloc&) {                                             \
    (c)->err = "host allocation failed";                                      \
    return CPPPL_E_NOMEM;                                                     \
  }                                                                           \
  catch (const std::exception& e) {                                           \
    (c)->err = e.what();                                                      \
    return CPPPL_E_STATE;                                                     \
  }                                                                           \
  (c)->err.clear();                                                           \
  return CPPPL_OK;

extern "C" {

CPPPL_API cpppl_status cpppl_workspace_size(const cpppl_dims* dims, cpppl_precision prec,
                                            size_t* bytes) {
  if (!bytes) return CPPPL_E_ARG;
  try {
    validate_dims(dims);
    if (prec != CPPPL_FP64 && prec != CPPPL_BF16 && prec != CPPPL_FP8_E4M3) return CPPPL_E_ARG;
    if (prec == CPPPL_FP8_E4M3 && dims->v % 8 != 0) return CPPPL_E_ARG;
    *bytes = build_plan(*dims, prec).total;
  } catch (...) {
    return CPPPL_E_ARG;
  }
  return CPPPL_OK;
}

CPPPL_API cpppl_status cpppl_create(const cpppl_dims* dims, cpppl_precision prec, int device,
                                    void* hip_stream, cpppl_ctx** out) {
  if (!out) return CPPPL_E_ARG;
  *out = nullptr;
  try {
    validate_dims(dims);
  } catch (...) {
    return CPPPL_E_ARG;
  }
  if (prec != CPPPL_FP64 && prec != CPPPL_BF16 && prec != CPPPL_FP8_E4M3) return CPPPL_E_ARG;
  if (prec == CPPPL_FP8_E4M3 && dims->v % 8 != 0) return CPPPL_E_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CPPPL_E_HIP;
  cpppl_ctx* c = new (std::nothrow) cpppl_ctx();
  if (!c) return CPPPL_E_NOMEM;
  c->d = *dims;
  c->prec = prec;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->plan = build_plan(*dims, prec);
  if (hipSetDevice(device) != hipSuccess ||
      hipHostMalloc((void**)&c->host_scal, 2 * (S_COUNT * sizeof(double) + 16 * sizeof(int)),
                    hipHostMallocDefault) != hipSuccess ||
      hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_main, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_side, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_done[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_done[1], hipEventDisableTiming) != hipSuccess) {
    if (c->host_scal) (void)hipHostFree(c->host_scal);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->ev_main) (void)hipEventDestroy(c->ev_main);
    if (c->ev_side) (void)hipEventDestroy(c->ev_side);
    if (c->ev_done[0]) (void)hipEventDestroy(c->ev_done[0]);
    delete c;
    return CPPPL_E_HIP;
  }
  c->host_status = (int*)(c->host_scal + S_COUNT);
  *out = c;
  return CPPPL_OK;
}

CPPPL_API cpppl_status cpppl_bind_workspace(cpppl_ctx* c, void* dev_ptr, size_t bytes) {
  API_TRY(c)
  if (!dev_ptr) throw std::invalid_argument("workspace pointer is NULL");
  if (((uintptr_t)dev_ptr) % ALIGN) throw std::invalid_argument("workspace must be 256-byte aligned");
  if (bytes < c->plan.total)
    throw StatusError(CPPPL_E_NOMEM, "workspace too small: need " + std::to_string(c->plan.total) +
                                         " bytes, got " + std::to_string(bytes));
  c->ws = (char*)dev_ptr;
  c->ws_bytes = bytes;
  c->have_t = c->have_b = c->have_factors = c->planted = false;
  c->norm_valid = c->ybeta_valid = c->tau_valid = c->ws_valid = false;
  zero_ints(c->at<int>(c->plan.status), 16, c->stream);
  zero_doubles(c->at<double>(c->plan.scal), S_COUNT, c->stream);
  API_CATCH(c)
}

CPPPL_API cpppl_status cpppl_destroy(cpppl_ctx* c) {
  if (!c) return CPPPL_E_ARG;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  if (c->ev_main) (void)hipEventDestroy(c->ev_main);
  if (c->ev_side) (void)hipEventDestroy(c->ev_side);
  for (hipEvent_t e : c->ev_done)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->host_scal) (void)hipHostFree(c->host_scal);
  delete c;
  return CPPPL_OK;
}

CPPPL_API cpppl_status cpppl_load_t2(cpppl_ctx* c, const double* t, int on_device) {
  API_TRY(c)
  need_ws(c);
  if (!t) throw std::invalid_argument("t is NULL");
  const int64_t n = c->d.o * c->d.o * c->d.v * c->d.v;
  if (c->d.singles) {  // keep the raw doubles; t64 holds what the chain contracts
    load_device_or_host(c, c->at(c->plan.t2raw), t, (size_t)n * 8, on_device);
    check_finite_input(c, c->at<double>(c->plan.t2raw), n, "t2");
    dress_t(c);
  } else {
    load_device_or_host(c, c->at(c->plan.t64), t, (size_t)n * 8, on_device);
    check_finite_input(c, c->at<double>(c->plan.t64), n, "t2");
    derive_t(c);
  }
  c->have_t = true;
  c->planted = false;
  c->norm_valid = false;
  c->ybeta_valid = c->tau_valid = false;
  API_CATCH(c)
}

CPPPL_API cpppl_status cpppl_load_singles(cpppl_ctx* c, const double* t1, const double* b_vo,
                                          int on_device) {
  API_TRY(c)
  need_ws(c);
  if (!c->d.singles)
    throw StatusError(CPPPL_E_UNSUPPORTED, "context created without room for singles (dims.singles = 0)");
  if (c->planted) throw StatusError(CPPPL_E_STATE, "no singles dressing for a planted tensor");
  if (!c->have_t || !c->have_b) throw StatusError(CPPPL_E_STATE, "load t2 and the DF tensor first");
  const Plan& p = c->plan;
  const int64_t o = c->d.o, v = c->d.v, X = c->d.nx;
  if (t1) {
    if (!b_vo) throw std::invalid_argument("b_vo is NULL");
    load_device_or_host(c, c->at(p.t1), t1, (size_t)(o * v) * 8, on_device);
    load_device_or_host(c, c->at(p.bvo), b_vo, (size_t)(X * v * o) * 8, on_device);
    check_finite_input(c, c->at<double>(p.t1), o * v, "t1");
    check_finite_input(c, c->at<double>(p.bvo), X * v * o, "the virtual-occupied DF block");
    c->singles_on = true;
    derive_dbar(c);
  } else {
    c->singles_on = false;
  }
  dress_t(c);
  c->norm_valid = false;
  c->ybeta_valid = c->tau_valid = false;
  API_CATCH(c)
}

CPPPL_API cpppl_status cpppl_load_df(cpppl_ctx* c, const double* b, int on_device) {
  API_TRY(c)
  need_ws(c);
  if (!b) throw std::invalid_argument("b is NULL");
  const int64_t v = c->d.v, X = c->d.nx, n = X * v * v;
  const Plan& p = c->plan;
  load_device_or_host(c, c->at(p.b64), b, (size_t)n * 8, on_device);
  check_finite_input(c, c->at<double>(p.b64), n, "the DF tensor");
  derive_b(c, p.b64, BLayouts{p.b64T, p.b64P, p.b16T, p.b16P, p.b8T, p.b8P, p.sB, p.sBx});
  if (c->singles_on) derive_dbar(c);
  c->have_b = true;
  c->planted = false;
  c->norm_valid = false;
  c->ybeta_valid = c->tau_valid = false;
  API_CATCH(c)
}

CPPPL_API cpppl_status cpppl_load_planted(cpppl_ctx* c, const double* fi, const double* fj,
                                          const double* fa, const double* fb, const double* lam,
                                          int64_t rank_p, int on_device) {
  API_TRY(c)
  need_ws(c);
  if (!fi || !fj || !fa || !fb) throw std::invalid_argument("planted factor is NULL");
  if (rank_p < 1 || rank_p > c->d.rank) throw std::invalid_argument("planted rank must be in [1, rank]");
  const Plan& p = c->plan;
  const double* src[4] = {fi, fj, fa, fb};
  for (int m = 0; m < 4; ++m) {
    const int64_t n = nmode(c->d, m);
    load_device_or_host(c, c->at(p.stage), src[m], (size_t)(n * rank_p) * 8, on_device);
    transpose_batched(c->at<double>(p.stage), c->at(p.FpT[m]), DType::F64, 1, n, rank_p, c->stream);
  }
  if (lam) {
    load_device_or_host(c, c->at(p.lamp), lam, (size_t)rank_p * 8, on_device);
  } else {
    std::vector<double> ones((size_t)rank_p, 1.0);
    load_device_or_host(c, c->at(p.lamp), ones.data(), (size_t)rank_p * 8, 0);
  }
  c->rank_p = rank_p;
  c->planted = true;
  c->norm_valid = false;
  c->ybeta_valid = c->tau_valid = false;
  API_CATCH(c)
}

CPPPL_API cpppl_status cpppl_norm_r2(cpppl_ctx* c, double* norm_r2, double* energy_exact) {
  API_TRY(c)
  need_ws(c);
  if (!norm_r2) throw std::invalid_argument("norm_r2 is NULL");
  if (!c->planted && !(c->have_t && c->have_b)) throw StatusError(CPPPL_E_STATE, "load t2 and B first");
  ensure_norm(c);
  CPPPL_HIP(hipMemcpyAsync(c->host_scal, c->at(c->plan.scal), S_COUNT * 8, hipMemcpyDeviceToHost, c->stream));
  sync(c);
  *norm_r2 = c->host_scal[S_NORM_R2];
  if (energy_exact) *energy_exact = c->host_scal[S_E_EXACT];
  API_CATCH(c)
}

CPPPL_API cpppl_status cpppl_set_factors(cpppl_ctx* c, const double* fi, const double* fj,
                                         const double* fa, const double* fb, const double* lam,
                                         int on_device) {
  API_TRY(c)
  need_ws(c);
  if (!fi || !fj || !fa || !fb) throw std::invalid_argument("factor is NULL");
  const Plan& p = c->plan;
  const int64_t R = c->d.rank;
  const double* src[4] = {fi, fj, fa, fb};
  for (int m = 0; m < 4; ++m) {
    const int64_t n = nmode(c->d, m);
    load_device_or_host(c, c->at(p.stage), src[m], (size_t)(n * R) * 8, on_device);
    check_finite_input(c, c->at<double>(p.stage), n * R, "a factor");
    transpose_batched(c->at<double>(p.stage), c->at(p.FT[m]), DType::F64, 1, n, R, c->stream);
  }
  if (lam) {
    load_device_or_host(c, c->at(p.lam), lam, (size_t)R * 8, on_device);
  } else {
    std::vector<double> ones((size_t)R, 1.0);
    load_device_or_host(c, c->at(p.lam), ones.data(), (size_t)R * 8, 0);
  }
  init_after_factors(c);
  c->ws_valid = false;
  API_CATCH(c)
}

CPPPL_API cpppl_status cpppl_init_random(cpppl_ctx* c, uint64_t seed) {
  API_TRY(c)
  need_ws(c);
  const Plan& p = c->plan;
  const int64_t R = c->d.rank;
  uint64_t offset = 0;
  for (int m = 0; m < 4; ++m) {  // API order (i, j, a, b), element (row, r) is draw offset + row R + r
    const int64_t n = nmode(c->d, m);
    random_factor(c->at<double>(p.FT[m]), n, R, seed, offset, c->stream);
    offset += (uint64_t)(n * R);
  }
  fill_doubles(c->at<double>(p.lam), R, 1.0, c->stream);
  init_after_factors(c);
  c->ws_valid = false;
  sync(c);
  API_CATCH(c)
}

CPPPL_API cpppl_status cpppl_get_factors(cpppl_ctx* c, double* fi, double* fj, double* fa,
                                         double* fb, double* lam, int on_device) {
  API_TRY(c)
  need_ws(c);
  if (!c->have_factors) throw StatusError(CPPPL_E_STATE, "no factors set");
  const Plan& p = c->plan;
  const int64_t R = c->d.rank;
  double* dst[4] = {fi, fj, fa, fb};
  for (int m = 0; m < 4; ++m) {
    if (!dst[m]) continue;
    const int64_t n = nmode(c->d, m);
    transpose_batched(c->at<double>(p.FT[m]), c->at(p.stage), DType::F64, 1, R, n, c->stream);
    CPPPL_HIP(hipMemcpyAsync(dst[m], c->at(p.stage), (size_t)(n * R) * 8,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    if (!on_device) sync(c);
  }
  if (lam)
    CPPPL_HIP(hipMemcpyAsync(lam, c->at(p.lam), (size_t)R * 8,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  sync(c);
  API_CATCH(c)
}

CPPPL_API cpppl_status cpppl_mttkrp(cpppl_ctx* c, int mode, cpppl_precision prec, double* m_out,
                                    int on_device) {
  API_TRY(c)
  if (mode < 0 || mode > 3) throw std::invalid_argument("mode must be 0..3");
  if (!m_out) throw std::invalid_argument("m_out is NULL");
  require_inputs(c);
  if (prec != CPPPL_FP64 && prec != c->prec)
    throw StatusError(CPPPL_E_UNSUPPORTED, "MTTKRP precision must be FP64 or the context's");
  mttkrp_into_MT(c, path_for(c, prec == CPPPL_FP64 ? DType::F64 : DType::BF16), mode);
  const int64_t n = nmode(c->d, mode), R = c->d.rank;
  transpose_batched(c->at<double>(c->plan.MT), c->at(c->plan.stage), DType::F64, 1, R, n, c->stream);
  CPPPL_HIP(hipMemcpyAsync(m_out, c->at(c->plan.stage), (size_t)(n * R) * 8,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  sync(c);
  API_CATCH(c)
}

CPPPL_API cpppl_status cpppl_fit(cpppl_ctx* c, double* fit, double* inner, double* cp_norm2) {
  API_TRY(c)
  require_inputs(c);
  ensure_norm(c);
  const Plan& p = c->plan;
  mttkrp_into_MT(c, path_for(c, DType::F64), 1);
  const double* G[4];
  for (int m = 0; m < 4; ++m) G[m] = c->at<double>(p.gram[m]);
  fit_scalars(c->at<double>(p.MT), c->at<double>(p.FT[1]), c->d.o, c->at<double>(p.lam), G, c->d.rank,
              c->at<double>(p.scal) + S_NORM_R2, c->at<double>(p.rowbuf),
              c->at<double>(p.scal) + S_JUDGE, c->stream);
  CPPPL_HIP(hipMemcpyAsync(c->host_scal, c->at(p.scal), S_COUNT * 8, hipMemcpyDeviceToHost, c->stream));
  sync(c);
  if (fit) *fit = c->host_scal[S_JUDGE + 3];
  if (inner) *inner = c->host_scal[S_JUDGE + 0];
  if (cp_norm2) *cp_norm2 = c->host_scal[S_JUDGE + 1];
  API_CATCH(c)
}

CPPPL_API cpppl_status cpppl_reconstruct(cpppl_ctx* c, double* out, int symmetrize, int on_device) {
  API_TRY(c)
  need_ws(c);
  if (!out) throw std::invalid_argument("out is NULL");
  if (!c->have_factors) throw StatusError(CPPPL_E_STATE, "set the factors first");
  const Plan& p = c->plan;
  const int64_t o = c->d.o, v = c->d.v, R = c->d.rank;
  double* dst = on_device ? out : c->at<double>(p.dt64);  // dt64 stages a host result
  // KR(gamma, rho) diag(lambda) and KR(alpha, beta), both R x (pairs); the
  // second lives in the intermediate region, whose cached Y_beta is dropped
  khatri_rao_t(c->at<double>(p.FT[0]), c->at<double>(p.FT[1]), o, R, c->at(p.Kt), DType::F64,
               c->stream, nullptr, c->at<double>(p.lam));
  khatri_rao_t(c->at<double>(p.FT[2]), c->at<double>(p.FT[3]), v, R, c->at(p.big), DType::F64,
               c->stream);
  c->ybeta_valid = c->tau_valid = false;
  Gemm g;  // CP[ij][ab] = sum_r Kt[r][ij] Ka[r][ab]
  g.M = o * o; g.N = v * v; g.K = R;
  g.A = c->at(p.Kt); g.sam = 1; g.sak = o * o;
  g.B = c->at(p.big); g.sbk = v * v; g.sbn = 1;
  g.C = dst; g.scm = v * v; g.ctype = DType::F64;
  gemm_f64(g, c->stream);
  if (symmetrize) symmetrize_pairs(dst, o, v, c->stream);
  if (!on_device)
    CPPPL_HIP(hipMemcpyAsync(out, dst, (size_t)(o * o * v * v) * 8, hipMemcpyDeviceToHost, c->stream));
  sync(c);
  API_CATCH(c)
}

CPPPL_API cpppl_status cpppl_jacobi_step(cpppl_ctx* c, const double* w, const double* e_occ,
                                         const double* e_vir, double scale, double* dt,
                                         int on_device) {
  API_TRY(c)
  need_ws(c);
  if (!w || !e_occ || !e_vir || !dt) throw std::invalid_argument("NULL argument");
  if (!std::isfinite(scale)) throw std::invalid_argument("scale must be finite");
  if (c->planted || !c->have_t || !c->have_b) throw StatusError(CPPPL_E_STATE, "load t2 and B first");
  if (!c->have_factors) throw StatusError(CPPPL_E_STATE, "set the factors first");
  const Plan& p = c->plan;
  const int64_t o = c->d.o, v = c->d.v, R = c->d.rank;
  const int64_t n = o * o * v * v;
  // the doubles amplitudes (the raw t2 when a singles dressing is on)
  const double* t = c->at<double>(c->singles_on ? p.t2raw : p.t64);
  load_device_or_host(c, c->at(p.eorb), e_occ, (size_t)o * 8, on_device);
  load_device_or_host(c, c->at<double>(p.eorb) + o, e_vir, (size_t)v * 8, on_device);
  const double* wd = w;
  if (!on_device) {  // stage w where dt is formed
    load_device_or_host(c, c->at(p.dt64), w, (size_t)n * 8, 0);
    wd = c->at<double>(p.dt64);
  }
  // CP (FP64, one GEMM of two Khatri-Rao products, as in cpppl_reconstruct) into dt64T
  khatri_rao_t(c->at<double>(p.FT[0]), c->at<double>(p.FT[1]), o, R, c->at(p.Kt), DType::F64,
               c->stream, nullptr, c->at<double>(p.lam));
  khatri_rao_t(c->at<double>(p.FT[2]), c->at<double>(p.FT[3]), v, R, c->at(p.big), DType::F64,
               c->stream);
  c->ybeta_valid = c->tau_valid = false;
  Gemm g;
  g.M = o * o; g.N = v * v; g.K = R;
  g.A = c->at(p.Kt); g.sam = 1; g.sak = o * o;
  g.B = c->at(p.big); g.sbk = v * v; g.sbn = 1;
  g.C = c->at(p.dt64T); g.scm = v * v; g.ctype = DType::F64;
  gemm_f64(g, c->stream);
  double* out = on_device ? dt : c->at<double>(p.dt64);
  jacobi_delta(c->at<double>(p.dt64T), wd, c->at<double>(p.eorb), c->at<double>(p.eorb) + o, scale,
               t, out, o, v, c->stream);
  if (!on_device)
    CPPPL_HIP(hipMemcpyAsync(dt, out, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
  sync(c);
  API_CATCH(c)
}

CPPPL_API cpppl_status cpppl_energy(cpppl_ctx* c, double* e_cp) {
  API_TRY(c)
  if (!e_cp) throw std::invalid_argument("e_cp is NULL");
  require_inputs(c);
  if (c->planted) throw StatusError(CPPPL_E_UNSUPPORTED, "no amplitudes for a planted tensor");
  compute_energy(c, c->at<double>(c->plan.scal) + S_ENERGY);
  CPPPL_HIP(hipMemcpyAsync(c->host_scal, c->at(c->plan.scal), S_COUNT * 8, hipMemcpyDeviceToHost, c->stream));
  sync(c);
  *e_cp = c->host_scal[S_ENERGY];
  API_CATCH(c)
}

CPPPL_API cpppl_status cpppl_als(cpppl_ctx* c, const cpppl_als_opts* opts, cpppl_als_report* rep) {
  API_TRY(c)
  if (!opts || !rep) throw std::invalid_argument("opts/report is NULL");
  if (opts->max_sweeps < 0 || opts->refine_fp64_sweeps < 0) throw std::invalid_argument("negative sweep count");
  if (opts->stop_rule < 0 || opts->stop_rule > 3) throw std::invalid_argument("stop_rule must be 0..3");
  if (!(opts->refine_tol >= 0.0)) throw std::invalid_argument("refine_tol must be >= 0");
  if (!(opts->refine_etol >= 0.0)) throw std::invalid_argument("refine_etol must be >= 0");
  if (opts->stop_window < 0 || opts->stop_window > 64) throw std::invalid_argument("stop_window must be 0..64");
  const int win = opts->stop_window > 1 ? opts->stop_window : 1;
  c->want_eta = opts->eta != 0 || opts->stop_rule == 2;
  std::vector<double> main_fits, main_energies;
  require_inputs(c);
  if (c->planted && (opts->stop_rule == 3 || opts->energy_every || opts->refine_etol > 0.0))
    throw StatusError(CPPPL_E_UNSUPPORTED, "no energy for a planted tensor");
  // energy every sweep: on request, for the energy stop rule, and in the FP64
  // refinement when it stops on the energy change
  const bool energy_main = opts->energy_every != 0 || opts->stop_rule == 3;
  const bool energy_refine = energy_main || opts->refine_etol > 0.0;
  ensure_norm(c);
  const Plan& p = c->plan;
  c->timing = opts->timing != 0;
  c->ev_used = 0;
  c->segs.clear();
  rep->sweeps_done = 0;
  rep->refine_done = 0;
  rep->ridge_retries = 0;
  rep->careful_sweeps = 0;
  rep->energy_cp = std::numeric_limits<double>::quiet_NaN();
  for (int k = 0; k < 16; ++k) { rep->ms_class[k] = 0.0; rep->n_class[k] = 0; }
  const DType main_dt = c->prec != CPPPL_FP64 ? DType::BF16 : DType::F64;
  const int total = opts->max_sweeps + (c->prec != CPPPL_FP64 ? opts->refine_fp64_sweeps : 0);
  double prev_fit = std::numeric_limits<double>::quiet_NaN();
  double prev_energy = std::numeric_limits<double>::quiet_NaN();
  drop_early_fork(c);
  sync(c);
  const auto t_start = std::chrono::steady_clock::now();
  auto t_prev = t_start;
  bool stop_main = false;
  // A sweep is issued before the host reads the previous sweep's results, so
  // the GPU does not idle while the host checks a fit or a pivot status.  A
  // sweep issued past a stop, or after a sweep whose pivot failed, is rolled
  // back from its snapshot.  (With the near-optimal cache, whose ring holds
  // the last six iterates, sweeps are issued one at a time.)
  const bool ahead = !opts->near_cache;
  auto next_of = [&](int s) {
    if (s < opts->max_sweeps && stop_main) s = opts->max_sweeps;
    return s < total ? s : -1;
  };
  auto path_of = [&](int s) { return path_for(c, s >= opts->max_sweeps ? DType::F64 : main_dt); };
  const size_t slot_bytes = S_COUNT * 8 + 16 * sizeof(int);
  auto host_slot = [&](int k) { return c->host_scal + (size_t)k * (S_COUNT + 8); };
  // Status words 2 and 3 (by sweep parity) flag a failed pivot in an alpha
  // inverse forked during the previous sweep; alpha_word[slot] names the one
  // that belongs to the sweep in that slot (-1: none).
  int alpha_word[2] = {-1, -1};
  // sweep s with its snapshot in the other slot; its scalars and status go to
  // that slot's host buffer, marked by ev_done[slot]
  auto issue = [&](int s) {
    const int slot = c->snap ^ 1;
    alpha_word[slot] = c->alpha_forked ? 2 + (s & 1) : -1;
    snapshot(c, slot);
    zero_ints(c->at<int>(p.status), 1, c->stream);
    const int early = ahead && !c->planted && next_of(s + 1) >= 0 ? 2 + ((s + 1) & 1) : -1;
    c->want_energy = s >= opts->max_sweeps ? energy_refine : energy_main;
    c->inject_now = early >= 0 && s + 1 == c->inject_alpha_fault;
    (void)sweep(c, path_of(s), false, early);
    c->inject_now = false;
    if (opts->near_cache)
      copy_factor_set(c, p.nearRing + (size_t)(rep->sweeps_done % 6) * factor_set_bytes(c), true);
    CPPPL_HIP(hipMemcpyAsync(host_slot(slot), c->at(p.scal), slot_bytes, hipMemcpyDeviceToHost,
                             c->stream));
    CPPPL_HIP(hipEventRecord(c->ev_done[slot], c->stream));
    return slot;
  };
  int cur = next_of(0);
  int cur_slot = cur >= 0 ? issue(cur) : 0;
  while (cur >= 0) {
    int nxt = ahead ? next_of(cur + 1) : -1;
    const int nxt_slot = nxt >= 0 ? issue(nxt) : 0;
    CPPPL_HIP(hipEventSynchronize(c->ev_done[cur_slot]));
    double* hs = host_slot(cur_slot);
    int retries = 0;
    const int* hst = (const int*)(hs + S_COUNT);
    if (hst[0] || (alpha_word[cur_slot] >= 0 && hst[alpha_word[cur_slot]])) {
      // a pivot of the W inverse failed: drop the sweep issued after this one and redo
      // this sweep from its snapshot with ridge retries
      sync(c);
      nxt = -1;
      restore_snapshot(c, cur_slot);
      CPPPL_HIP(hipMemcpyAsync(c->at<double>(p.scal) + S_CP2_PREV, hs + S_ETA + 2, 8,
                               hipMemcpyHostToDevice, c->stream));
      c->want_energy = cur >= opts->max_sweeps ? energy_refine : energy_main;
      retries = sweep(c, path_of(cur), true);
      rep->careful_sweeps++;
      if (opts->near_cache)
        copy_factor_set(c, p.nearRing + (size_t)(rep->sweeps_done % 6) * factor_set_bytes(c), true);
      CPPPL_HIP(hipMemcpyAsync(hs, c->at(p.scal), S_COUNT * 8, hipMemcpyDeviceToHost, c->stream));
      sync(c);
    }
    const bool refining = cur >= opts->max_sweeps;
    rep->ridge_retries += retries;
    const double fit = hs[S_FIT + 3];
    const double eta = c->want_eta ? hs[S_ETA + 3] : std::numeric_limits<double>::quiet_NaN();
    const bool have_e = cur >= opts->max_sweeps ? energy_refine : energy_main;
    const double energy = have_e ? hs[S_ENERGY] : std::numeric_limits<double>::quiet_NaN();
    if (!std::isfinite(fit) || !std::isfinite(hs[S_FIT + 1])) {
      sync(c);
      throw StatusError(CPPPL_E_NONFINITE, "non-finite fit after sweep " + std::to_string(cur + 1));
    }
    const auto t_now = std::chrono::steady_clock::now();
    const double ms = std::chrono::duration<double, std::milli>(t_now - t_prev).count();
    t_prev = t_now;
    if (rep->fit_hist && rep->sweeps_done < opts->history_cap) rep->fit_hist[rep->sweeps_done] = fit;
    if (rep->eta_hist && rep->sweeps_done < opts->history_cap) rep->eta_hist[rep->sweeps_done] = eta;
    if (rep->ms_hist && rep->sweeps_done < opts->history_cap) rep->ms_hist[rep->sweeps_done] = ms;
    if (rep->energy_hist && rep->sweeps_done < opts->history_cap)
      rep->energy_hist[rep->sweeps_done] = energy;
    rep->sweeps_done++;
    if (refining) rep->refine_done++;
    rep->fit = fit;
    rep->eta = eta;
    rep->inner = hs[S_FIT + 0];
    rep->cp_norm2 = hs[S_FIT + 1];
    rep->loss = hs[S_FIT + 4];
    bool done = false;
    if (!refining) {
      main_fits.push_back(fit);
      const size_t nf = main_fits.size();
      if (opts->stop_rule == 1 && nf > (size_t)win &&
          std::fabs(fit - main_fits[nf - 1 - win]) / win < opts->tol)
        stop_main = true;
      if (opts->stop_rule == 2 && eta < opts->tol) stop_main = true;
      main_energies.push_back(energy);
      const size_t ne = main_energies.size();
      if (opts->stop_rule == 3 && ne > (size_t)win &&
          std::fabs(energy - main_energies[ne - 1 - win]) / win < opts->tol)
        stop_main = true;
    } else if (opts->refine_tol > 0.0 || opts->refine_etol > 0.0) {
      // the refinement stops once every criterion that is set holds; the
      // energy change is taken between two FP64 sweeps (the last main sweep's
      // energy, if any, came from low-precision operands)
      const bool fit_ok = opts->refine_tol <= 0.0 || std::fabs(fit - prev_fit) < opts->refine_tol;
      const bool e_ok = opts->refine_etol <= 0.0 ||
                        (rep->refine_done >= 2 && std::fabs(energy - prev_energy) < opts->refine_etol);
      done = fit_ok && e_ok;
    }
    prev_fit = fit;
    prev_energy = energy;
    const int want = done ? -1 : next_of(cur + 1);
    if (nxt >= 0 && nxt != want) {
      // the sweep issued ahead is past a stop: back to the state after this
      // sweep (factors from the next snapshot, scalars from this readback)
      sync(c);
      c->alpha_forked = false;  // forked from the state being rolled back
      restore_snapshot(c, nxt_slot);
      CPPPL_HIP(hipMemcpyAsync(c->at(p.scal), hs, S_COUNT * 8, hipMemcpyHostToDevice, c->stream));
      sync(c);
      nxt = -1;
    }
    if (nxt < 0 && want >= 0) {
      cur = want;
      cur_slot = issue(cur);
    } else {
      cur = nxt;
      cur_slot = nxt_slot;
    }
  }
  if (opts->near_cache && rep->sweeps_done > 5) {  // the (n-5)th iterate becomes the cache
    const size_t sb = factor_set_bytes(c);
    copy_d2d(c, p.nearCache, p.nearRing + (size_t)((rep->sweeps_done - 6) % 6) * sb, sb);
    c->near_valid = true;
  }
  if (opts->energy) {
    compute_energy(c, c->at<double>(p.scal) + S_ENERGY);
    CPPPL_HIP(hipMemcpyAsync(c->host_scal, c->at(p.scal), S_COUNT * 8, hipMemcpyDeviceToHost, c->stream));
  }
  sync(c);
  c->alpha_forked = false;
  c->want_energy = false;
  c->inject_alpha_fault = -1;
  rep->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  if (opts->energy) rep->energy_cp = c->host_scal[S_ENERGY];
  if (c->timing) {
    for (auto& sg : c->segs) {
      float ms = 0.f;
      CPPPL_HIP(hipEventElapsedTime(&ms, sg.a, sg.b));
      rep->ms_class[sg.cls] += ms;
      rep->n_class[sg.cls] += sg.calls;
    }
    c->segs.clear();
    c->timing = false;
  }
  API_CATCH(c)
}

CPPPL_API cpppl_status cpppl_test_inject_alpha_fault(cpppl_ctx* c, int sweep) {
  if (!c || sweep < -1) return CPPPL_E_ARG;
  c->inject_alpha_fault = sweep;
  return CPPPL_OK;
}

CPPPL_API const char* cpppl_last_error(const cpppl_ctx* c) { return c ? c->err.c_str() : "null context"; }

#ifndef CPPPL_SRC_HASH
#define CPPPL_SRC_HASH "unknown"
#endif
CPPPL_API const char* cpppl_build_hash(void) { return CPPPL_SRC_HASH; }

CPPPL_API const char* cpppl_status_str(cpppl_status s) {
  switch (s) {
    case CPPPL_OK: return "ok";
    case CPPPL_E_ARG: return "invalid argument";
    case CPPPL_E_STATE: return "invalid state";
    case CPPPL_E_HIP: return "HIP error";
    case CPPPL_E_NOMEM: return "out of memory";
    case CPPPL_E_NOT_SPD: return "normal equations not positive definite";
    case CPPPL_E_NONFINITE: return "non-finite values";
    case CPPPL_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

}  // extern "C"
