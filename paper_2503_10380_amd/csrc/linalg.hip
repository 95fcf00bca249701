// Block sweep-operator inverse of the ALS normal-equation matrix, FP64.
//
// Sweeping pivot block k of a symmetric matrix A (D = A_kk^{-1}):
//   A_ij <- A_ij - A_ik D A_kj   (i, j != k)
//   A_ik <- A_ik D,  A_kj <- D A_kj,  A_kk <- -D
// After every block has been swept once, A holds -A^{-1}.
//
// One launch per block step, one work-group per 64 x 64 output tile of the
// upper triangle (it also writes the mirror tile), two matrix buffers
// alternating so no launch reads what it writes.  The pivot
// inverse is looked ahead: the work-group whose output tile is the next
// diagonal block (dispatched first) inverts that tile right after computing it
// and publishes D for the next launch, so each 64 x 64 inverse is done once per
// step instead of once per work-group.  The first pivot is inverted by a
// one-group launch of its own.
//
// The 64 x 64 pivot inverse runs in registers, each wave holding a slab of
// 16 rows in the f64 matrix-core result layout, as four 16-wide block sweeps.
// The wave that owns a panel's rows inverts its 16 x 16 pivot block in place,
// two pivots per step (pivot block by readlane, pivot columns by DPP row
// broadcasts, pivot rows by 64-bit bpermutes, reciprocal refined by Newton
// steps) and publishes the inverse and its rows; the other waves form their
// column-panel products and rank-16 updates on the matrix cores with operands
// taken from registers (the matrix is symmetric, so the published pivot rows
// also give the pivot columns).  The owner of the next panel updates its rows
// first and starts the next pivot inverse while the others finish, so a panel
// needs one barrier.
#include "linalg.h"

#include <utility>

namespace cpppl {

namespace {

constexpr int NB = INV_NB;
constexpr int LD = NB + 1;
constexpr int PW = 16;  // panel width of the blocked pivot inverse
constexpr int KS = NB / 4;  // k-steps of a 64-deep f64 MFMA product

// LDS scratch of the pivot inverse: the published pivot rows (16 x LDR) and
// pivot inverse (16 x 16) of two consecutive panels; also used to move a
// register tile into the slab layout (NB x LD).
constexpr int LDR = NB + 16;
constexpr int GJ_PANEL = PW * LDR + PW * PW;
constexpr int GJ_SCRATCH = (2 * GJ_PANEL + NB > NB * LD) ? 2 * GJ_PANEL + NB : NB * LD;
constexpr int T1_SIZE = NB * LD > GJ_SCRATCH ? NB * LD : GJ_SCRATCH;

// Register tiles use the v_mfma_f64_16x16x4f64 accumulator layout: wave w owns
// the 32 x 32 sub-tile (rows 32 (w / 2) + ..., columns 32 (w % 2) + ...) as
// 2 x 2 blocks of 16 x 16; element (row, col) of a block is register row / 4
// of lane col + 16 (row % 4).
struct RTile {
  d4_t v[2][2];
};
__device__ __forceinline__ int rt_row(int i, int r) {
  return 32 * ((threadIdx.x >> 6) >> 1) + 16 * i + 4 * r + ((threadIdx.x & 63) >> 4);
}
__device__ __forceinline__ int rt_col(int j) {
  return 32 * ((threadIdx.x >> 6) & 1) + 16 * j + (threadIdx.x & 15);
}

__device__ __forceinline__ void rt_zero(RTile& t) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) t.v[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
}

// acc += (NEG ? -X : X)[rows][0:K] . Y[0:K][cols] with X (row stride ldx) and
// Y (row stride ldy) in LDS, on the f64 matrix cores.
template <int K, bool NEG>
__device__ __forceinline__ void mfma_mm(const double* X, int ldx, const double* Y, int ldy,
                                        RTile& acc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
#pragma unroll 4
  for (int k0 = 0; k0 < K; k0 += 4) {
    double a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double x = X[(32 * wm + 16 * i + (lane & 15)) * ldx + k0 + (lane >> 4)];
      a[i] = NEG ? -x : x;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = Y[(k0 + (lane >> 4)) * ldy + 32 * wn + 16 * j + (lane & 15)];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc.v[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc.v[i][j], 0, 0, 0);
  }
}

// As mfma_mm with K = NB, the right operand already in registers in the
// matrix-core B layout: bf[s][j] = Y(4 s + lane / 16, 32 (wave % 2) + 16 j + lane % 16).
template <bool NEG>
__device__ __forceinline__ void mfma_mm_rb(const double* X, int ldx, const double (&bf)[KS][2],
                                           RTile& acc) {
  const int lane = threadIdx.x & 63, wm = (threadIdx.x >> 6) >> 1;
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    double a[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double x = X[(32 * wm + 16 * i + (lane & 15)) * ldx + 4 * s + (lane >> 4)];
      a[i] = NEG ? -x : x;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc.v[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bf[s][j], acc.v[i][j], 0, 0, 0);
  }
}

__device__ __forceinline__ double readlane_f64(double x, int src) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1 / p from the hardware estimate and two Newton-Raphson steps
// (r <- r + r (1 - p r)); each step squares the relative error.
__device__ __forceinline__ double recip_nr(double p) {
  double r = __builtin_amdgcn_rcp(p);
  double e = fma(-p, r, 1.0);
  r = fma(r, e, r);
  e = fma(-p, r, 1.0);
  return fma(r, e, r);
}

// Value of lane 16 (lane / 16) + Q: a broadcast inside each row of 16 lanes.
template <int Q>
__device__ __forceinline__ double row_bcast_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, 0x150 + Q, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x150 + Q, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1 / sqrt(d) from the hardware estimate and two Newton-Raphson steps
// (y <- y (3 - d y^2) / 2); each step squares the relative error.
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  y = y * fma(-0.5 * d, y * y, 1.5);
  return y * fma(-0.5 * d, y * y, 1.5);
}

// In-wave Gauss-Jordan inverse (in place) of a 16 x 16 SPD block held in the
// f64 matrix-core result layout: lane l holds column l % 16, rows 4 c + l / 16
// in register c.  Element (i, j) is register i / 4 of lane 16 (i % 4) + j, so
// the pivot rows at a lane's column come from lanes 16 (k % 4) + l % 16 and the
// pivot columns at a lane's rows from lane 16 (l / 16) + k (a broadcast inside
// each row of 16 lanes).
//
// The pivots are taken two at a time, K = {k, k + 1}, each step one rank-2
// update g_ij -= C_i . R_j with R_j = D (g_Kj + e_K(j)), C_i = g_iK - e_K(i)
// and D the inverse of the 2 x 2 pivot block [[a, b], [b, c]] (a c - b^2 > 0
// for an SPD matrix).  For i, j outside K this is the block elimination
// g_ij - g_iK D g_Kj; it also turns the pivot rows into D g_Kj, the pivot
// columns into -g_iK D and the pivot block into D, which is what two single
// pivot steps (pivot -> 1 / p, row -> g_kj / p, column -> -g_ik / p) leave, so
// no entry needs a case of its own and the dependent chain is one 2 x 2
// inverse per two pivots.
template <int K>
__device__ __forceinline__ bool gj16_pair_step(d4_t& g) {
  constexpr int kr = K >> 2, kq = K & 3;  // rows K, K + 1: lane rows kq, kq + 1 of register kr
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, rq = lane >> 4;
  const double a = readlane_f64(g[kr], 16 * kq + K);
  const double b = readlane_f64(g[kr], 16 * kq + K + 1);
  const double c = readlane_f64(g[kr], 16 * (kq + 1) + K + 1);
  const double r0 = __shfl(g[kr], 16 * kq + col);        // g(K, col)
  const double r1 = __shfl(g[kr], 16 * (kq + 1) + col);  // g(K + 1, col)
  double c0[4], c1[4];                                   // g(row, K), g(row, K + 1)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    c0[q] = row_bcast_f64<K>(g[q]);
    c1[q] = row_bcast_f64<K + 1>(g[q]);
  }
  const double det = fma(-b, b, a * c);
  // a pivot block that is not positive definite is flagged and inverted with
  // 1 / det replaced by 1, so every entry stays finite
  const bool bad = !(a > 0.0) || !(det > 0.0) || !isfinite(det);
  double id = recip_nr(det);
  if (bad) id = 1.0;
  const double d00 = c * id, d01 = -b * id, d11 = a * id;
  const double u0 = r0 + (col == K ? 1.0 : 0.0), u1 = r1 + (col == K + 1 ? 1.0 : 0.0);
  const double R0 = fma(d00, u0, d01 * u1);
  const double R1 = fma(d01, u0, d11 * u1);
  c0[kr] -= (rq == kq) ? 1.0 : 0.0;
  c1[kr] -= (rq == kq + 1) ? 1.0 : 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) g[q] = fma(-c0[q], R0, fma(-c1[q], R1, g[q]));
  return !bad;
}

__device__ __forceinline__ bool gj16_block(d4_t& g) {
  bool ok = gj16_pair_step<0>(g);
  ok = gj16_pair_step<2>(g) && ok;
  ok = gj16_pair_step<4>(g) && ok;
  ok = gj16_pair_step<6>(g) && ok;
  ok = gj16_pair_step<8>(g) && ok;
  ok = gj16_pair_step<10>(g) && ok;
  ok = gj16_pair_step<12>(g) && ok;
  ok = gj16_pair_step<14>(g) && ok;
  return ok;
}

// A slab: wave w holds rows 16 w .. 16 w + 15 of an NB x NB tile as four
// 16 x 16 blocks in the matrix-core result layout: block j, register r of lane
// l is element (16 w + 4 r + l / 16, 16 j + l % 16).
struct Slab {
  d4_t b[NB / PW];
};
__device__ __forceinline__ int sl_row(int r) { return 16 * (threadIdx.x >> 6) + 4 * r + ((threadIdx.x & 63) >> 4); }
__device__ __forceinline__ int sl_col(int j) { return 16 * j + (threadIdx.x & 15); }

// P <- P^{-1} for the NB x NB SPD tile held as a slab.  The tile is first
// scaled to unit diagonal, S P S with S = diag(P)^{-1/2}, so that every pivot
// met afterwards (a Schur complement of a unit-diagonal SPD matrix) is at most
// 1, where the uniform pivot steps of gj16_block lose no precision; the result
// is scaled back, P^{-1} = S (S P S)^{-1} S.  A diagonal entry that is <= 0 or
// not finite counts as a bad pivot and is replaced by 1.  Then four 16-wide
// block sweeps (they leave -P^{-1}, negated at the end).  Panel p: wave p
// inverts its diagonal block (D), publishes D and its other blocks (the pivot
// rows), and replaces its blocks by -D and D P_pj; every other wave w forms
// Cp = P_wp D and its transpose (P_wp read as the transposed pivot rows),
// updates P_wj -= Cp P_pj and sets P_wp = Cp.  `ws` holds GJ_SCRATCH doubles.
// Returns false (in the wave that met it) if a pivot was not positive.
__device__ bool gj_inverse_slab(Slab& P, double* ws) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane >> 4, lc = lane & 15;
  bool ok = true;
  double* dg = ws + 2 * GJ_PANEL;  // the diagonal (NB)
  {
    // lanes whose column matches one of their rows hold a diagonal entry of block `wave`
    const int q = lc >> 2;
#pragma unroll
    for (int j = 0; j < NB / PW; ++j)
      if (j == wave && (lc & 3) == lr)
        dg[16 * j + lc] = q == 0 ? P.b[j][0] : (q == 1 ? P.b[j][1] : (q == 2 ? P.b[j][2] : P.b[j][3]));
  }
  __syncthreads();
  double sr[4], sc[NB / PW];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double d = dg[16 * wave + 4 * r + lr];
    if (!(d > 0.0) || !isfinite(d)) { ok = false; d = 1.0; }
    sr[r] = rsqrt_nr(d);
  }
#pragma unroll
  for (int j = 0; j < NB / PW; ++j) {
    double d = dg[16 * j + lc];
    if (!(d > 0.0) || !isfinite(d)) d = 1.0;
    sc[j] = rsqrt_nr(d);
  }
#pragma unroll
  for (int j = 0; j < NB / PW; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) P.b[j][r] *= sr[r] * sc[j];
#pragma unroll
  for (int p = 0; p < NB / PW; ++p) {
    double* Rp = ws + (p & 1) * GJ_PANEL;  // pivot rows (PW x LDR)
    double* Dp = Rp + PW * LDR;           // pivot inverse (PW x PW)
    d4_t dreg;
    if (wave == p) {
      ok = gj16_block(P.b[p]) && ok;
      dreg = P.b[p];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        Dp[(4 * r + lr) * PW + lc] = dreg[r];
#pragma unroll
        for (int j = 0; j < NB / PW; ++j)
          if (j != p) Rp[(4 * r + lr) * LDR + 16 * j + lc] = P.b[j][r];
      }
    }
    __syncthreads();
    if (wave == p) {  // own rows: P_pj <- D P_pj, P_pp <- -D
#pragma unroll
      for (int j = 0; j < NB / PW; ++j) {
        if (j == p) continue;
        d4_t acc = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(dreg[s2], P.b[j][s2], acc, 0, 0, 0);
        P.b[j] = acc;
      }
      P.b[p] = -dreg;
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) dreg[r] = Dp[(4 * r + lr) * PW + lc];
      double rw[4];  // P_pw (= P_wp^T) in B / A operand layout
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) rw[s2] = Rp[(4 * s2 + lr) * LDR + 16 * wave + lc];
      d4_t cp = d4_t{0.0, 0.0, 0.0, 0.0}, cpt = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        cp = __builtin_amdgcn_mfma_f64_16x16x4f64(rw[s2], dreg[s2], cp, 0, 0, 0);    // P_wp D
        cpt = __builtin_amdgcn_mfma_f64_16x16x4f64(dreg[s2], rw[s2], cpt, 0, 0, 0);  // D P_pw
      }
      // the next pivot's block first, so its inverse can start at once
      constexpr int order[4][4] = {{1, 2, 3, 0}, {2, 3, 0, 1}, {3, 0, 1, 2}, {0, 1, 2, 3}};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int j = order[p][t];
        if (j == p) continue;
        double rj[4];
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) rj[s2] = Rp[(4 * s2 + lr) * LDR + 16 * j + lc];
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2)
          P.b[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-cpt[s2], rj[s2], P.b[j], 0, 0, 0);
      }
      P.b[p] = cp;
    }
  }
#pragma unroll
  for (int j = 0; j < NB / PW; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) P.b[j][r] *= -(sr[r] * sc[j]);
  return ok;
}

// Pads rows / columns >= n of the tile with the identity (the tile is zero there).
__device__ __forceinline__ void rt_pad_identity(RTile& t, int n) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt_row(i, r), col = rt_col(j);
        if (row >= n || col >= n) t.v[i][j][r] = (row == col) ? 1.0 : 0.0;
      }
}

__device__ __forceinline__ void rt_store(const RTile& t, double* O, int64_t ld, int nr, int nc) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt_row(i, r), col = rt_col(j);
        if (row < nr && col < nc) O[row * ld + col] = t.v[i][j][r];
      }
}

__device__ __forceinline__ void slab_store(const Slab& t, double* O) {
#pragma unroll
  for (int j = 0; j < NB / PW; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) O[sl_row(r) * NB + sl_col(j)] = t.b[j][r];
}

// Inverts diagonal block 0 of A (n = min(NB, R) rows) into Dout (NB x NB,
// identity-padded).
__global__ __launch_bounds__(256) void first_pivot_kernel(const double* __restrict__ A,
                                                          double* __restrict__ Dout, int64_t R,
                                                          int* status) {
  __shared__ double ws[GJ_SCRATCH];
  const int n = (int)min((int64_t)NB, R);
  Slab p;
#pragma unroll
  for (int j = 0; j < NB / PW; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = sl_row(r), col = sl_col(j);
      p.b[j][r] = (row < n && col < n) ? A[row * R + col] : (row == col ? 1.0 : 0.0);
    }
  const bool ok = gj_inverse_slab(p, ws);
  if (!ok && (threadIdx.x & 63) == 0) status[0] = 1;
  slab_store(p, Dout);
}

// Tiles (I, J) with I <= J of a T x T tile grid, numbered row by row.
__device__ __forceinline__ int64_t upper_index(int64_t I, int64_t J, int64_t T) {
  return I * T - I * (I - 1) / 2 + (J - I);
}
__device__ __forceinline__ void upper_coords(int64_t u, int64_t T, int64_t& I, int64_t& J) {
  I = 0;
  while (u >= T - I) {
    u -= T - I;
    ++I;
  }
  J = I + u;
}

// One block step of the sweep; Dk = A_kk^{-1} (NB x NB) comes from the previous
// launch.  The swept matrix stays symmetric, so one group computes tile (I, J)
// for I <= J and also writes its transpose to (J, I).  The group whose output
// is diagonal block k + 1 also inverts that block into Dnext.
__global__ __launch_bounds__(256, 2) void sweep_kernel(const double* __restrict__ A,
                                                    double* __restrict__ O,
                                                    const double* __restrict__ Dk,
                                                    double* __restrict__ Dnext, int64_t R,
                                                    int64_t kb, int* status) {
  __shared__ double D[NB * LD];
  __shared__ double T1[T1_SIZE];  // A_Ik, then A_Ik D; the pivot inverse's scratch
  const int tid = threadIdx.x, lane = tid & 63, wn = (tid >> 6) & 1;
  const int64_t T = (R + NB - 1) / NB;
  const int64_t nu = T * (T + 1) / 2;
  // the next pivot's group is dispatched first
  const int64_t first = (kb + 1 < T) ? upper_index(kb + 1, kb + 1, T) : 0;
  int64_t I, J;
  upper_coords((blockIdx.x + first) % nu, T, I, J);
  const int64_t k0 = kb * NB, i0 = I * NB, j0 = J * NB;
  const int nk = (int)min((int64_t)NB, R - k0);
  const int ni = (int)min((int64_t)NB, R - i0);
  const int nj = (int)min((int64_t)NB, R - j0);
  const bool general = I != kb && J != kb;
  const bool need1 = I != kb;  // A_Ik
  const bool need2 = J != kb;  // A_kJ

  // A_Ik via LDS (coalesced rows), A_kJ straight into B-operand registers
  constexpr int PER = NB * NB / 256;
  double r1[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + q * 256, i = e / NB, j = e % NB;
    r1[q] = (need1 && i < ni && j < nk) ? A[(i0 + i) * R + k0 + j] : 0.0;
  }
  double bf[KS][2];
#pragma unroll
  for (int s = 0; s < KS; ++s)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int kr = 4 * s + (lane >> 4), col = 32 * wn + 16 * j + (lane & 15);
      bf[s][j] = (need2 && kr < nk && col < nj) ? A[(k0 + kr) * R + j0 + col] : 0.0;
    }
  RTile acc;  // A_IJ for the general tiles
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt_row(i, r), col = rt_col(j);
        acc.v[i][j][r] = (general && row < ni && col < nj) ? A[(i0 + row) * R + j0 + col] : 0.0;
      }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + q * 256, i = e / NB, j = e % NB;
    D[i * LD + j] = Dk[i * NB + j];
    T1[i * LD + j] = r1[q];
  }
  __syncthreads();

  RTile out;
  if (!need1 && !need2) {  // -D
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) out.v[i][j][r] = -D[rt_row(i, r) * LD + rt_col(j)];
  } else if (!need2) {  // A_Ik D
    rt_zero(out);
    mfma_mm<NB, false>(T1, LD, D, LD, out);
  } else if (!need1) {  // D A_kJ
    rt_zero(out);
    mfma_mm_rb<false>(D, LD, bf, out);
  } else {  // A_IJ - (A_Ik D) A_kJ
    RTile c;
    rt_zero(c);
    mfma_mm<NB, false>(T1, LD, D, LD, c);
    __syncthreads();  // every lane has read T1 before it is overwritten with C
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) T1[rt_row(i, r) * LD + rt_col(j)] = c.v[i][j][r];
    __syncthreads();
    out = acc;
    mfma_mm_rb<true>(T1, LD, bf, out);
  }
  rt_store(out, O + i0 * R + j0, R, ni, nj);
  if (I != J) {  // the mirror tile (J, I), transposed through LDS for row-wise stores
    __syncthreads();  // every lane has read T1
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) T1[rt_col(j) * LD + rt_row(i, r)] = out.v[i][j][r];
    __syncthreads();
    for (int e = tid; e < NB * NB; e += 256) {
      const int r = e / NB, cc = e % NB;
      if (r < nj && cc < ni) O[(j0 + r) * R + i0 + cc] = T1[r * LD + cc];
    }
  }

  if (I == kb + 1 && J == kb + 1) {  // look ahead: invert the next pivot block
    __syncthreads();                 // T1 is free: move the tile into the slab layout
    rt_pad_identity(out, ni);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) T1[rt_row(i, r) * LD + rt_col(j)] = out.v[i][j][r];
    __syncthreads();
    Slab piv;
#pragma unroll
    for (int j = 0; j < NB / PW; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) piv.b[j][r] = T1[sl_row(r) * LD + sl_col(j)];
    __syncthreads();  // T1 becomes the inverse's scratch
    const bool ok = gj_inverse_slab(piv, T1);
    if (!ok && lane == 0) status[0] = 1;
    slab_store(piv, Dnext);
  }
}

__global__ __launch_bounds__(256) void ridge_kernel(double* A, int64_t R, double delta) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < R; i += 256) s += A[i * R + i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  const double shift = delta * sh[0] / (double)R;
  for (int64_t i = threadIdx.x; i < R; i += 256) A[i * R + i] += shift;
}

}  // namespace

double* spd_inverse_neg(double* bufA, double* bufB, double* dbuf, int64_t R, int* status,
                        hipStream_t s) {
  const int64_t T = (R + NB - 1) / NB;
  if (T <= 0) return bufA;
  hipLaunchKernelGGL(first_pivot_kernel, dim3(1), dim3(256), 0, s, bufA, dbuf, R, status);
  CPPPL_LAUNCH_CHECK("first_pivot");
  double* in = bufA;
  double* out = bufB;
  for (int64_t kb = 0; kb < T; ++kb) {
    const double* dk = dbuf + (kb & 1) * NB * NB;
    double* dn = dbuf + ((kb + 1) & 1) * NB * NB;
    hipLaunchKernelGGL(sweep_kernel, dim3((unsigned)(T * (T + 1) / 2)), dim3(256), 0, s, in, out,
                       dk, dn, R, kb, status);
    CPPPL_LAUNCH_CHECK("sweep");
    std::swap(in, out);
  }
  return in;
}

void add_ridge(double* A, int64_t R, double delta, hipStream_t s) {
  hipLaunchKernelGGL(ridge_kernel, dim3(1), dim3(256), 0, s, A, R, delta);
  CPPPL_LAUNCH_CHECK("ridge");
}

}  // namespace cpppl
