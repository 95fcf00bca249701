// Block sweep-operator inverse of the ALS normal-equation matrix, FP64.
//
// Sweeping pivot block k of a symmetric matrix A (D = A_kk^{-1}):
//   A_ij <- A_ij - A_ik D A_kj   (i, j != k)
//   A_ik <- A_ik D,  A_kj <- D A_kj,  A_kk <- -D
// After every block has been swept once, A holds -A^{-1}.
//
// One launch per block step, one work-group per 64 x 64 output tile, two
// matrix buffers alternating so no launch reads what it writes.  The pivot
// inverse is looked ahead: the work-group whose output tile is the next
// diagonal block (dispatched first) inverts that tile right after computing it
// and publishes D for the next launch, so each 64 x 64 inverse is done once per
// step instead of once per work-group.  The first pivot is inverted by a
// one-group launch of its own.
//
// The 64 x 64 pivot inverse runs in registers: four 16-wide block sweeps, each
// with the 16 x 16 pivot block inverted inside one wave (readlane / DPP /
// bpermute, reciprocal refined by Newton steps) and the rank-16 update on the
// f64 matrix cores.  Symmetry is used throughout: the pivot column panel is
// the transposed pivot row panel, and D times the pivot rows is the transposed
// column panel times D.
#include "linalg.h"

#include <utility>

namespace cpppl {

namespace {

constexpr int NB = INV_NB;
constexpr int LD = NB + 1;
constexpr int PW = 16;  // panel width of the blocked pivot inverse
constexpr int KS = NB / 4;  // k-steps of a 64-deep f64 MFMA product

// LDS scratch of the pivot inverse: two pivot-row panels (PW x LD), two
// column-panel products (NB x 17) and the 16 x 16 pivot inverse (PW x 17).
constexpr int GJ_SCRATCH = 2 * PW * LD + 2 * NB * 17 + PW * 17;
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

// Value of lane (4 (lane / 4) + Q): a broadcast inside each group of four lanes.
template <int Q>
__device__ __forceinline__ double quad_bcast_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, Q * 0x55, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), Q * 0x55, 0xf, 0xf, false);
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

// In-wave Gauss-Jordan inverse of a 16 x 16 SPD block held 4 elements per
// lane: lane l holds row l / 4, columns 4 (l % 4) + c.  The pivot comes by
// readlane, the pivot column by a DPP broadcast inside the lane's group of
// four, the pivot row by bpermute; no LDS or barrier is involved.
__device__ __forceinline__ bool gj16_wave(double (&g)[4]) {
  const int lane = threadIdx.x & 63;
  const int i = lane >> 2, q = lane & 3;
  bool ok = true;
#pragma unroll
  for (int k = 0; k < PW; ++k) {
    const int kc = k & 3, kl = k >> 2;
    double p = readlane_f64(g[kc], 4 * k + kl);
    const bool bad = !(p > 0.0) || !isfinite(p);
    ok = ok && !bad;
    if (bad) p = 1.0;
    double rk[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) rk[c] = __shfl(g[c], 4 * k + q);
    double ck;
    switch (kl) {
      case 0: ck = quad_bcast_f64<0>(g[kc]); break;
      case 1: ck = quad_bcast_f64<1>(g[kc]); break;
      case 2: ck = quad_bcast_f64<2>(g[kc]); break;
      default: ck = quad_bcast_f64<3>(g[kc]); break;
    }
    const double inv = recip_nr(p);
    const double colv = -ck * inv;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = 4 * q + c;
      const double r = rk[c] * inv;
      const double gen = fma(-ck, r, g[c]);
      const double on_row = (j == k) ? inv : r;
      const double off_row = (j == k) ? colv : gen;
      g[c] = (i == k) ? on_row : off_row;
    }
  }
  return ok;
}

// P <- P^{-1} for the NB x NB SPD tile P held in registers (RTile layout), by
// four 16-wide block sweeps.  Per panel: the pivot rows go to LDS, wave 0
// inverts the 16 x 16 pivot block, every wave forms its 16 rows of
// Cp = P_{:,panel} D on the matrix cores (P_{:,panel} read as the transposed
// row panel), and the rank-16 update P -= Cp P_{panel,:} runs on the matrix
// cores; the row panel becomes Cp^T, the column panel Cp, the pivot block -D.
// Panel buffers alternate, so a panel needs three barriers.  `ws` is LDS
// scratch of GJ_SCRATCH doubles.  Returns false if a pivot was not positive.
__device__ bool gj_inverse_regs(RTile& P, double* ws) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double* Dp = ws + 2 * PW * LD + 2 * NB * 17;  // D (16 x 17)
  bool ok = true;
#pragma unroll
  for (int pnl = 0; pnl < NB / PW; ++pnl) {
    const int q0 = pnl * PW;
    double* Rp = ws + (pnl & 1) * PW * LD;                 // pivot rows (16 x LD)
    double* Cp = ws + 2 * PW * LD + (pnl & 1) * NB * 17;  // P_{:,panel} D (NB x 17)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rt_row(i, r);
          if (row >= q0 && row < q0 + PW) Rp[(row - q0) * LD + rt_col(j)] = P.v[i][j][r];
        }
    __syncthreads();
    if (wave == 0) {
      double g[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) g[c] = Rp[(lane >> 2) * LD + q0 + 4 * (lane & 3) + c];
      ok = gj16_wave(g) && ok;
#pragma unroll
      for (int c = 0; c < 4; ++c) Dp[(lane >> 2) * 17 + 4 * (lane & 3) + c] = g[c];
    }
    __syncthreads();
    {  // rows 16 wave .. 16 wave + 15 of Cp: A(m, k) = Rp[k][16 wave + m], B(k, n) = D[k][n]
      d4_t c = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < PW / 4; ++s) {
        const double a = Rp[(4 * s + (lane >> 4)) * LD + 16 * wave + (lane & 15)];
        const double b = Dp[(4 * s + (lane >> 4)) * 17 + (lane & 15)];
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) Cp[(16 * wave + 4 * r + (lane >> 4)) * 17 + (lane & 15)] = c[r];
    }
    __syncthreads();
    mfma_mm<PW, true>(Cp, 17, Rp, LD, P);  // P -= Cp Rp
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rt_row(i, r), col = rt_col(j);
          const bool ip = row >= q0 && row < q0 + PW, jp = col >= q0 && col < q0 + PW;
          if (ip && jp) P.v[i][j][r] = -Dp[(row - q0) * 17 + (col - q0)];
          else if (ip) P.v[i][j][r] = Cp[col * 17 + (row - q0)];
          else if (jp) P.v[i][j][r] = Cp[row * 17 + (col - q0)];
        }
  }
  // the sweeps leave -P^{-1}
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) P.v[i][j] = -P.v[i][j];
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

// Inverts diagonal block 0 of A (n = min(NB, R) rows) into Dout (NB x NB,
// identity-padded).
__global__ __launch_bounds__(256) void first_pivot_kernel(const double* __restrict__ A,
                                                          double* __restrict__ Dout, int64_t R,
                                                          int* status) {
  __shared__ double ws[GJ_SCRATCH];
  const int n = (int)min((int64_t)NB, R);
  RTile p;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt_row(i, r), col = rt_col(j);
        p.v[i][j][r] = (row < n && col < n) ? A[row * R + col] : 0.0;
      }
  rt_pad_identity(p, n);
  const bool ok = gj_inverse_regs(p, ws);
  if (!ok && threadIdx.x == 0) status[0] = 1;
  rt_store(p, Dout, NB, NB, NB);
}

// One block step of the sweep; Dk = A_kk^{-1} (NB x NB) comes from the previous
// launch.  The group whose output is diagonal block k + 1 also inverts that
// block into Dnext.
__global__ __launch_bounds__(256) void sweep_kernel(const double* __restrict__ A,
                                                    double* __restrict__ O,
                                                    const double* __restrict__ Dk,
                                                    double* __restrict__ Dnext, int64_t R,
                                                    int64_t kb, int* status) {
  __shared__ double D[NB * LD];
  __shared__ double T1[T1_SIZE];  // A_Ik, then A_Ik D; the pivot inverse's scratch
  const int tid = threadIdx.x, lane = tid & 63, wn = (tid >> 6) & 1;
  const int64_t T = (R + NB - 1) / NB;
  const int64_t nt = T * T;
  // the next pivot's group is dispatched first
  const int64_t first = (kb + 1 < T) ? (kb + 1) * T + kb + 1 : 0;
  const int64_t t = (blockIdx.x + first) % nt;
  const int64_t I = t / T, J = t % T;
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

  if (I == kb + 1 && J == kb + 1) {  // look ahead: invert the next pivot block
    __syncthreads();                 // T1 is free for the inverse's scratch
    rt_pad_identity(out, ni);
    const bool ok = gj_inverse_regs(out, T1);
    if (!ok && tid == 0) status[0] = 1;
    rt_store(out, Dnext, NB, NB, NB);
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
    hipLaunchKernelGGL(sweep_kernel, dim3((unsigned)(T * T)), dim3(256), 0, s, in, out, dk, dn, R,
                       kb, status);
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
