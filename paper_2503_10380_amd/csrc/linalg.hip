// Block sweep-operator inverse of the ALS normal-equation matrix, FP64.
//
// Sweeping pivot block k of a symmetric matrix A (D = A_kk^{-1}):
//   A_ij <- A_ij - A_ik D A_kj   (i, j != k)
//   A_ik <- A_ik D,  A_kj <- D A_kj,  A_kk <- -D
// After every block has been swept once, A holds -A^{-1}.  One launch per
// block step; work-group (I, J) re-inverts the 64 x 64 pivot block in LDS
// (blocked Gauss-Jordan, no pivoting: the pivots of an SPD matrix are
// positive) and then writes output tile (I, J) from the input buffer into the
// other buffer.  The 64 x 64 products use 4 x 4 register micro-tiles per lane.
#include "linalg.h"

#include <utility>

namespace cpppl {

namespace {

constexpr int NB = INV_NB;
constexpr int LD = NB + 1;

constexpr int PW = 16;  // panel width of the blocked Gauss-Jordan inverse

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

// In-wave Gauss-Jordan inverse of a 16 x 16 block held 4 elements per lane:
// lane l holds row l / 4, columns 4 (l % 4) + c.  Pivot rows and columns move
// between lanes by shuffles, so no barrier is involved.
__device__ __forceinline__ bool gj16_wave(double (&g)[4]) {
  const int lane = threadIdx.x & 63;
  const int i = lane >> 2;
  bool ok = true;
#pragma unroll
  for (int k = 0; k < PW; ++k) {
    const int kc = k & 3, kl = k >> 2;
    double p = __shfl(g[kc], 4 * k + kl);
    const bool bad = !(p > 0.0) || !isfinite(p);
    ok = ok && !bad;
    if (bad) p = 1.0;
    const double inv = 1.0 / p;
    double rk[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) rk[c] = __shfl(g[c], 4 * k + (lane & 3)) * inv;
    const double ck = __shfl(g[kc], 4 * i + kl);
    const double colv = -ck * inv;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = 4 * (lane & 3) + c;
      const double gen = g[c] - ck * rk[c];
      const double on_row = (j == k) ? inv : rk[c];
      const double off_row = (j == k) ? colv : gen;
      g[c] = (i == k) ? on_row : off_row;
    }
  }
  return ok;
}

// P <- P^{-1} for the NB x NB SPD tile P held in registers (RTile layout), by
// four 16-wide block sweeps: per panel, the pivot rows and columns are
// published in LDS, wave 0 inverts the 16 x 16 pivot block with shuffles, and
// the rank-16 update runs on the matrix cores.  `ws` is LDS scratch of at
// least 2 * 16 * LD + 2 * NB * 17 + 16 * 17 doubles.  Returns false if a pivot
// was not positive.
__device__ bool gj_inverse_regs(RTile& P, double* ws) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double* Rp = ws;                   // pivot rows    (16 x LD)
  double* DR = ws + PW * LD;         // D . pivot rows (16 x LD)
  double* Pc = ws + 2 * PW * LD;     // pivot columns (NB x 17)
  double* Cp = Pc + NB * 17;         // pivot columns . D (NB x 17)
  double* Dp = Cp + NB * 17;         // D (16 x 17)
  bool ok = true;
  for (int q0 = 0; q0 < NB; q0 += PW) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rt_row(i, r), col = rt_col(j);
          const double v = P.v[i][j][r];
          if (row >= q0 && row < q0 + PW) Rp[(row - q0) * LD + col] = v;
          if (col >= q0 && col < q0 + PW) Pc[row * 17 + (col - q0)] = v;
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
    for (int e = tid; e < NB * PW; e += blockDim.x) {  // Cp = Pc D
      const int i = e / PW, j = e % PW;
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < PW; ++l) s += Pc[i * 17 + l] * Dp[l * 17 + j];
      Cp[i * 17 + j] = s;
    }
    for (int e = tid; e < PW * NB; e += blockDim.x) {  // DR = D Rp
      const int i = e / NB, j = e % NB;
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < PW; ++l) s += Dp[i * 17 + l] * Rp[l * LD + j];
      DR[i * LD + j] = s;
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
          else if (ip) P.v[i][j][r] = DR[(row - q0) * LD + col];
          else if (jp) P.v[i][j][r] = Cp[row * 17 + (col - q0)];
        }
    __syncthreads();
  }
  // the sweeps leave -P^{-1}
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) P.v[i][j] = -P.v[i][j];
  return ok;
}

__device__ __forceinline__ void rt_zero(RTile& t) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) t.v[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
}
__device__ __forceinline__ void rt_to_lds(const RTile& t, double* S, double scale) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) S[rt_row(i, r) * LD + rt_col(j)] = scale * t.v[i][j][r];
}

// One block step of the sweep.  Work-group (I, J) writes output tile (I, J).
__global__ __launch_bounds__(256) void sweep_kernel(const double* __restrict__ A,
                                                    double* __restrict__ O, int64_t R, int64_t kb,
                                                    int* status) {
  __shared__ double D[NB * LD];
  __shared__ double T12[2 * NB * LD];  // T1 | T2; also the inverse's scratch
  double* T1 = T12;
  double* T2 = T12 + NB * LD;
  static_assert(2 * PW * LD + 2 * NB * 17 + PW * 17 <= 2 * NB * LD, "scratch fits in T1|T2");
  const int tid = threadIdx.x;
  const int64_t T = (R + NB - 1) / NB;
  const int64_t I = blockIdx.x / T, J = blockIdx.x % T;
  const int64_t k0 = kb * NB, i0 = I * NB, j0 = J * NB;
  const int nk = (int)min((int64_t)NB, R - k0);
  const int ni = (int)min((int64_t)NB, R - i0);
  const int nj = (int)min((int64_t)NB, R - j0);
  const bool need1 = (J == kb && I != kb) || (I != kb && J != kb);  // A_Ik
  const bool need2 = (I == kb && J != kb) || (I != kb && J != kb);  // A_kJ
  const bool general = I != kb && J != kb;

  // global reads of this tile's operands go out before the pivot inverse
  constexpr int PER = NB * NB / 256;
  double r1[PER], r2[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + q * 256, i = e / NB, j = e % NB;
    r1[q] = (need1 && i < ni && j < nk) ? A[(i0 + i) * R + k0 + j] : 0.0;
    r2[q] = (need2 && i < nk && j < nj) ? A[(k0 + i) * R + j0 + j] : 0.0;
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
  // pivot block (identity-padded) straight into registers, inverted there
  RTile piv;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt_row(i, r), col = rt_col(j);
        piv.v[i][j][r] = (row < nk && col < nk) ? A[(k0 + row) * R + k0 + col]
                                                : (row == col ? 1.0 : 0.0);
      }
  const bool ok = gj_inverse_regs(piv, T12);  // T1|T2 serve as scratch until the operands land
  if (!ok && blockIdx.x == 0 && tid == 0) status[0] = 1;
  rt_to_lds(piv, D, 1.0);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + q * 256, i = e / NB, j = e % NB;
    T1[i * LD + j] = r1[q];
    T2[i * LD + j] = r2[q];
  }
  __syncthreads();

  RTile out;
  if (I == kb && J == kb) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) out.v[i][j] = -piv.v[i][j];
  } else if (J == kb) {  // A_Ik D
    rt_zero(out);
    mfma_mm<NB, false>(T1, LD, D, LD, out);
  } else if (I == kb) {  // D A_kJ
    rt_zero(out);
    mfma_mm<NB, false>(D, LD, T2, LD, out);
  } else {  // A_IJ - (A_Ik D) A_kJ
    RTile c;
    rt_zero(c);
    mfma_mm<NB, false>(T1, LD, D, LD, c);
    __syncthreads();  // every lane has read T1 before it is overwritten with C
    rt_to_lds(c, T1, 1.0);
    __syncthreads();
    out = acc;
    mfma_mm<NB, true>(T1, LD, T2, LD, out);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt_row(i, r), col = rt_col(j);
        if (row < ni && col < nj) O[(i0 + row) * R + j0 + col] = out.v[i][j][r];
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

double* spd_inverse_neg(double* bufA, double* bufB, int64_t R, int* status, hipStream_t s) {
  const int64_t T = (R + NB - 1) / NB;
  double* in = bufA;
  double* out = bufB;
  for (int64_t kb = 0; kb < T; ++kb) {
    hipLaunchKernelGGL(sweep_kernel, dim3((unsigned)(T * T)), dim3(256), 0, s, in, out, R, kb,
                       status);
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
