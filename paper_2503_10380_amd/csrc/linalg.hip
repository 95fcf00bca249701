// Block sweep-operator inverse of the ALS normal-equation matrix, FP64.
//
// Sweeping pivot block k of a symmetric matrix A (D = A_kk^{-1}):
//   A_ij <- A_ij - A_ik D A_kj   (i, j != k)
//   A_ik <- A_ik D,  A_kj <- D A_kj,  A_kk <- -D
// After every block has been swept once, A holds -A^{-1}.  One launch per
// block step; work-group (I, J) re-inverts the 64 x 64 pivot block in LDS
// (Gauss-Jordan, no pivoting: the pivots of an SPD matrix are positive) and
// then writes output tile (I, J) from the input buffer into the other buffer.
// The 64 x 64 products use 4 x 4 register micro-tiles per lane.
#include "linalg.h"

#include <utility>

namespace cpppl {

namespace {

constexpr int NB = INV_NB;
constexpr int LD = NB + 1;

// In-place Gauss-Jordan inverse of the NB x NB block P (row stride LD) in LDS.
// Lane t keeps the 4 x 4 block (rows 4 (t / 16) + r, columns 4 (t % 16) + c) in
// registers; at pivot k the owners of row k and column k publish them through
// LDS vectors that alternate between two buffers, so one barrier per pivot
// suffices.
__device__ bool gj_inverse(double* P, double (*sr)[NB], double (*sc)[NB]) {
  const int tid = threadIdx.x;
  const int i0 = 4 * (tid >> 4), j0 = 4 * (tid & 15);
  double a[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) a[r][c] = P[(i0 + r) * LD + j0 + c];
  bool ok = true;
  for (int k = 0; k < NB; ++k) {
    const int b = k & 1;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (i0 + r == k) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sr[b][j0 + c] = a[r][c];
      }
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (j0 + c == k) {
#pragma unroll
        for (int r = 0; r < 4; ++r) sc[b][i0 + r] = a[r][c];
      }
    __syncthreads();
    double p = sr[b][k];
    const bool bad = !(p > 0.0) || !isfinite(p);
    ok = ok && !bad;
    if (bad) p = 1.0;
    const double inv = 1.0 / p;
    double rowk[4], colk[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) rowk[c] = sr[b][j0 + c] * inv;
#pragma unroll
    for (int r = 0; r < 4; ++r) colk[r] = sc[b][i0 + r];
    // branch-free update: every lane computes all four cases and selects
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool ri = (i0 + r == k);
      const double colv = -colk[r] * inv;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const bool cj = (j0 + c == k);
        const double gen = a[r][c] - colk[r] * rowk[c];
        const double on_row = cj ? inv : rowk[c];
        const double off_row = cj ? colv : gen;
        a[r][c] = ri ? on_row : off_row;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) P[(i0 + r) * LD + j0 + c] = a[r][c];
  __syncthreads();
  return ok;
}

// acc += X[rows of this lane][:] . Y[:][cols of this lane]; lane t owns rows
// 4 (t / 16) + r and columns (t % 16) + 16 c.
__device__ inline void mm64(const double* X, const double* Y, double acc[4][4]) {
  const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
  for (int l = 0; l < NB; ++l) {
    double a[4], b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = X[(4 * ti + r) * LD + l];
#pragma unroll
    for (int c = 0; c < 4; ++c) b[c] = Y[l * LD + tj + 16 * c];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
  }
}

__device__ inline void load_tile(const double* A, int64_t R, int64_t r0, int64_t c0, int nr,
                                 int nc, double* T) {
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
    const int i = e / NB, j = e % NB;
    T[i * LD + j] = (i < nr && j < nc) ? A[(r0 + i) * R + c0 + j] : 0.0;
  }
}

__global__ __launch_bounds__(256) void sweep_kernel(const double* __restrict__ A,
                                                    double* __restrict__ O, int64_t R, int64_t kb,
                                                    int* status) {
  __shared__ double D[NB * LD];
  __shared__ double T1[NB * LD];
  __shared__ double T2[NB * LD];
  __shared__ double sr[2][NB], sc[2][NB];
  const int tid = threadIdx.x;
  const int64_t T = (R + NB - 1) / NB;
  const int64_t I = blockIdx.x / T, J = blockIdx.x % T;
  const int64_t k0 = kb * NB, i0 = I * NB, j0 = J * NB;
  const int nk = (int)min((int64_t)NB, R - k0);
  const int ni = (int)min((int64_t)NB, R - i0);
  const int nj = (int)min((int64_t)NB, R - j0);

  // pivot block, padded with the identity
  for (int e = tid; e < NB * NB; e += blockDim.x) {
    const int i = e / NB, j = e % NB;
    D[i * LD + j] = (i < nk && j < nk) ? A[(k0 + i) * R + k0 + j] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  const bool ok = gj_inverse(D, sr, sc);
  if (!ok && blockIdx.x == 0 && tid == 0) status[0] = 1;

  const int ti = tid >> 4, tj = tid & 15;
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;

  if (I == kb && J == kb) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] = -D[(4 * ti + r) * LD + tj + 16 * c];
  } else if (J == kb) {  // A_Ik D
    load_tile(A, R, i0, k0, ni, nk, T1);
    __syncthreads();
    mm64(T1, D, acc);
  } else if (I == kb) {  // D A_kJ
    load_tile(A, R, k0, j0, nk, nj, T2);
    __syncthreads();
    mm64(D, T2, acc);
  } else {  // A_IJ - (A_Ik D) A_kJ
    load_tile(A, R, i0, k0, ni, nk, T1);
    load_tile(A, R, k0, j0, nk, nj, T2);
    __syncthreads();
    mm64(T1, D, acc);
    __syncthreads();  // every lane has read T1 before it is overwritten with C
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) T1[(4 * ti + r) * LD + tj + 16 * c] = acc[r][c];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
    mm64(T1, T2, acc);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int i = 4 * ti + r, j = tj + 16 * c;
        if (i < ni && j < nj) acc[r][c] = A[(i0 + i) * R + j0 + j] - acc[r][c];
      }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = 4 * ti + r, j = tj + 16 * c;
      if (i < ni && j < nj) O[(i0 + i) * R + j0 + j] = acc[r][c];
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
