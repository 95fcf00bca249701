// Blocked right-looking Cholesky and the two triangular solves of the ALS
// normal equations, FP64.
//
// Per 64-wide block column: one kernel factors the diagonal block in LDS
// (every work-group redundantly, so no inter-group wait is needed) and the
// work-groups then solve the panel rows below it, one row per lane, against
// the factored block; the trailing update is an FP64 matrix-core GEMM.  The
// solves walk block rows the same way: a small kernel solves one block row
// (one right-hand-side column per lane) and a GEMM updates the rest.
// Partial blocks are padded with the identity.
#include "linalg.h"

#include "gemm.h"

namespace cpppl {

namespace {

constexpr int NB = CHOL_NB;

// Loads the (padded) diagonal block at k0 into D and factors it in place.
// Returns false (block-uniformly) if a pivot was bad.
__device__ inline bool factor_diag(const double* A, int64_t R, int64_t k0, int nb,
                                   double (*D)[NB + 1]) {
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * NB; e += blockDim.x) {
    const int i = e / NB, j = e % NB;
    double v;
    if (i < nb && j < nb) v = (j <= i) ? A[(k0 + i) * R + k0 + j] : 0.0;
    else v = (i == j) ? 1.0 : 0.0;
    D[i][j] = v;
  }
  __syncthreads();
  bool ok = true;
  for (int j = 0; j < NB; ++j) {
    const double d = D[j][j];
    const bool bad = !(d > 0.0) || !isfinite(d);
    ok = ok && !bad;
    const double sd = bad ? 1.0 : sqrt(d);
    __syncthreads();
    if (tid == 0) D[j][j] = sd;
    const double inv = 1.0 / sd;
    for (int i = j + 1 + tid; i < NB; i += blockDim.x) D[i][j] *= inv;
    __syncthreads();
    const int m = NB - j - 1;
    for (int e = tid; e < m * m; e += blockDim.x) {
      const int i = j + 1 + e / m, l = j + 1 + e % m;
      if (l <= i) D[i][l] -= D[i][j] * D[l][j];
    }
    __syncthreads();
  }
  return ok;
}

// Block 0 saves the factored (padded) diagonal block to Dsave; blocks b >= 1
// solve panel rows k0 + nb + (b-1)*SUB + lane:  x L_kk^T = a.  The diagonal
// block of A is only read here, so no block waits on another.  Each lane keeps
// its row in its own LDS column Xs[.][lane] (conflict-free, no spills).
constexpr int SUB = 128;

__global__ __launch_bounds__(SUB) void chol_panel_kernel(double* A, int64_t R, int64_t k0,
                                                         double* Dsave, int* status) {
  __shared__ double D[NB][NB + 1];
  __shared__ double Xs[NB][SUB];
  const int nb = (int)min((int64_t)NB, R - k0);
  const bool ok = factor_diag(A, R, k0, nb, D);
  const int tid = threadIdx.x;
  if (blockIdx.x == 0) {
    if (!ok && tid == 0) status[0] = 1;
    double* out = Dsave + (k0 / NB) * NB * NB;
    for (int e = tid; e < NB * NB; e += blockDim.x) out[e] = D[e / NB][e % NB];
    return;
  }
  const int64_t row = k0 + nb + (int64_t)(blockIdx.x - 1) * SUB + tid;
  if (row >= R) return;
  double* a = A + row * R + k0;
  for (int j = 0; j < NB; ++j) Xs[j][tid] = (j < nb) ? a[j] : 0.0;
  for (int j = 0; j < nb; ++j) {
    const double xj = Xs[j][tid] / D[j][j];
    Xs[j][tid] = xj;
    for (int l = j + 1; l < nb; ++l) Xs[l][tid] -= xj * D[l][j];
  }
  for (int j = 0; j < nb; ++j) a[j] = Xs[j][tid];
}

// Forward (lower) or backward (transposed lower) substitution on block row k0
// of X (R x n), one right-hand-side column per lane, kept in Xs[.][lane].
template <bool FORWARD>
__global__ __launch_bounds__(SUB) void trsm_diag_kernel(const double* Dsave, int64_t R, int64_t k0,
                                                        double* X, int64_t n) {
  __shared__ double D[NB][NB + 1];
  __shared__ double Xs[NB][SUB];
  const int nb = (int)min((int64_t)NB, R - k0);
  const double* src = Dsave + (k0 / NB) * NB * NB;
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) D[e / NB][e % NB] = src[e];
  __syncthreads();
  const int tid = threadIdx.x;
  const int64_t c = (int64_t)blockIdx.x * SUB + tid;
  if (c >= n) return;
  for (int i = 0; i < nb; ++i) Xs[i][tid] = X[(k0 + i) * n + c];
  if (FORWARD) {
    for (int j = 0; j < nb; ++j) {
      const double xj = Xs[j][tid] / D[j][j];
      Xs[j][tid] = xj;
      for (int i = j + 1; i < nb; ++i) Xs[i][tid] -= D[i][j] * xj;
    }
  } else {
    for (int j = nb - 1; j >= 0; --j) {
      const double xj = Xs[j][tid] / D[j][j];
      Xs[j][tid] = xj;
      for (int i = 0; i < j; ++i) Xs[i][tid] -= D[j][i] * xj;
    }
  }
  for (int i = 0; i < nb; ++i) X[(k0 + i) * n + c] = Xs[i][tid];
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

int64_t diag_save_elems(int64_t R) { return ((R + NB - 1) / NB) * NB * NB; }

void cholesky(double* A, int64_t R, double* Dsave, int* status, hipStream_t s) {
  for (int64_t k0 = 0; k0 < R; k0 += NB) {
    const int64_t nb = std::min<int64_t>(NB, R - k0);
    const int64_t below = R - k0 - nb;
    const unsigned blocks = 1 + (unsigned)((below + SUB - 1) / SUB);
    hipLaunchKernelGGL(chol_panel_kernel, dim3(blocks), dim3(SUB), 0, s, A, R, k0, Dsave, status);
    CPPPL_LAUNCH_CHECK("chol_panel");
    if (below > 0) {
      // A22 -= L21 L21^T  (full square; only the lower part is used later)
      Gemm g;
      g.M = below; g.N = below; g.K = nb;
      g.A = A + (k0 + nb) * R + k0; g.sam = R; g.sak = 1;
      g.B = A + (k0 + nb) * R + k0; g.sbn = R; g.sbk = 1;
      g.C = A + (k0 + nb) * R + k0 + nb; g.scm = R;
      g.ctype = DType::F64; g.alpha = -1.0; g.beta = 1.0;
      gemm_f64(g, s);
    }
  }
}

void spd_solve(const double* L, const double* Dsave, int64_t R, double* X, int64_t n,
               hipStream_t s) {
  const unsigned cb = (unsigned)((n + SUB - 1) / SUB);
  for (int64_t k0 = 0; k0 < R; k0 += NB) {
    const int64_t nb = std::min<int64_t>(NB, R - k0);
    hipLaunchKernelGGL(trsm_diag_kernel<true>, dim3(cb), dim3(SUB), 0, s, Dsave, R, k0, X, n);
    CPPPL_LAUNCH_CHECK("trsm_fwd");
    const int64_t below = R - k0 - nb;
    if (below > 0) {
      Gemm g;  // X[k0+nb:, :] -= L[k0+nb:, k0:k0+nb] X[k0:k0+nb, :]
      g.M = below; g.N = n; g.K = nb;
      g.A = L + (k0 + nb) * R + k0; g.sam = R; g.sak = 1;
      g.B = X + k0 * n; g.sbk = n; g.sbn = 1;
      g.C = X + (k0 + nb) * n; g.scm = n;
      g.ctype = DType::F64; g.alpha = -1.0; g.beta = 1.0;
      gemm_f64(g, s);
    }
  }
  const int64_t nblk = (R + NB - 1) / NB;
  for (int64_t kb = nblk - 1; kb >= 0; --kb) {
    const int64_t k0 = kb * NB;
    const int64_t nb = std::min<int64_t>(NB, R - k0);
    hipLaunchKernelGGL(trsm_diag_kernel<false>, dim3(cb), dim3(SUB), 0, s, Dsave, R, k0, X, n);
    CPPPL_LAUNCH_CHECK("trsm_bwd");
    if (k0 > 0) {
      Gemm g;  // X[:k0, :] -= L[k0:k0+nb, :k0]^T X[k0:k0+nb, :]
      g.M = k0; g.N = n; g.K = nb;
      g.A = L + k0 * R; g.sam = 1; g.sak = R;
      g.B = X + k0 * n; g.sbk = n; g.sbn = 1;
      g.C = X; g.scm = n;
      g.ctype = DType::F64; g.alpha = -1.0; g.beta = 1.0;
      gemm_f64(g, s);
    }
  }
}

void add_ridge(double* A, int64_t R, double delta, hipStream_t s) {
  hipLaunchKernelGGL(ridge_kernel, dim3(1), dim3(256), 0, s, A, R, delta);
  CPPPL_LAUNCH_CHECK("ridge");
}

}  // namespace cpppl
