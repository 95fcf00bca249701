// Element-wise, layout and reduction kernels of the CP-PPL sweep.
// Every reduction here is deterministic: fixed grids, fixed-order tree sums,
// no floating-point atomics.
#include "ops.h"

#include "fp8.h"

#include <algorithm>
#include <stdexcept>

namespace cpppl {

namespace {

constexpr int TPB = 256;

inline unsigned blocks_for(int64_t n, int64_t cap = 1 << 20) {
  int64_t b = (n + TPB - 1) / TPB;
  if (b < 1) b = 1;
  return (unsigned)std::min<int64_t>(b, cap);
}

// Fixed-order tree sum over one 256-lane block; result valid in lane 0.
__device__ inline double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

template <typename TO>
__device__ inline void put(void* y, int64_t i, double v) {
  ((TO*)y)[i] = Conv<TO>::from_f64(v);
}
__device__ inline void put_dt(void* y, DType t, int64_t i, double v) {
  if (t == DType::F64) put<double>(y, i, v);
  else if (t == DType::F32) put<float>(y, i, v);
  else put<bf16_t>(y, i, v);
}
__device__ inline double get_dt(const void* x, DType t, int64_t i) {
  if (t == DType::F64) return ((const double*)x)[i];
  if (t == DType::F32) return (double)((const float*)x)[i];
  return (double)bf16_to_f32(((const bf16_t*)x)[i]);
}

__global__ void transpose_kernel(const double* __restrict__ x, void* y, DType yt, int64_t rows,
                                 int64_t cols) {
  __shared__ double tile[32][33];
  const int64_t b = blockIdx.z;
  const double* xb = x + b * rows * cols;
  const int64_t yoff = b * rows * cols;
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  for (int i = threadIdx.y; i < 32; i += 8) {
    const int64_t r = r0 + i, c = c0 + threadIdx.x;
    if (r < rows && c < cols) tile[i][threadIdx.x] = xb[r * cols + c];
  }
  __syncthreads();
  for (int i = threadIdx.y; i < 32; i += 8) {
    const int64_t c = c0 + i, r = r0 + threadIdx.x;
    if (r < rows && c < cols) put_dt(y, yt, yoff + c * rows + r, tile[threadIdx.x][i]);
  }
}

__global__ void permute_pxq_kernel(const double* __restrict__ b, void* out, DType ot, int64_t nx,
                                   int64_t v) {
  const int64_t total = nx * v * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = e % v, x = (e / v) % nx, p = e / (v * nx);
    put_dt(out, ot, e, b[(x * v + p) * v + q]);
  }
}

__global__ void convert_kernel(const double* __restrict__ x, void* y, DType yt, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    put_dt(y, yt, i, x[i]);
}

__global__ void axpy1_kernel(const double* __restrict__ x, double* y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] += x[i];
}

__global__ void kr_kernel(const double* __restrict__ gT, const double* __restrict__ rT, int64_t o,
                          int64_t R, void* Kt, DType kt, const float* __restrict__ ij_scale,
                          const double* __restrict__ r_scale) {
  const int64_t total = R * o * o;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / (o * o), ij = e % (o * o);
    const int64_t i = ij / o, j = ij % o;
    double k = gT[r * o + i] * rT[r * o + j];
    if (ij_scale) k *= (double)ij_scale[ij];
    if (r_scale) k *= r_scale[r];
    put_dt(Kt, kt, e, k);
  }
}

// x[i][j][a][b] <- (x[i][j][a][b] + x[j][i][b][a]) / 2, each pair once.
__global__ void symmetrize_pairs_kernel(double* x, int64_t o, int64_t v) {
  const int64_t n = o * o * v * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ij = e / (v * v), ab = e % (v * v);
    const int64_t i = ij / o, j = ij % o, a = ab / v, b = ab % v;
    const int64_t f = (j * o + i) * v * v + b * v + a;
    if (e < f) {
      const double m = 0.5 * (x[e] + x[f]);
      x[e] = m;
      x[f] = m;
    }
  }
}

// dt[ijab] = (w[ijab] + s (cp[ijab] + cp[jiba]) / 2) / (e_i + e_j - e_a - e_b) - t[ijab]
__global__ void jacobi_delta_kernel(const double* cp, const double* w, const double* e_occ,
                                    const double* e_vir, double s, const double* t, double* dt,
                                    int64_t o, int64_t v) {
  const int64_t n = o * o * v * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ij = e / (v * v), ab = e % (v * v);
    const int64_t i = ij / o, j = ij % o, a = ab / v, b = ab % v;
    const int64_t f = (j * o + i) * v * v + b * v + a;
    const double ladder = 0.5 * (cp[e] + cp[f]);
    const double d = e_occ[i] + e_occ[j] - e_vir[a] - e_vir[b];
    dt[e] = (w[e] + s * ladder) / d - t[e];
  }
}

// One work-group per row: the least power of two 2^e (e in [-126, 127]) with
// max |x| <= 448 * 2^e, i.e. the row scaled by 2^-e fits the e4m3 range.
__global__ __launch_bounds__(TPB) void e4m3_scale_kernel(const double* __restrict__ x, int64_t len,
                                                         float* scale) {
  __shared__ double sh[TPB];
  const double* row = x + blockIdx.x * len;
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += TPB) m = fmax(m, fabs(row[i]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    m = sh[0];
    int e = 0;
    if (m > 0.0) {
      int k;
      frexp(m / 448.0, &k);  // m / 448 in [2^(k-1), 2^k) up to rounding
      e = k < -126 ? -126 : (k > 127 ? 127 : k);
      while (e > -126 && m <= ldexp(448.0, e - 1)) --e;  // exact comparisons
      while (e < 127 && m > ldexp(448.0, e)) ++e;
    }
    scale[blockIdx.x] = ldexpf(1.0f, e);
  }
}

__global__ void quantize_e4m3_kernel(const double* __restrict__ x, uint8_t* q, int64_t n,
                                     const float* __restrict__ scale, int64_t div, int64_t mod,
                                     int64_t grp) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double s = (double)scale[((i / div) % mod) / grp];
    q[i] = e4m3_encode(x[i] / s);
  }
}

__global__ void expand_scales_kernel(const float* __restrict__ sc, float* out, int64_t nx, int64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nx * v;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = sc[i / v];
}

__global__ void dress_tau_kernel(const double* __restrict__ t2, const double* __restrict__ t1,
                                 double* tau, int64_t o, int64_t v) {
  const int64_t n = o * o * v * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ij = e / (v * v), cd = e % (v * v);
    const int64_t i = ij / o, j = ij % o, cc = cd / v, d = cd % v;
    tau[e] = t2[e] + t1[i * v + cc] * t1[j * v + d];
  }
}

__global__ void hadamard_kernel(const double* __restrict__ g1, const double* __restrict__ g2,
                                const double* __restrict__ g3, double* w, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = g1[i] * g2[i];
    if (g3) v *= g3[i];
    w[i] = v;
  }
}

__global__ __launch_bounds__(TPB) void row_normalize_kernel(double* FT, int64_t n, double* lam) {
  __shared__ double sh[TPB];
  const int64_t r = blockIdx.x;
  double* row = FT + r * n;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += TPB) s += row[i] * row[i];
  s = block_sum(s, sh);
  const double nrm = sqrt(s);
  if (threadIdx.x == 0) lam[r] = nrm;
  if (nrm > 0.0) {
    const double inv = 1.0 / nrm;
    for (int64_t i = threadIdx.x; i < n; i += TPB) row[i] *= inv;
  }
}

__global__ __launch_bounds__(TPB) void finish_factor_kernel(const double* __restrict__ part,
                                                             int splits, int64_t R, int64_t n,
                                                             double alpha, double* FT, double* lam,
                                                             void* lowp) {
  __shared__ double sh[TPB];
  const int64_t r = blockIdx.x;
  double* row = FT + r * n;
  const int64_t stride = R * n;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += TPB) {
    double acc = 0.0;
    for (int q = 0; q < splits; ++q) acc += part[q * stride + r * n + i];
    const double v = alpha * acc;
    row[i] = v;
    s += v * v;
  }
  s = block_sum(s, sh);
  const double nrm = sqrt(s);
  if (threadIdx.x == 0) lam[r] = nrm;
  const double inv = nrm > 0.0 ? 1.0 / nrm : 1.0;
  for (int64_t i = threadIdx.x; i < n; i += TPB) {
    const double v = nrm > 0.0 ? row[i] * inv : row[i];
    row[i] = v;
    if (lowp) put_dt(lowp, DType::BF16, r * n + i, v);
  }
}

__global__ void occ_reduce_kernel(const double* __restrict__ HT, const double* __restrict__ other,
                                  double* M, int64_t o, int64_t R, int which) {
  const int64_t total = R * o;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / o, p = e % o;
    const double* h = HT + r * o * o;
    const double* w = other + r * o;
    double acc = 0.0;
    if (which == 0) {
      for (int64_t q = 0; q < o; ++q) acc += h[p * o + q] * w[q];
    } else {
      for (int64_t q = 0; q < o; ++q) acc += h[q * o + p] * w[q];
    }
    M[e] = acc;
  }
}

// rowbuf[r] = lamA[r] * sum_r' lamB[r'] * prod_k X_k[r][r']
__global__ __launch_bounds__(TPB) void weighted_rows_kernel(const double* X0, const double* X1,
                                                            const double* X2, const double* X3,
                                                            const double* lamA, const double* lamB,
                                                            int64_t R, double* rowbuf) {
  __shared__ double sh[TPB];
  const int64_t r = blockIdx.x;
  double s = 0.0;
  for (int64_t c = threadIdx.x; c < R; c += TPB) {
    const int64_t i = r * R + c;
    s += lamB[c] * X0[i] * X1[i] * X2[i] * X3[i];
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) rowbuf[r] = lamA[r] * s;
}

// Row r of the fit terms: rowbuf[r] = lam_r sum_c lam_c (G0 .* G1 .* G2 .* G3)_rc
// (||CP||^2 by Grams) and rowbuf[R + r] = lam_r sum_k MT[r][k] FT[r][k] (<R, CP>
// from the last mode's MTTKRP).
__global__ __launch_bounds__(TPB) void fit_rows_kernel(const double* X0, const double* X1,
                                                       const double* X2, const double* X3,
                                                       const double* lam, const double* MT,
                                                       const double* FT, int64_t n, int64_t R,
                                                       double* rowbuf) {
  __shared__ double sh[TPB];
  const int64_t r = blockIdx.x;
  double s = 0.0;
  for (int64_t c = threadIdx.x; c < R; c += TPB) {
    const int64_t i = r * R + c;
    s += lam[c] * X0[i] * X1[i] * X2[i] * X3[i];
  }
  s = block_sum(s, sh);
  double d = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += TPB) d += MT[r * n + k] * FT[r * n + k];
  d = block_sum(d, sh);
  if (threadIdx.x == 0) {
    rowbuf[r] = lam[r] * s;
    rowbuf[R + r] = lam[r] * d;
  }
}

__global__ __launch_bounds__(TPB) void fit_finish_kernel(int64_t R, const double* rowbuf,
                                                         const double* norm_r2, double* sc) {
  __shared__ double sh[TPB];
  double cp = 0.0, in = 0.0;
  for (int64_t r = threadIdx.x; r < R; r += TPB) {
    cp += rowbuf[r];
    in += rowbuf[R + r];
  }
  cp = block_sum(cp, sh);
  in = block_sum(in, sh);
  if (threadIdx.x == 0) {
    const double n2 = *norm_r2;
    double res2 = n2 - 2.0 * in + cp;
    if (res2 < 0.0) res2 = 0.0;
    sc[0] = in;
    sc[1] = cp;
    sc[2] = res2;
    sc[3] = 1.0 - sqrt(res2) / sqrt(n2);
    sc[4] = 0.5 * res2;
  }
}

// Up to four (src, dst, count) copies of doubles in one launch.
struct CopyList {
  const double* src[5];
  double* dst[5];
  int64_t n[5];
  int count;
};
__global__ __launch_bounds__(TPB) void copy_list_kernel(const CopyList L) {
  for (int q = 0; q < L.count; ++q)
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < L.n[q]; i += (int64_t)gridDim.x * TPB)
      L.dst[q][i] = L.src[q][i];
}

__global__ __launch_bounds__(TPB) void sum_rows_kernel(const double* rowbuf, int64_t R,
                                                       double* out) {
  __shared__ double sh[TPB];
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < R; r += TPB) s += rowbuf[r];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(TPB) void energy_rows_kernel(const void* tau, DType tt,
                                                          const double* aT, const double* bT,
                                                          const double* lam, int64_t v,
                                                          double* rowbuf) {
  __shared__ double sh[TPB];
  const int64_t r = blockIdx.x;
  const double* a = aT + r * v;
  const double* b = bT + r * v;
  const int64_t base = r * v * v;
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < v * v; e += TPB) {
    const int64_t p = e / v, q = e % v;
    s += a[p] * get_dt(tau, tt, base + e) * b[q];
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) rowbuf[r] = lam[r] * s;
}

constexpr int SUM_BLOCKS = 1024;

__global__ __launch_bounds__(TPB) void sumsq_dot_partial_kernel(const double* x, const double* y,
                                                                int64_t rows, int64_t cols,
                                                                int64_t ldx, int64_t ldy,
                                                                double* partial) {
  __shared__ double sh[TPB];
  double s2 = 0.0, sd = 0.0;
  const int64_t n = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n; e += (int64_t)SUM_BLOCKS * TPB) {
    const int64_t i = e / cols, j = e % cols;
    const double xv = x[i * ldx + j];
    s2 += xv * xv;
    sd += xv * y[i * ldy + j];
  }
  s2 = block_sum(s2, sh);
  sd = block_sum(sd, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s2;
    partial[2 * blockIdx.x + 1] = sd;
  }
}

__global__ __launch_bounds__(TPB) void sumsq_dot_final_kernel(const double* partial, double* acc) {
  __shared__ double sh[TPB];
  double s2 = 0.0, sd = 0.0;
  for (int b = threadIdx.x; b < SUM_BLOCKS; b += TPB) {
    s2 += partial[2 * b];
    sd += partial[2 * b + 1];
  }
  s2 = block_sum(s2, sh);
  sd = block_sum(sd, sh);
  if (threadIdx.x == 0) {
    acc[0] += s2;
    acc[1] += sd;
  }
}

__global__ void set_scalar_kernel(double* p, double v) { *p = v; }

__global__ void finish_eta_kernel(double* sc) {
  const double nn = sc[0], np = sc[1], pp = sc[2];
  double d = nn - 2.0 * np + pp;
  if (d < 0.0) d = 0.0;
  sc[3] = sqrt(d) / sqrt(pp);
}

__global__ void nonfinite_kernel(const double* x, int64_t n, int* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) *flag = 1;
}

__global__ void zero_ints_kernel(int* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}
__global__ void zero_doubles_kernel(double* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used counter-based: output
// number c + 1 of the generator seeded with `seed`, mapped to [-1, 1) exactly.
__device__ inline double splitmix_uniform(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1p-52 - 1.0;
}

// FT[r][i] (R x n) = U[-1, 1) draw number offset + i R + r.
__global__ void random_factor_kernel(double* FT, int64_t n, int64_t R, uint64_t seed, uint64_t offset) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * R;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n, i = e % n;
    FT[e] = splitmix_uniform(seed, offset + (uint64_t)(i * R + r));
  }
}

__global__ void fill_doubles_kernel(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void hadamard_scale_cols_kernel(const double* X0, const double* X1, const double* X2,
                                           const double* lamP, double* C, int64_t R, int64_t P) {
  const int64_t total = R * P;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    C[e] = X0[e] * X1[e] * X2[e] * lamP[e % P];
}

__global__ __launch_bounds__(TPB) void aligned_delta_kernel(const double* F1, const double* F0,
                                                            int64_t n, float* y, int64_t ldy) {
  __shared__ double sh[TPB];
  const int64_t r = blockIdx.x;
  double d = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += TPB) d += F1[r * n + i] * F0[r * n + i];
  d = block_sum(d, sh);
  const double sg = d < 0.0 ? -1.0 : 1.0;
  for (int64_t i = threadIdx.x; i < n; i += TPB)
    y[r * ldy + i] = (float)(sg * F1[r * n + i] - F0[r * n + i]);
}

__global__ void pack_rows_kernel(const double* x, const double* scale_inv, int64_t R, int64_t n,
                                 float* y, int64_t ldy, int64_t off) {
  const int64_t total = R * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n, i = e % n;
    double v = x[e];
    if (scale_inv) v *= scale_inv[r];
    y[r * ldy + off + i] = (float)v;
  }
}

__global__ void add_rows_kernel(const float* y, int64_t ldy, int64_t off, int64_t R, int64_t n,
                                double* x) {
  const int64_t total = R * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n, i = e % n;
    x[e] += (double)y[r * ldy + off + i];
  }
}

}  // namespace

void transpose_batched(const double* x, void* y, DType yt, int64_t batch, int64_t rows,
                       int64_t cols, hipStream_t s) {
  if (batch <= 0 || rows <= 0 || cols <= 0) return;
  dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32), (unsigned)batch);
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(32, 8), 0, s, x, y, yt, rows, cols);
  CPPPL_LAUNCH_CHECK("transpose");
}

void permute_pxq(const double* b, void* out, DType ot, int64_t nx, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(permute_pxq_kernel, dim3(blocks_for(nx * v * v)), dim3(TPB), 0, s, b, out, ot,
                     nx, v);
  CPPPL_LAUNCH_CHECK("permute_pxq");
}

void convert(const double* x, void* y, DType yt, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(convert_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, x, y, yt, n);
  CPPPL_LAUNCH_CHECK("convert");
}

void axpy1(const double* x, double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(axpy1_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, x, y, n);
  CPPPL_LAUNCH_CHECK("axpy1");
}

void khatri_rao_t(const double* gT, const double* rT, int64_t o, int64_t R, void* Kt, DType kt,
                  hipStream_t s, const float* ij_scale, const double* r_scale) {
  hipLaunchKernelGGL(kr_kernel, dim3(blocks_for(R * o * o)), dim3(TPB), 0, s, gT, rT, o, R, Kt, kt,
                     ij_scale, r_scale);
  CPPPL_LAUNCH_CHECK("khatri_rao");
}

void e4m3_row_scales(const double* x, int64_t rows, int64_t len, float* scale, hipStream_t s) {
  if (rows <= 0) return;
  if (rows > 0x7fffffffLL) throw std::invalid_argument("e4m3_row_scales: too many rows");
  hipLaunchKernelGGL(e4m3_scale_kernel, dim3((unsigned)rows), dim3(TPB), 0, s, x, len, scale);
  CPPPL_LAUNCH_CHECK("e4m3_row_scales");
}

void quantize_e4m3(const double* x, uint8_t* q, int64_t n, const float* scale, int64_t div,
                   int64_t mod, int64_t grp, hipStream_t s) {
  if (n <= 0) return;
  if (div <= 0 || mod <= 0 || grp <= 0) throw std::invalid_argument("quantize_e4m3: bad scale map");
  hipLaunchKernelGGL(quantize_e4m3_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, x, q, n, scale, div,
                     mod, grp);
  CPPPL_LAUNCH_CHECK("quantize_e4m3");
}

void expand_scales(const float* scale, float* out, int64_t nx, int64_t v, hipStream_t s) {
  if (nx * v <= 0) return;
  hipLaunchKernelGGL(expand_scales_kernel, dim3(blocks_for(nx * v)), dim3(TPB), 0, s, scale, out, nx, v);
  CPPPL_LAUNCH_CHECK("expand_scales");
}

void symmetrize_pairs(double* x, int64_t o, int64_t v, hipStream_t s) {
  const int64_t n = o * o * v * v;
  if (n <= 0) return;
  hipLaunchKernelGGL(symmetrize_pairs_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, x, o, v);
  CPPPL_LAUNCH_CHECK("symmetrize_pairs");
}

void jacobi_delta(const double* cp, const double* w, const double* e_occ, const double* e_vir,
                  double scale, const double* t, double* dt, int64_t o, int64_t v, hipStream_t s) {
  const int64_t n = o * o * v * v;
  if (n <= 0) return;
  hipLaunchKernelGGL(jacobi_delta_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, cp, w, e_occ, e_vir,
                     scale, t, dt, o, v);
  CPPPL_LAUNCH_CHECK("jacobi_delta");
}

void dress_tau(const double* t2, const double* t1, double* tau, int64_t o, int64_t v, hipStream_t s) {
  const int64_t n = o * o * v * v;
  if (n <= 0) return;
  hipLaunchKernelGGL(dress_tau_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, t2, t1, tau, o, v);
  CPPPL_LAUNCH_CHECK("dress_tau");
}

void hadamard(const double* g1, const double* g2, const double* g3, double* w, int64_t n,
              hipStream_t s) {
  hipLaunchKernelGGL(hadamard_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, g1, g2, g3, w, n);
  CPPPL_LAUNCH_CHECK("hadamard");
}

void row_normalize(double* FT, int64_t R, int64_t n, double* lam, hipStream_t s) {
  hipLaunchKernelGGL(row_normalize_kernel, dim3((unsigned)R), dim3(TPB), 0, s, FT, n, lam);
  CPPPL_LAUNCH_CHECK("row_normalize");
}

void finish_factor(const double* part, int splits, int64_t R, int64_t n, double alpha, double* FT,
                   double* lam, void* lowp, hipStream_t s) {
  if (R <= 0 || n <= 0) return;
  hipLaunchKernelGGL(finish_factor_kernel, dim3((unsigned)R), dim3(TPB), 0, s, part, splits, R, n,
                     alpha, FT, lam, lowp);
  CPPPL_LAUNCH_CHECK("finish_factor");
}

void occ_reduce(const double* HT, const double* other, double* M, int64_t o, int64_t R, int which,
                hipStream_t s) {
  hipLaunchKernelGGL(occ_reduce_kernel, dim3(blocks_for(R * o)), dim3(TPB), 0, s, HT, other, M, o,
                     R, which);
  CPPPL_LAUNCH_CHECK("occ_reduce");
}

void fit_scalars(const double* MT, const double* FT, int64_t n, const double* lam,
                 const double* const G[4], int64_t R, const double* norm_r2, double* rowbuf,
                 double* sc, hipStream_t s) {
  hipLaunchKernelGGL(fit_rows_kernel, dim3((unsigned)R), dim3(TPB), 0, s, G[0], G[1], G[2], G[3],
                     lam, MT, FT, n, R, rowbuf);
  CPPPL_LAUNCH_CHECK("fit_rows");
  hipLaunchKernelGGL(fit_finish_kernel, dim3(1), dim3(TPB), 0, s, R, rowbuf, norm_r2, sc);
  CPPPL_LAUNCH_CHECK("fit_finish");
}

void copy_doubles(const double* const* src, double* const* dst, const int64_t* n, int count,
                  hipStream_t s) {
  if (count < 1 || count > 5) throw std::invalid_argument("copy_doubles: 1..5 copies");
  CopyList L{};
  int64_t mx = 0;
  for (int q = 0; q < count; ++q) {
    L.src[q] = src[q];
    L.dst[q] = dst[q];
    L.n[q] = n[q];
    mx = std::max(mx, n[q]);
  }
  L.count = count;
  const int64_t blocks = std::min<int64_t>(std::max<int64_t>(1, (mx + TPB - 1) / TPB), 1024);
  hipLaunchKernelGGL(copy_list_kernel, dim3((unsigned)blocks), dim3(TPB), 0, s, L);
  CPPPL_LAUNCH_CHECK("copy_list");
}

void weighted_hadamard_sum(const double* const X[4], const double* lamA, const double* lamB,
                           int64_t R, double* rowbuf, double* out, hipStream_t s) {
  hipLaunchKernelGGL(weighted_rows_kernel, dim3((unsigned)R), dim3(TPB), 0, s, X[0], X[1], X[2],
                     X[3], lamA, lamB, R, rowbuf);
  CPPPL_LAUNCH_CHECK("weighted_rows");
  hipLaunchKernelGGL(sum_rows_kernel, dim3(1), dim3(TPB), 0, s, rowbuf, R, out);
  CPPPL_LAUNCH_CHECK("sum_rows");
}

void energy_from_tau(const void* tau, DType tt, const double* aT, const double* bT,
                     const double* lam, int64_t R, int64_t v, double* rowbuf, double* out,
                     hipStream_t s) {
  hipLaunchKernelGGL(energy_rows_kernel, dim3((unsigned)R), dim3(TPB), 0, s, tau, tt, aT, bT, lam,
                     v, rowbuf);
  CPPPL_LAUNCH_CHECK("energy_rows");
  hipLaunchKernelGGL(sum_rows_kernel, dim3(1), dim3(TPB), 0, s, rowbuf, R, out);
  CPPPL_LAUNCH_CHECK("energy_sum");
}

void sumsq_dot_accumulate(const double* x, const double* y, int64_t rows, int64_t cols,
                          int64_t ldx, int64_t ldy, double* partial, double* acc, hipStream_t s) {
  hipLaunchKernelGGL(sumsq_dot_partial_kernel, dim3(SUM_BLOCKS), dim3(TPB), 0, s, x, y, rows, cols,
                     ldx, ldy, partial);
  CPPPL_LAUNCH_CHECK("sumsq_dot_partial");
  hipLaunchKernelGGL(sumsq_dot_final_kernel, dim3(1), dim3(TPB), 0, s, partial, acc);
  CPPPL_LAUNCH_CHECK("sumsq_dot_final");
}

void set_scalar(double* p, double v, hipStream_t s) {
  hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, s, p, v);
  CPPPL_LAUNCH_CHECK("set_scalar");
}

void finish_eta(double* sc_eta, hipStream_t s) {
  hipLaunchKernelGGL(finish_eta_kernel, dim3(1), dim3(1), 0, s, sc_eta);
  CPPPL_LAUNCH_CHECK("finish_eta");
}

void nonfinite_check(const double* x, int64_t n, int* flag, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(nonfinite_kernel, dim3(blocks_for(n, 4096)), dim3(TPB), 0, s, x, n, flag);
  CPPPL_LAUNCH_CHECK("nonfinite");
}

void zero_ints(int* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zero_ints_kernel, dim3(blocks_for(n, 4096)), dim3(TPB), 0, s, p, n);
  CPPPL_LAUNCH_CHECK("zero_ints");
}

void zero_doubles(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zero_doubles_kernel, dim3(blocks_for(n, 4096)), dim3(TPB), 0, s, p, n);
  CPPPL_LAUNCH_CHECK("zero_doubles");
}

void random_factor(double* FT, int64_t n, int64_t R, uint64_t seed, uint64_t offset, hipStream_t s) {
  if (n * R <= 0) return;
  hipLaunchKernelGGL(random_factor_kernel, dim3(blocks_for(n * R)), dim3(TPB), 0, s, FT, n, R, seed, offset);
  CPPPL_LAUNCH_CHECK("random_factor");
}

void fill_doubles(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_doubles_kernel, dim3(blocks_for(n, 4096)), dim3(TPB), 0, s, p, n, v);
  CPPPL_LAUNCH_CHECK("fill_doubles");
}

void hadamard_scale_cols(const double* X0, const double* X1, const double* X2, const double* lamP,
                         double* C, int64_t R, int64_t P, hipStream_t s) {
  hipLaunchKernelGGL(hadamard_scale_cols_kernel, dim3(blocks_for(R * P)), dim3(TPB), 0, s, X0, X1,
                     X2, lamP, C, R, P);
  CPPPL_LAUNCH_CHECK("hadamard_scale_cols");
}

void aligned_delta_f32(const double* F1, const double* F0, int64_t R, int64_t n, float* y,
                       int64_t ldy, hipStream_t s) {
  hipLaunchKernelGGL(aligned_delta_kernel, dim3((unsigned)R), dim3(TPB), 0, s, F1, F0, n, y, ldy);
  CPPPL_LAUNCH_CHECK("aligned_delta");
}

void pack_rows_f32(const double* x, const double* scale_inv, int64_t R, int64_t n, float* y,
                   int64_t ldy, int64_t off, hipStream_t s) {
  hipLaunchKernelGGL(pack_rows_kernel, dim3(blocks_for(R * n)), dim3(TPB), 0, s, x, scale_inv, R,
                     n, y, ldy, off);
  CPPPL_LAUNCH_CHECK("pack_rows");
}

void add_rows_from_f32(const float* y, int64_t ldy, int64_t off, int64_t R, int64_t n, double* x,
                       hipStream_t s) {
  hipLaunchKernelGGL(add_rows_kernel, dim3(blocks_for(R * n)), dim3(TPB), 0, s, y, ldy, off, R, n,
                     x);
  CPPPL_LAUNCH_CHECK("add_rows");
}

}  // namespace cpppl
