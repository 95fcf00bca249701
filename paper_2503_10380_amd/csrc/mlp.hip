// Warm-start network: a ReLU multi-layer perceptron applied to every rank
// column independently, FP32, with hand-written forward / backward / Adam
// kernels (the layer products on the FP32 matrix cores).
// y = h_{L-1} W_L^T + b_L, h_l = relu(h_{l-1} W_l^T + b_l), loss =
// mean (y - target)^2, Adam (Kingma & Ba, arXiv:1412.6980, Algorithm 1).
// Weights start U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from a counter-based
// SplitMix64 stream (Steele, Lea & Flood, OOPSLA 2014); the last layer starts
// at zero, so an untrained network predicts no correction.
#include "mlp.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <stdexcept>

namespace cpppl {

namespace {

constexpr int ST = 64, SK = 16;

struct SArgs {
  int64_t M, N, K;
  const float* A;
  int64_t sam, sak;
  const float* B;
  int64_t sbk, sbn;
  float* C;
  int64_t scm;
  float alpha, beta;
  const float* bias;  // [N] or null
  int relu;
  const float* mask;  // output *= (mask[m * smm + n] > 0) if non-null
  int64_t smm;
};

// C = alpha A B (+ beta C) (+ bias) (relu) (* mask) on the FP32 matrix cores:
// 64 x 64 tiles, four waves (2 x 2) of 32 x 32, each 2 x 2 blocks of
// v_mfma_f32_16x16x4f32.  K is walked in slices of 16 staged k-major in LDS
// (As[k][m], Bs[k][n]), so a fragment read is one float per lane: lane l takes
// A(m0 + l % 16, k + l / 16) and B(k + l / 16, n0 + l % 16); the result
// element (i, j) of a 16 x 16 block is register i % 4 of lane j + 16 (i / 4).
__global__ __launch_bounds__(256) void sgemm_kernel(const SArgs a) {
  __shared__ float As[SK][ST + 1];
  __shared__ float Bs[SK][ST + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t tiles_n = (a.N + ST - 1) / ST;
  const int64_t m0 = (blockIdx.x / tiles_n) * ST, n0 = (blockIdx.x % tiles_n) * ST;
  f4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};
  const bool a_kc = a.sak == 1, b_nc = a.sbn == 1;
  for (int64_t k0 = 0; k0 < a.K; k0 += SK) {
#pragma unroll
    for (int q = 0; q < ST * SK / 256; ++q) {
      const int e = tid + q * 256;
      const int mm = a_kc ? e / SK : e % ST, kk = a_kc ? e % SK : e / ST;
      const int64_t gm = m0 + mm, gk = k0 + kk;
      As[kk][mm] = (gm < a.M && gk < a.K) ? a.A[gm * a.sam + gk * a.sak] : 0.f;
      const int nn = b_nc ? e % ST : e / SK, kb = b_nc ? e / ST : e % SK;
      const int64_t gn = n0 + nn, gkb = k0 + kb;
      Bs[kb][nn] = (gn < a.N && gkb < a.K) ? a.B[gkb * a.sbk + gn * a.sbn] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < SK; ks += 4) {
      float af[2], bfr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = As[ks + (lane >> 4)][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bfr[j] = Bs[ks + (lane >> 4)][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int64_t gn = n0 + wn * 32 + j * 16 + (lane & 15);
        if (gm >= a.M || gn >= a.N) continue;
        float v = a.alpha * acc[i][j][r];
        if (a.beta != 0.f) v += a.beta * a.C[gm * a.scm + gn];
        if (a.bias) v += a.bias[gn];
        if (a.relu) v = fmaxf(v, 0.f);
        if (a.mask && !(a.mask[gm * a.smm + gn] > 0.f)) v = 0.f;
        a.C[gm * a.scm + gn] = v;
      }
}

void sgemm(const SArgs& a, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0) return;
  const int64_t blocks = ((a.M + ST - 1) / ST) * ((a.N + ST - 1) / ST);
  hipLaunchKernelGGL(sgemm_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
  CPPPL_LAUNCH_CHECK("sgemm");
}

// db[n] = sum_rows g[row][n]
__global__ void colsum_kernel(const float* g, int64_t rows, int64_t n, float* db) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= n) return;
  float s = 0.f;
  for (int64_t r = 0; r < rows; ++r) s += g[r * n + c];
  db[c] = s;
}

constexpr int LB = 256, LBLOCKS = 256;
// d = 2 (y - t) / numel into g; per-block sums of (y - t)^2 into part
__global__ __launch_bounds__(LB) void mse_kernel(const float* y, const float* t, int64_t numel,
                                                 float* g, float* part) {
  __shared__ float sh[LB];
  float s = 0.f;
  const float sc = 2.f / (float)numel;
  for (int64_t i = blockIdx.x * (int64_t)LB + threadIdx.x; i < numel; i += (int64_t)LBLOCKS * LB) {
    const float d = y[i] - t[i];
    s += d * d;
    if (g) g[i] = sc * d;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = LB / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ __launch_bounds__(LB) void mse_final_kernel(const float* part, int64_t numel, float* out) {
  __shared__ float sh[LB];
  float s = 0.f;
  for (int b = threadIdx.x; b < LBLOCKS; b += LB) s += part[b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = LB / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0] / (float)numel;
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                            float b1, float b2, float eps, float bc1, float bc2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

__global__ void gather_rows_kernel(const float* src, int64_t ld, const int64_t* idx, int64_t n,
                                   int64_t w, float* dst) {
  const int64_t total = n * w;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / w, c = e % w;
    dst[e] = src[idx[r] * ld + c];
  }
}

__global__ void copy_rows_kernel(const float* src, int64_t lds, int64_t n, int64_t w, float* dst,
                                 int64_t ldd) {
  const int64_t total = n * w;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / w, c = e % w;
    dst[r * ldd + c] = src[r * lds + c];
  }
}

// Column statistics of the stored rows (one work-group per column, FP64 sums
// in a fixed order): center != 0 gives mean and 1 / std (1 where the column is
// constant), center == 0 gives 1 / rms kept as the scale rms itself (1 where
// the column is zero).
__global__ __launch_bounds__(256) void colstats_kernel(const float* x, int64_t n, int64_t w,
                                                       int center, float* mu, float* sc) {
  __shared__ double sh[256];
  const int64_t c = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += 256) s += (double)x[r * w + c];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  const double mean = center ? sh[0] / (double)n : 0.0;
  __syncthreads();
  double q = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += 256) {
    const double d = (double)x[r * w + c] - mean;
    q += d * d;
  }
  sh[threadIdx.x] = q;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double sd = sqrt(sh[0] / (double)n);
    const bool flat = !(sd > 1e-30 * (1.0 + fabs(mean)));
    if (center) {
      mu[c] = (float)mean;
      sc[c] = flat ? 1.0f : (float)(1.0 / sd);
    } else {
      sc[c] = flat ? 1.0f : (float)sd;
    }
  }
}

// x[r][c] = (x[r][c] - mu[c]) * inv[c]  (mu may be null), rows of stride ld
__global__ void std_rows_kernel(float* x, int64_t ld, int64_t n, int64_t w, const float* mu,
                                const float* inv, int divide) {
  const int64_t total = n * w;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / w, c = e % w;
    float v = x[r * ld + c];
    if (mu) v -= mu[c];
    x[r * ld + c] = divide ? v / inv[c] : v * inv[c];
  }
}

unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1 << 16)); }

uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// Counter-based uniform in [0, 1): element i of the stream keyed by seed.
double uniform01(uint64_t seed, uint64_t i) {
  return (double)(splitmix64(seed * 0x9E3779B97F4A7C15ull + i) >> 11) * (1.0 / 9007199254740992.0);
}

int max_width(const cpppl_mlp* m) { return *std::max_element(m->sizes.begin(), m->sizes.end()); }

// work layout for `rows`: H_1 .. H_L (activations), G0, G1 (gradients), XB, YB, IDX
struct Work {
  float* H[16];
  float* G0;
  float* G1;
  float* XB;
  float* YB;
  int64_t* IDX;
};
Work work_layout(cpppl_mlp* m, int64_t /*rows*/) {
  const int64_t rows = m->work_rows;  // one layout for every call
  Work w{};
  float* p = m->work;
  for (int l = 1; l <= m->nl; ++l) {
    w.H[l] = p;
    p += rows * m->sizes[l];
  }
  const int mw = max_width(m);
  w.G0 = p; p += rows * mw;
  w.G1 = p; p += rows * mw;
  w.XB = p; p += rows * m->sizes[0];
  w.YB = p; p += rows * m->sizes[m->nl];
  if (((uintptr_t)p) & 7) ++p;  // 8-byte alignment for the index array
  w.IDX = (int64_t*)p;
  return w;
}
int64_t work_floats(const cpppl_mlp* m, int64_t rows) {
  int64_t f = 0;
  for (int l = 1; l <= m->nl; ++l) f += rows * m->sizes[l];
  f += 2 * rows * max_width(m) + rows * (m->sizes[0] + m->sizes[m->nl]) + 2 * rows + 64;
  return f;
}

}  // namespace

void mlp_ensure_work(cpppl_mlp* m, int64_t rows) {
  if (rows <= m->work_rows) return;
  if (m->work) CPPPL_HIP(hipFree(m->work));
  m->work = nullptr;
  CPPPL_HIP(hipMalloc((void**)&m->work, (size_t)work_floats(m, rows) * 4));
  m->work_rows = rows;
}

void mlp_forward_dev(cpppl_mlp* m, const float* x, int64_t n, float* y, hipStream_t s) {
  mlp_ensure_work(m, n);
  Work w = work_layout(m, n);
  const float* h = x;
  for (int l = 1; l <= m->nl; ++l) {
    const int fi = m->sizes[l - 1], fo = m->sizes[l];
    SArgs a{};
    a.M = n; a.N = fo; a.K = fi;
    a.A = h; a.sam = fi; a.sak = 1;
    a.B = m->params + m->woff[l - 1]; a.sbk = 1; a.sbn = fi;   // W_l (fo x fi): B(k, n) = W[n][k]
    a.C = (l == m->nl && y) ? y : w.H[l]; a.scm = fo;
    a.alpha = 1.f; a.beta = 0.f;
    a.bias = m->params + m->boff[l - 1];
    a.relu = l < m->nl;
    sgemm(a, s);
    h = a.C;
  }
}

void mlp_loss_grad_dev(cpppl_mlp* m, const float* x, const float* t, int64_t n, hipStream_t s) {
  mlp_forward_dev(m, x, n, nullptr, s);
  Work w = work_layout(m, n);
  const int L = m->nl;
  const int64_t out = m->sizes[L];
  float* g = w.G0;
  float* gn = w.G1;
  hipLaunchKernelGGL(mse_kernel, dim3(LBLOCKS), dim3(LB), 0, s, w.H[L], t, n * out, g, m->scal + 8);
  CPPPL_LAUNCH_CHECK("mse");
  hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(LB), 0, s, m->scal + 8, n * out, m->scal);
  CPPPL_LAUNCH_CHECK("mse_final");
  for (int l = L; l >= 1; --l) {
    const int fi = m->sizes[l - 1], fo = m->sizes[l];
    const float* hin = (l == 1) ? x : w.H[l - 1];
    SArgs dw{};  // dW_l = G^T H_{l-1}  (fo x fi)
    dw.M = fo; dw.N = fi; dw.K = n;
    dw.A = g; dw.sam = 1; dw.sak = fo;
    dw.B = hin; dw.sbk = fi; dw.sbn = 1;
    dw.C = m->grads + m->woff[l - 1]; dw.scm = fi;
    dw.alpha = 1.f;
    sgemm(dw, s);
    hipLaunchKernelGGL(colsum_kernel, dim3(nblk(fo)), dim3(256), 0, s, g, n, (int64_t)fo,
                       m->grads + m->boff[l - 1]);
    CPPPL_LAUNCH_CHECK("colsum");
    if (l > 1) {
      SArgs dx{};  // G_{l-1} = (G W_l) * (H_{l-1} > 0)
      dx.M = n; dx.N = fi; dx.K = fo;
      dx.A = g; dx.sam = fo; dx.sak = 1;
      dx.B = m->params + m->woff[l - 1]; dx.sbk = fi; dx.sbn = 1;
      dx.C = gn; dx.scm = fi;
      dx.alpha = 1.f;
      dx.mask = w.H[l - 1]; dx.smm = fi;
      sgemm(dx, s);
      std::swap(g, gn);
    }
  }
}

void mlp_std_x_dev(cpppl_mlp* m, float* x, int64_t ldx, int64_t n, hipStream_t s) {
  if (!m->standardized || n <= 0) return;
  const int64_t in = m->sizes[0];
  hipLaunchKernelGGL(std_rows_kernel, dim3(nblk(n * in)), dim3(256), 0, s, x, ldx, n, in,
                     (const float*)m->x_mu, (const float*)m->x_inv, 0);
  CPPPL_LAUNCH_CHECK("std_rows");
}

void mlp_unscale_y_dev(cpppl_mlp* m, float* y, int64_t ldy, int64_t n, hipStream_t s) {
  if (!m->standardized || n <= 0) return;
  const int64_t out = m->sizes[m->nl];
  // y * y_sc (no centring, multiplying)
  hipLaunchKernelGGL(std_rows_kernel, dim3(nblk(n * out)), dim3(256), 0, s, y, ldy, n, out,
                     (const float*)nullptr, (const float*)m->y_sc, 0);
  CPPPL_LAUNCH_CHECK("unscale_rows");
}

void mlp_append_dev(cpppl_mlp* m, const float* x, int64_t ldx, const float* y, int64_t ldy,
                    int64_t n, hipStream_t s) {
  if (m->nrows + n > m->cap) throw std::invalid_argument("training set capacity exceeded");
  const int64_t in = m->sizes[0], out = m->sizes[m->nl];
  float* xd = m->xs + m->nrows * in;
  float* yd = m->ys + m->nrows * out;
  hipLaunchKernelGGL(copy_rows_kernel, dim3(nblk(n * in)), dim3(256), 0, s, x, ldx, n, in, xd, in);
  CPPPL_LAUNCH_CHECK("copy_rows");
  hipLaunchKernelGGL(copy_rows_kernel, dim3(nblk(n * out)), dim3(256), 0, s, y, ldy, n, out, yd,
                     out);
  CPPPL_LAUNCH_CHECK("copy_rows");
  if (m->standardized) {
    mlp_std_x_dev(m, xd, in, n, s);
    hipLaunchKernelGGL(std_rows_kernel, dim3(nblk(n * out)), dim3(256), 0, s, yd, out, n, out,
                       (const float*)nullptr, (const float*)m->y_sc, 1);
    CPPPL_LAUNCH_CHECK("std_rows");
  }
  m->nrows += n;
}

}  // namespace cpppl

using namespace cpppl;

#define MLP_TRY(m)                                   \
  if (!(m)) return CPPPL_E_ARG;                      \
  try {                                              \
    CPPPL_HIP(hipSetDevice((m)->device));
#define MLP_CATCH(m)                                                     \
  }                                                                      \
  catch (const HipError& e) {                                            \
    (m)->err = std::string(e.where) + ": " + hipGetErrorString(e.err);   \
    return CPPPL_E_HIP;                                                  \
  }                                                                      \
  catch (const std::invalid_argument& e) {                               \
    (m)->err = e.what();                                                 \
    return CPPPL_E_ARG;                                                  \
  }                                                                      \
  catch (const std::exception& e) {                                      \
    (m)->err = e.what();                                                 \
    return CPPPL_E_STATE;                                                \
  }                                                                      \
  return CPPPL_OK;

static void mlp_free(cpppl_mlp* m) {
  for (void* p : {(void*)m->params, (void*)m->grads, (void*)m->adam_m, (void*)m->adam_v,
                  (void*)m->xs, (void*)m->ys, (void*)m->work, (void*)m->scal, (void*)m->x_mu,
                  (void*)m->x_inv, (void*)m->y_sc})
    if (p) (void)hipFree(p);
  if (m->host_scal) (void)hipHostFree(m->host_scal);
}

extern "C" {

CPPPL_API cpppl_status cpppl_mlp_create(int in_dim, int hidden, int n_hidden, int out_dim,
                                        int64_t capacity, uint64_t seed, int device,
                                        cpppl_mlp** out) {
  if (!out) return CPPPL_E_ARG;
  *out = nullptr;
  if (in_dim <= 0 || out_dim <= 0 || hidden <= 0 || n_hidden < 0 || n_hidden > 8 || capacity < 0)
    return CPPPL_E_ARG;
  cpppl_mlp* m = new (std::nothrow) cpppl_mlp();
  if (!m) return CPPPL_E_NOMEM;
  m->device = device;
  m->sizes.push_back(in_dim);
  for (int i = 0; i < n_hidden; ++i) m->sizes.push_back(hidden);
  m->sizes.push_back(out_dim);
  m->nl = (int)m->sizes.size() - 1;
  int64_t off = 0;
  for (int l = 1; l <= m->nl; ++l) {
    m->woff.push_back(off);
    off += (int64_t)m->sizes[l] * m->sizes[l - 1];
    m->boff.push_back(off);
    off += m->sizes[l];
  }
  m->nparams = off;
  m->cap = capacity;
  try {
    CPPPL_HIP(hipSetDevice(device));
    const size_t pb = (size_t)m->nparams * 4;
    CPPPL_HIP(hipMalloc((void**)&m->params, pb));
    CPPPL_HIP(hipMalloc((void**)&m->grads, pb));
    CPPPL_HIP(hipMalloc((void**)&m->adam_m, pb));
    CPPPL_HIP(hipMalloc((void**)&m->adam_v, pb));
    CPPPL_HIP(hipMemset(m->adam_m, 0, pb));
    CPPPL_HIP(hipMemset(m->adam_v, 0, pb));
    CPPPL_HIP(hipMalloc((void**)&m->xs, (size_t)std::max<int64_t>(1, capacity * in_dim) * 4));
    CPPPL_HIP(hipMalloc((void**)&m->ys, (size_t)std::max<int64_t>(1, capacity * out_dim) * 4));
    CPPPL_HIP(hipMalloc((void**)&m->scal, 1024 * 4));
    CPPPL_HIP(hipMalloc((void**)&m->x_mu, (size_t)in_dim * 4));
    CPPPL_HIP(hipMalloc((void**)&m->x_inv, (size_t)in_dim * 4));
    CPPPL_HIP(hipMalloc((void**)&m->y_sc, (size_t)out_dim * 4));
    CPPPL_HIP(hipHostMalloc((void**)&m->host_scal, 64 * 4, hipHostMallocDefault));
    std::vector<float> h((size_t)m->nparams, 0.f);
    for (int l = 1; l <= m->nl; ++l) {
      if (l == m->nl) continue;  // last layer starts at zero
      const int fi = m->sizes[l - 1], fo = m->sizes[l];
      const double bound = 1.0 / std::sqrt((double)fi);
      for (int64_t i = 0; i < (int64_t)fo * fi; ++i)
        h[m->woff[l - 1] + i] = (float)((2.0 * uniform01(seed, m->woff[l - 1] + i) - 1.0) * bound);
    }
    CPPPL_HIP(hipMemcpy(m->params, h.data(), pb, hipMemcpyHostToDevice));
  } catch (const HipError&) {
    mlp_free(m);
    delete m;
    return CPPPL_E_HIP;
  }
  *out = m;
  return CPPPL_OK;
}

CPPPL_API cpppl_status cpppl_mlp_destroy(cpppl_mlp* m) {
  if (!m) return CPPPL_E_ARG;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  mlp_free(m);
  delete m;
  return CPPPL_OK;
}

CPPPL_API cpppl_status cpppl_mlp_num_params(const cpppl_mlp* m, int64_t* n) {
  if (!m || !n) return CPPPL_E_ARG;
  *n = m->nparams;
  return CPPPL_OK;
}

CPPPL_API cpppl_status cpppl_mlp_get_params(cpppl_mlp* m, float* out, int on_device) {
  MLP_TRY(m)
  if (!out) throw std::invalid_argument("out is NULL");
  CPPPL_HIP(hipMemcpy(out, m->params, (size_t)m->nparams * 4,
                      on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  MLP_CATCH(m)
}

CPPPL_API cpppl_status cpppl_mlp_set_params(cpppl_mlp* m, const float* in, int on_device) {
  MLP_TRY(m)
  if (!in) throw std::invalid_argument("in is NULL");
  CPPPL_HIP(hipMemcpy(m->params, in, (size_t)m->nparams * 4,
                      on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
  CPPPL_HIP(hipMemset(m->adam_m, 0, (size_t)m->nparams * 4));
  CPPPL_HIP(hipMemset(m->adam_v, 0, (size_t)m->nparams * 4));
  m->adam_step = 0;
  MLP_CATCH(m)
}

// Copies n x w floats to a device staging buffer when the source is on the host.
static const float* stage_in(const float* src, int64_t n, int64_t w, int on_device, float* buf) {
  if (on_device) return src;
  CPPPL_HIP(hipMemcpy(buf, src, (size_t)(n * w) * 4, hipMemcpyHostToDevice));
  return buf;
}

CPPPL_API cpppl_status cpppl_mlp_forward(cpppl_mlp* m, const float* x, int64_t n, float* y,
                                         int on_device) {
  MLP_TRY(m)
  if (!x || !y || n <= 0) throw std::invalid_argument("bad forward arguments");
  mlp_ensure_work(m, n);
  Work w = work_layout(m, n);
  const float* xd = stage_in(x, n, m->sizes[0], on_device, w.XB);
  float* yd = on_device ? y : w.YB;
  mlp_forward_dev(m, xd, n, yd, nullptr);
  if (!on_device)
    CPPPL_HIP(hipMemcpy(y, yd, (size_t)(n * m->sizes[m->nl]) * 4, hipMemcpyDeviceToHost));
  CPPPL_HIP(hipDeviceSynchronize());
  MLP_CATCH(m)
}

CPPPL_API cpppl_status cpppl_mlp_grad(cpppl_mlp* m, const float* x, const float* y, int64_t n,
                                      float* loss, float* grads, int on_device) {
  MLP_TRY(m)
  if (!x || !y || n <= 0) throw std::invalid_argument("bad grad arguments");
  mlp_ensure_work(m, n);
  Work w = work_layout(m, n);
  const float* xd = stage_in(x, n, m->sizes[0], on_device, w.XB);
  const float* yd = stage_in(y, n, m->sizes[m->nl], on_device, w.YB);
  mlp_loss_grad_dev(m, xd, yd, n, nullptr);
  CPPPL_HIP(hipDeviceSynchronize());
  if (loss) CPPPL_HIP(hipMemcpy(loss, m->scal, 4, hipMemcpyDeviceToHost));
  if (grads)
    CPPPL_HIP(hipMemcpy(grads, m->grads, (size_t)m->nparams * 4,
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  MLP_CATCH(m)
}

CPPPL_API cpppl_status cpppl_mlp_add_rows(cpppl_mlp* m, const float* x, const float* y,
                                          int64_t n, int on_device) {
  MLP_TRY(m)
  if (!x || !y || n < 0) throw std::invalid_argument("bad rows");
  if (m->nrows + n > m->cap) throw std::invalid_argument("training set capacity exceeded");
  const int64_t in = m->sizes[0], out = m->sizes[m->nl];
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  CPPPL_HIP(hipMemcpy(m->xs + m->nrows * in, x, (size_t)(n * in) * 4, k));
  CPPPL_HIP(hipMemcpy(m->ys + m->nrows * out, y, (size_t)(n * out) * 4, k));
  m->nrows += n;
  MLP_CATCH(m)
}

CPPPL_API cpppl_status cpppl_mlp_num_rows(const cpppl_mlp* m, int64_t* n) {
  if (!m || !n) return CPPPL_E_ARG;
  *n = m->nrows;
  return CPPPL_OK;
}

CPPPL_API cpppl_status cpppl_mlp_get_rows(cpppl_mlp* m, float* x, float* y, int on_device) {
  MLP_TRY(m)
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  CPPPL_HIP(hipDeviceSynchronize());
  if (x) CPPPL_HIP(hipMemcpy(x, m->xs, (size_t)(m->nrows * m->sizes[0]) * 4, k));
  if (y) CPPPL_HIP(hipMemcpy(y, m->ys, (size_t)(m->nrows * m->sizes[m->nl]) * 4, k));
  MLP_CATCH(m)
}

CPPPL_API cpppl_status cpppl_mlp_clear_rows(cpppl_mlp* m) {
  if (!m) return CPPPL_E_ARG;
  m->nrows = 0;
  return CPPPL_OK;
}

CPPPL_API cpppl_status cpppl_mlp_train(cpppl_mlp* m, int epochs, float lr, int64_t batch,
                                       uint64_t seed, float* loss_hist) {
  MLP_TRY(m)
  if (epochs < 0 || !(lr > 0.f)) throw std::invalid_argument("bad training arguments");
  if (m->nrows == 0) throw std::invalid_argument("no training rows");
  const int64_t n = m->nrows;
  const bool full = batch <= 0 || batch >= n;
  const int64_t bs = full ? n : batch;
  mlp_ensure_work(m, std::max(bs, n));
  Work w = work_layout(m, std::max(bs, n));
  const int64_t in = m->sizes[0], out = m->sizes[m->nl];
  std::vector<int64_t> perm((size_t)n);
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  uint64_t ctr = 0;
  for (int ep = 0; ep < epochs; ++ep) {
    if (!full) {  // Fisher-Yates with the counter-based stream
      for (int64_t i = n - 1; i > 0; --i) {
        const int64_t j = (int64_t)(uniform01(seed, ctr++) * (double)(i + 1));
        std::swap(perm[i], perm[std::min(j, i)]);
      }
      CPPPL_HIP(hipMemcpy(w.IDX, perm.data(), (size_t)n * 8, hipMemcpyHostToDevice));
    }
    for (int64_t s0 = 0; s0 < n; s0 += bs) {
      const int64_t nb = std::min(bs, n - s0);
      const float* xb = m->xs + s0 * in;
      const float* yb = m->ys + s0 * out;
      if (!full) {
        hipLaunchKernelGGL(gather_rows_kernel, dim3(nblk(nb * in)), dim3(256), 0, nullptr, m->xs, in,
                           w.IDX + s0, nb, in, w.XB);
        hipLaunchKernelGGL(gather_rows_kernel, dim3(nblk(nb * out)), dim3(256), 0, nullptr, m->ys,
                           out, w.IDX + s0, nb, out, w.YB);
        CPPPL_LAUNCH_CHECK("gather_rows");
        xb = w.XB;
        yb = w.YB;
      }
      mlp_loss_grad_dev(m, xb, yb, nb, nullptr);
      m->adam_step++;
      const double bc1 = 1.0 - std::pow(0.9, (double)m->adam_step);
      const double bc2 = 1.0 - std::pow(0.999, (double)m->adam_step);
      hipLaunchKernelGGL(adam_kernel, dim3(nblk(m->nparams)), dim3(256), 0, nullptr, m->params,
                         m->grads, m->adam_m, m->adam_v, m->nparams, lr, 0.9f, 0.999f, 1e-8f,
                         (float)bc1, (float)bc2);
      CPPPL_LAUNCH_CHECK("adam");
    }
    if (loss_hist) {  // loss over all stored rows after the epoch
      mlp_forward_dev(m, m->xs, n, nullptr, nullptr);
      Work wn = work_layout(m, n);
      hipLaunchKernelGGL(mse_kernel, dim3(LBLOCKS), dim3(LB), 0, nullptr, wn.H[m->nl], m->ys,
                         n * out, (float*)nullptr, m->scal + 8);
      hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(LB), 0, nullptr, m->scal + 8, n * out,
                         m->scal);
      CPPPL_LAUNCH_CHECK("mse");
      CPPPL_HIP(hipMemcpy(&loss_hist[ep], m->scal, 4, hipMemcpyDeviceToHost));
    }
  }
  CPPPL_HIP(hipDeviceSynchronize());
  MLP_CATCH(m)
}

CPPPL_API cpppl_status cpppl_mlp_standardize(cpppl_mlp* m) {
  MLP_TRY(m)
  if (m->standardized) throw std::logic_error("the network is already standardised");
  if (m->nrows < 2) throw std::invalid_argument("standardising needs at least two stored rows");
  const int64_t in = m->sizes[0], out = m->sizes[m->nl], n = m->nrows;
  hipLaunchKernelGGL(colstats_kernel, dim3((unsigned)in), dim3(256), 0, nullptr, m->xs, n, in, 1,
                     m->x_mu, m->x_inv);
  CPPPL_LAUNCH_CHECK("colstats_x");
  hipLaunchKernelGGL(colstats_kernel, dim3((unsigned)out), dim3(256), 0, nullptr, m->ys, n, out, 0,
                     (float*)nullptr, m->y_sc);
  CPPPL_LAUNCH_CHECK("colstats_y");
  m->standardized = true;
  mlp_std_x_dev(m, m->xs, in, n, nullptr);
  hipLaunchKernelGGL(std_rows_kernel, dim3(nblk(n * out)), dim3(256), 0, nullptr, m->ys, out, n,
                     out, (const float*)nullptr, (const float*)m->y_sc, 1);
  CPPPL_LAUNCH_CHECK("std_rows");
  CPPPL_HIP(hipDeviceSynchronize());
  MLP_CATCH(m)
}

CPPPL_API cpppl_status cpppl_mlp_get_standardization(cpppl_mlp* m, float* x_mu, float* x_inv,
                                                     float* y_sc) {
  MLP_TRY(m)
  if (!m->standardized) throw std::logic_error("the network is not standardised");
  const int64_t in = m->sizes[0], out = m->sizes[m->nl];
  if (x_mu) CPPPL_HIP(hipMemcpy(x_mu, m->x_mu, (size_t)in * 4, hipMemcpyDeviceToHost));
  if (x_inv) CPPPL_HIP(hipMemcpy(x_inv, m->x_inv, (size_t)in * 4, hipMemcpyDeviceToHost));
  if (y_sc) CPPPL_HIP(hipMemcpy(y_sc, m->y_sc, (size_t)out * 4, hipMemcpyDeviceToHost));
  MLP_CATCH(m)
}

CPPPL_API cpppl_status cpppl_mlp_save(cpppl_mlp* m, const char* path) {
  MLP_TRY(m)
  if (!path) throw std::invalid_argument("path is NULL");
  std::vector<float> h((size_t)m->nparams);
  CPPPL_HIP(hipMemcpy(h.data(), m->params, (size_t)m->nparams * 4, hipMemcpyDeviceToHost));
  FILE* f = fopen(path, "wb");
  if (!f) throw std::invalid_argument("cannot open file for writing");
  const char magic[8] = {'C', 'P', 'P', 'P', 'L', 'M', 'L', 'P'};
  const int32_t nl = m->nl;
  bool ok = fwrite(magic, 1, 8, f) == 8 && fwrite(&nl, 4, 1, f) == 1;
  for (int s : m->sizes) {
    const int32_t v = s;
    ok = ok && fwrite(&v, 4, 1, f) == 1;
  }
  ok = ok && fwrite(h.data(), 4, h.size(), f) == h.size();
  // the standardisation: a flag, then x_mu, x_inv (in_dim) and y_sc (out_dim)
  const int64_t in = m->sizes[0], out = m->sizes[m->nl];
  const int32_t sflag = m->standardized ? 1 : 0;
  ok = ok && fwrite(&sflag, 4, 1, f) == 1;
  if (m->standardized) {
    std::vector<float> st((size_t)(2 * in + out));
    CPPPL_HIP(hipMemcpy(st.data(), m->x_mu, (size_t)in * 4, hipMemcpyDeviceToHost));
    CPPPL_HIP(hipMemcpy(st.data() + in, m->x_inv, (size_t)in * 4, hipMemcpyDeviceToHost));
    CPPPL_HIP(hipMemcpy(st.data() + 2 * in, m->y_sc, (size_t)out * 4, hipMemcpyDeviceToHost));
    ok = ok && fwrite(st.data(), 4, st.size(), f) == st.size();
  }
  fclose(f);
  if (!ok) throw std::invalid_argument("write failed");
  MLP_CATCH(m)
}

CPPPL_API cpppl_status cpppl_mlp_load(cpppl_mlp* m, const char* path) {
  MLP_TRY(m)
  if (!path) throw std::invalid_argument("path is NULL");
  FILE* f = fopen(path, "rb");
  if (!f) throw std::invalid_argument("cannot open file");
  char magic[8];
  int32_t nl = 0;
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "CPPPLMLP", 8) == 0 &&
            fread(&nl, 4, 1, f) == 1 && nl == m->nl;
  for (int i = 0; ok && i <= m->nl; ++i) {
    int32_t v = 0;
    ok = fread(&v, 4, 1, f) == 1 && v == m->sizes[i];
  }
  std::vector<float> h((size_t)m->nparams);
  ok = ok && fread(h.data(), 4, h.size(), f) == h.size();
  const int64_t in = m->sizes[0], out = m->sizes[m->nl];
  int32_t sflag = 0;
  ok = ok && fread(&sflag, 4, 1, f) == 1 && (sflag == 0 || sflag == 1);
  std::vector<float> st((size_t)(2 * in + out));
  if (ok && sflag) ok = fread(st.data(), 4, st.size(), f) == st.size();
  fclose(f);
  if (!ok) throw std::invalid_argument("file does not hold a network of this shape");
  CPPPL_HIP(hipMemcpy(m->params, h.data(), (size_t)m->nparams * 4, hipMemcpyHostToDevice));
  if (sflag) {
    CPPPL_HIP(hipMemcpy(m->x_mu, st.data(), (size_t)in * 4, hipMemcpyHostToDevice));
    CPPPL_HIP(hipMemcpy(m->x_inv, st.data() + in, (size_t)in * 4, hipMemcpyHostToDevice));
    CPPPL_HIP(hipMemcpy(m->y_sc, st.data() + 2 * in, (size_t)out * 4, hipMemcpyHostToDevice));
  }
  m->standardized = sflag != 0;
  MLP_CATCH(m)
}

}  // extern "C"
