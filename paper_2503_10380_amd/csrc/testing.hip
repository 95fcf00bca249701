// Kernel-level test hooks (cpppl_testing.h).
#include <algorithm>
#include <cstdio>
#include <stdexcept>

#include "../../include/cpppl_testing.h"
#include "fp8.h"
#include "gemm.h"
#include "linalg.h"
#include "ops.h"

using namespace cpppl;

namespace {
__global__ void dequant_kernel(const uint8_t* __restrict__ q, int64_t chunks, float scale,
                               uint4* out) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < chunks;
       c += (int64_t)gridDim.x * blockDim.x)
    out[c] = e4m3x8_to_bf16(*(const uint2*)(q + 8 * c), scale);
}
}  // namespace

extern "C" {

CPPPL_API cpppl_status cpppl_test_gemm(int in_dtype, int64_t M, int64_t N, int64_t K, int64_t batch,
                                       const void* A, int64_t sam, int64_t sak, int64_t sab,
                                       const void* B, int64_t sbk, int64_t sbn, int64_t sbb,
                                       void* Cp, int64_t scm, int64_t scb, int c_dtype, double alpha,
                                       double beta, int splits, void* partial, void* stream) {
  try {
    Gemm g;
    g.M = M; g.N = N; g.K = K; g.batch = batch;
    g.A = A; g.sam = sam; g.sak = sak; g.sab = sab;
    g.B = B; g.sbk = sbk; g.sbn = sbn; g.sbb = sbb;
    g.C = Cp; g.scm = scm; g.scb = scb;
    g.ctype = c_dtype == 0 ? DType::F64 : (c_dtype == 1 ? DType::F32 : DType::BF16);
    g.alpha = alpha; g.beta = beta; g.splits = splits; g.partial = partial;
    hipStream_t s = (hipStream_t)stream;
    if (in_dtype == 0) gemm_f64(g, s);
    else gemm_bf16(g, s);
    if (hipStreamSynchronize(s) != hipSuccess) return CPPPL_E_HIP;
  } catch (const std::invalid_argument& e) {
    fprintf(stderr, "cpppl_test_gemm: %s\n", e.what());
    return CPPPL_E_ARG;
  } catch (const HipError& e) {
    fprintf(stderr, "cpppl_test_gemm: %s: %s\n", e.where, hipGetErrorString(e.err));
    return CPPPL_E_HIP;
  }
  return CPPPL_OK;
}

CPPPL_API cpppl_status cpppl_test_gemm_e4m3b(int64_t M, int64_t N, int64_t K, int64_t batch,
                                             const void* A, int64_t sam, int64_t sak, int64_t sab,
                                             const uint8_t* B, int64_t sbn, int64_t sbb,
                                             const float* bscale, int bscale_mode, void* Cp,
                                             int64_t scm, int64_t scb, int c_dtype, int splits,
                                             void* partial, void* stream) {
  try {
    Gemm g;
    g.M = M; g.N = N; g.K = K; g.batch = batch;
    g.A = A; g.sam = sam; g.sak = sak; g.sab = sab;
    g.B = B; g.sbk = 1; g.sbn = sbn; g.sbb = sbb;
    g.b_fp8 = true; g.bscale = bscale; g.bscale_mode = bscale_mode;
    g.C = Cp; g.scm = scm; g.scb = scb;
    g.ctype = c_dtype == 0 ? DType::F64 : (c_dtype == 1 ? DType::F32 : DType::BF16);
    g.splits = splits; g.partial = partial;
    hipStream_t s = (hipStream_t)stream;
    gemm_bf16(g, s);
    if (hipStreamSynchronize(s) != hipSuccess) return CPPPL_E_HIP;
  } catch (const std::invalid_argument& e) {
    fprintf(stderr, "cpppl_test_gemm_e4m3b: %s\n", e.what());
    return CPPPL_E_ARG;
  } catch (const HipError& e) {
    fprintf(stderr, "cpppl_test_gemm_e4m3b: %s: %s\n", e.where, hipGetErrorString(e.err));
    return CPPPL_E_HIP;
  }
  return CPPPL_OK;
}

CPPPL_API cpppl_status cpppl_test_quantize_e4m3(const double* x, int64_t rows, int64_t len,
                                                uint8_t* q, float* scale, void* stream) {
  if (rows < 0 || len <= 0) return CPPPL_E_ARG;
  try {
    hipStream_t s = (hipStream_t)stream;
    e4m3_row_scales(x, rows, len, scale, s);
    quantize_e4m3(x, q, rows * len, scale, len, rows > 0 ? rows : 1, 1, s);
    if (hipStreamSynchronize(s) != hipSuccess) return CPPPL_E_HIP;
  } catch (const std::invalid_argument& e) {
    fprintf(stderr, "cpppl_test_quantize_e4m3: %s\n", e.what());
    return CPPPL_E_ARG;
  } catch (const HipError& e) {
    fprintf(stderr, "cpppl_test_quantize_e4m3: %s: %s\n", e.where, hipGetErrorString(e.err));
    return CPPPL_E_HIP;
  }
  return CPPPL_OK;
}

CPPPL_API cpppl_status cpppl_test_dequant_e4m3(const uint8_t* q, int64_t n, float scale,
                                               uint16_t* out, void* stream) {
  if (n < 0 || n % 8 != 0) return CPPPL_E_ARG;
  if (((uintptr_t)q & 7) || ((uintptr_t)out & 15)) return CPPPL_E_ARG;
  const int64_t chunks = n / 8;
  if (chunks == 0) return CPPPL_OK;
  hipStream_t s = (hipStream_t)stream;
  const unsigned blocks = (unsigned)std::min<int64_t>((chunks + 255) / 256, 65536);
  hipLaunchKernelGGL(dequant_kernel, dim3(blocks), dim3(256), 0, s, q, chunks, scale, (uint4*)out);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return CPPPL_E_HIP;
  return CPPPL_OK;
}

CPPPL_API cpppl_status cpppl_test_spd_solve(double* W, int64_t R, const double* X, double* Y,
                                            int64_t n, double* work, int* status, void* stream) {
  try {
    hipStream_t s = (hipStream_t)stream;
    double* inv = spd_inverse_neg(W, work, work + R * R, R, status, s);
    Gemm g;
    g.M = R; g.N = n; g.K = R;
    g.A = inv; g.sam = R; g.sak = 1;
    g.B = X; g.sbk = n; g.sbn = 1;
    g.C = Y; g.scm = n; g.ctype = DType::F64; g.alpha = -1.0;
    gemm_f64(g, s);
    if (hipStreamSynchronize(s) != hipSuccess) return CPPPL_E_HIP;
  } catch (const HipError& e) {
    fprintf(stderr, "cpppl_test_spd_solve: %s: %s\n", e.where, hipGetErrorString(e.err));
    return CPPPL_E_HIP;
  }
  return CPPPL_OK;
}

}
