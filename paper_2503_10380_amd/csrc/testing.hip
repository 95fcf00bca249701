// Kernel-level test hooks (cpppl_testing.h).
#include <cstdio>
#include <stdexcept>

#include "../../include/cpppl_testing.h"
#include "gemm.h"
#include "linalg.h"

using namespace cpppl;

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
