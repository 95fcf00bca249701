/*
 * cpppl_testing.h -- kernel-level test hooks of libcpppl (not part of the
 * product ABI; used by the parity tests to check the matrix-core GEMM and the
 * block sweep-operator SPD inverse in isolation).  All pointers are device pointers on the
 * current HIP device; work is enqueued on `stream` and the call synchronises it.
 */
#ifndef CPPPL_TESTING_H
#define CPPPL_TESTING_H

#include <stdint.h>

#include "cpppl.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C[b](m,n) = alpha sum_k A[b](m,k) B[b](k,n) + beta C[b](m,n) with
 * A(m,k) at A + b*sab + m*sam + k*sak, B(k,n) at B + b*sbb + k*sbk + n*sbn,
 * C(m,n) at C + b*scb + m*scm + n.  in_dtype 0: FP64 operands, 1: BF16
 * operands (uint16 storage); c_dtype 0: FP64, 1: FP32, 2: BF16.  splits > 1
 * uses `partial` (splits*batch*M*N doubles). */
CPPPL_API cpppl_status cpppl_test_gemm(int in_dtype, int64_t M, int64_t N, int64_t K, int64_t batch,
                                       const void* A, int64_t sam, int64_t sak, int64_t sab,
                                       const void* B, int64_t sbk, int64_t sbn, int64_t sbb,
                                       void* C, int64_t scm, int64_t scb, int c_dtype, double alpha,
                                       double beta, int splits, void* partial, void* stream);

/* As cpppl_test_gemm with BF16 A and an e4m3 B that is k-contiguous
 * (sbk == 1, one byte per element), dequantised exactly inside the kernel and
 * multiplied by bscale[n] (bscale_mode 1), bscale[k] (mode 2; equal within
 * each aligned group of 8 k) or 1 (mode 0); the scales should be powers of two. */
CPPPL_API cpppl_status cpppl_test_gemm_e4m3b(int64_t M, int64_t N, int64_t K, int64_t batch,
                                             const void* A, int64_t sam, int64_t sak, int64_t sab,
                                             const uint8_t* B, int64_t sbn, int64_t sbb,
                                             const float* bscale, int bscale_mode, void* C,
                                             int64_t scm, int64_t scb, int c_dtype, int splits,
                                             void* partial, void* stream);

/* OCP e4m3 codes of a rows x len FP64 matrix with one power-of-two scale per
 * row (scale[r], the least 2^e with max |x[r][:]| <= 448 * 2^e), as the FP8
 * contexts store t and B: q[r][k] = e4m3(x[r][k] / scale[r]). */
CPPPL_API cpppl_status cpppl_test_quantize_e4m3(const double* x, int64_t rows, int64_t len,
                                                uint8_t* q, float* scale, void* stream);

/* out[i] = bfloat16 bits of decode(q[i]) * scale, by the conversion the GEMM
 * loader uses; n a multiple of 8. */
CPPPL_API cpppl_status cpppl_test_dequant_e4m3(const uint8_t* q, int64_t n, float scale,
                                               uint16_t* out, void* stream);

/* Y (R x n) = W^{-1} X for SPD W (R x R, overwritten; `work` holds
 * R*R + 8192 doubles) by the block sweep-operator inverse; status: 0 ok,
 * 1 bad pivot. */
CPPPL_API cpppl_status cpppl_test_spd_solve(double* W, int64_t R, const double* X, double* Y,
                                            int64_t n, double* work, int* status, void* stream);

/* Failure-path hook: in the next cpppl_als call on ctx, the W_alpha inverse
 * that is forked one sweep early for sweep `sweep` (0-based within that call;
 * forked while the sweep before it runs, only when sweeps are issued ahead)
 * reports a failed pivot although none failed.  The call then takes its
 * recovery path: the sweep issued ahead is dropped and that sweep is redone
 * synchronously from its snapshot under the ridge rule (report.careful_sweeps).
 * A host-side flag read when the sweep is issued; -1 clears it; cleared at the
 * end of every cpppl_als call.  E_ARG for a NULL ctx or sweep < -1. */
CPPPL_API cpppl_status cpppl_test_inject_alpha_fault(cpppl_ctx* ctx, int sweep);

#ifdef __cplusplus
}
#endif

#endif /* CPPPL_TESTING_H */
