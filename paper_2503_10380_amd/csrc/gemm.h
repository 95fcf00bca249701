// Strided, batched, split-K matrix-core GEMM for gfx950.
//
//   C[b](m, n) = alpha * sum_k A[b](m, k) * B[b](k, n) + beta * C[b](m, n)
//
// A(m, k) lives at A + b*sab + m*sam + k*sak and B(k, n) at B + b*sbb + k*sbk + n*sbn;
// for each operand one of its two strides must be 1 (the contiguous index may
// be either the contracted one or the free one).  C(m, n) lives at
// C + b*scb + m*scm + n.  With splits > 1 the K range is cut into `splits`
// chunks whose partial products go to `partial` (splits*batch*M*N accumulator
// elements) and are then summed in a fixed order (deterministic).
#pragma once

#include "common.h"

namespace cpppl {

enum class DType : int { F64 = 0, F32 = 1, BF16 = 2 };

struct Gemm {
  int64_t M = 0, N = 0, K = 0, batch = 1;
  const void* A = nullptr;
  int64_t sam = 0, sak = 0, sab = 0;
  const void* B = nullptr;
  int64_t sbk = 0, sbn = 0, sbb = 0;
  void* C = nullptr;
  int64_t scm = 0, scb = 0;
  DType ctype = DType::F64;
  double alpha = 1.0, beta = 0.0;
  int splits = 1;
  void* partial = nullptr;
  // gemm_f64 only: with splits > 1, leave the partial products in `partial`
  // (splits x batch x M x N, split-major) for the caller to sum; C is not written.
  bool keep_partials = false;
  // gemm_bf16 only: B holds OCP e4m3 codes (one byte each, k-contiguous),
  // dequantised to bfloat16 on the way into LDS and multiplied by a scale
  // (exact for power-of-two scales): bscale_mode 0 none, 1 bscale[n] (per
  // column of C), 2 bscale[k] (must be equal within each aligned group of 8 k).
  bool b_fp8 = false;
  const float* bscale = nullptr;
  int bscale_mode = 0;
};

// A and B in FP64, accumulation in FP64 (v_mfma_f64_16x16x4f64).  Returns
// the number of K splits used (at most g.splits: K is cut in whole slices).
int gemm_f64(const Gemm& g, hipStream_t s);
// A and B in bfloat16 (B optionally e4m3, see Gemm::b_fp8), accumulation in
// FP32 (v_mfma_f32_16x16x32_bf16); beta must be 0 unless split.
void gemm_bf16(const Gemm& g, hipStream_t s);

// Split count giving roughly `target_blocks` work-groups, with at least
// `min_k` of K per split.
int choose_splits(int64_t tiles, int64_t K, int64_t target_blocks, int64_t min_k, int max_splits);

int64_t gemm_tiles_f64(int64_t M, int64_t N);
// 128 x 128 output tiles of an M x N result (the tiles of every split-K gemm_bf16).
int64_t gemm_tiles_bf16(int64_t M, int64_t N);

}  // namespace cpppl
