// Shared device/host helpers for the CP-PPL gfx950 library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef uint16_t bf16_t;  // storage type of bfloat16 values

namespace cpppl {

// Round-to-nearest-even float -> bfloat16 (NaN kept quiet).
__host__ __device__ inline bf16_t f32_to_bf16(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (bf16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__host__ __device__ inline float bf16_to_f32(bf16_t h) {
  uint32_t u = ((uint32_t)h) << 16;
  return __builtin_bit_cast(float, u);
}

// Two floats to packed bfloat16 (round to nearest even), one v_cvt_pk_bf16_f32
// on gfx950: `lo` in the low half.  The same rounding as f32_to_bf16 for every
// finite value; the software form compiles to a NaN test and a branch per value.
__device__ inline uint32_t pack_bf16x2(float lo, float hi) {
  typedef float f2_t __attribute__((ext_vector_type(2)));
  typedef __bf16 b2_t __attribute__((ext_vector_type(2)));
  const f2_t x = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(x, b2_t));
}

template <typename T> struct Conv;
template <> struct Conv<double> {
  __device__ static inline double from_f64(double x) { return x; }
  __device__ static inline double to_f64(double x) { return x; }
};
template <> struct Conv<float> {
  __device__ static inline float from_f64(double x) { return (float)x; }
  __device__ static inline double to_f64(float x) { return (double)x; }
};
template <> struct Conv<bf16_t> {
  __device__ static inline bf16_t from_f64(double x) { return f32_to_bf16((float)x); }
  __device__ static inline double to_f64(bf16_t x) { return (double)bf16_to_f32(x); }
};

// Map a dispatch-order block id to a logical id so that each of the 8 XCDs
// (which receive blocks round-robin) works on one contiguous range of
// logical ids; neighbouring tiles then share that XCD's L2.
__device__ inline int64_t xcd_remap(int64_t bid, int64_t nblocks) {
  const int64_t X = 8;
  if (nblocks < X) return bid;
  int64_t per = nblocks / X, rem = nblocks % X;
  int64_t xcd = bid % X, idx = bid / X;
  int64_t start = xcd * per + (xcd < rem ? xcd : rem);
  return start + idx;
}

// Launch-error helper used by host launchers.
struct HipError {
  hipError_t err;
  const char* where;
};

}  // namespace cpppl

#define CPPPL_LAUNCH_CHECK(where)                                  \
  do {                                                             \
    hipError_t e__ = hipGetLastError();                            \
    if (e__ != hipSuccess) throw cpppl::HipError{e__, where};      \
  } while (0)

#define CPPPL_HIP(call)                                            \
  do {                                                             \
    hipError_t e__ = (call);                                       \
    if (e__ != hipSuccess) throw cpppl::HipError{e__, #call};      \
  } while (0)
