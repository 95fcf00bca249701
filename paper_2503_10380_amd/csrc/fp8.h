// OCP FP8 e4m3 (1 sign, 4 exponent bits with bias 7, 3 mantissa bits; no
// infinities, 0x7F / 0xFF are NaN, largest finite magnitude 448) as used by
// gfx950: encoding with round-to-nearest-even and saturation, decoding to FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cpppl {

constexpr float E4M3_MAX = 448.0f;

// Nearest e4m3 code of x (ties to even mantissa), magnitudes above 448
// saturate to 448, NaN maps to the NaN code.
__device__ __forceinline__ uint8_t e4m3_encode(double x) {
  if (x != x) return 0x7F;
  const uint8_t sign = (x < 0.0 || (x == 0.0 && __double_as_longlong(x) < 0)) ? 0x80 : 0x00;
  double a = fabs(x);
  if (a >= 448.0) return sign | 0x7E;
  if (a < 0.015625) {  // below 2^-6: subnormal codes m 2^-9, m = 0..7 (m = 8 is 2^-6)
    const double q = rint(a * 512.0);
    return sign | (uint8_t)q;
  }
  int k;
  const double f = frexp(a, &k);  // a = f 2^k, f in [0.5, 1)
  int e = k - 1;                  // a = (2 f) 2^e, 2 f in [1, 2)
  double q = rint((2.0 * f - 1.0) * 8.0);
  if (q == 8.0) {
    q = 0.0;
    e += 1;
  }
  if (e > 8 || (e == 8 && q > 6.0)) return sign | 0x7E;
  return sign | (uint8_t)(((e + 7) << 3) | (int)q);
}

// Value of an e4m3 code (the NaN codes decode to 480, never produced above).
__device__ __forceinline__ float e4m3_decode(uint32_t c) {
  const uint32_t e = (c >> 3) & 0xF, m = c & 7;
  float v;
  if (e == 0) {
    v = (float)m * 0.001953125f;  // m 2^-9
  } else {
    v = __uint_as_float(((c & 0x7F) << 20)) * 1.329227995784916e36f;  // (1 + m/8) 2^(e-7): 2^120
  }
  return (c & 0x80) ? -v : v;
}

// Eight e4m3 codes (byte i of q = element i) times `scale` as eight bfloat16
// (element i in bits 16 (i % 2) of word i / 2), by the gfx950 scaled
// conversion; exact when `scale` is a power of two and the products stay in
// the normal bfloat16 range.
__device__ __forceinline__ uint4 e4m3x8_to_bf16(uint2 q, float scale) {
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  const bf16x2_t w0 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(q.x, scale, false);
  const bf16x2_t w1 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(q.x, scale, true);
  const bf16x2_t w2 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(q.y, scale, false);
  const bf16x2_t w3 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(q.y, scale, true);
  return make_uint4(__builtin_bit_cast(uint32_t, w0), __builtin_bit_cast(uint32_t, w1),
                    __builtin_bit_cast(uint32_t, w2), __builtin_bit_cast(uint32_t, w3));
}

}  // namespace cpppl
