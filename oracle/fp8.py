"""OCP FP8 E4M3 numbers and the scaled e4m3 storage of t and B (FP8 ablation).

Format (OCP 8-bit floating point specification, E4M3 variant): one sign bit,
four exponent bits with bias 7 and three mantissa bits.  Exponent field 0
holds the subnormals m * 2^-9 (m = 0..7); fields 1..15 hold (1 + m/8) *
2^(field - 7).  There are no infinities; S.1111.111 is NaN, so the largest
finite magnitude is 1.75 * 2^8 = 448.  Encoding rounds to the nearest value,
ties to the even mantissa, and saturates at +-448.

Scaled storage (the reading taken for the FP8 ablation of the mixed-precision
MTTKRP): t is stored per (i, j) row of its (o^2 x v^2) matrix and B per
X slice (v x v), each with one power-of-two scale s, the least 2^e
(e in [-126, 127]) with max |x| <= 448 s (s = 1 for an all-zero row); the
stored value is e4m3(x / s) and the value the contraction uses is
decode(code) * s.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Pinned by the spec
values, a brute-force nearest-value search and the error bound in
tests/test_oracle_fp8.py.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0
NAN_CODES = (0x7F, 0xFF)


def e4m3_decode(codes) -> np.ndarray:
    """Value of each e4m3 code (NaN for the two NaN codes)."""
    c = np.asarray(codes).astype(np.int64) & 0xFF
    field = (c >> 3) & 0xF
    man = (c & 7).astype(np.float64)
    mag = np.where(field == 0, man * 2.0 ** -9, (1.0 + man / 8.0) * np.exp2(field - 7.0))
    mag = np.where((c & 0x7F) == 0x7F, np.nan, mag)
    return np.where(c & 0x80, -mag, mag)


def e4m3_encode(x) -> np.ndarray:
    """Nearest e4m3 code (ties to even mantissa), saturating at +-448; NaN -> 0x7F.

    In the binade [2^e, 2^(e+1)) (e >= -6; e = -6 also covers the subnormals)
    the representable magnitudes are n * 2^(e-3) with n = 8..15 (n = 0..7 for
    the subnormals), and the code magnitude is 8 (e + 6) + n, which also gives
    the right code when rounding carries n to 16 (the next binade).
    """
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    inrange = a < E4M3_MAX                              # False for NaN and inf too
    ar = np.where(inrange, a, 0.0)
    _, k = np.frexp(ar)                                 # ar = f 2^k, f in [0.5, 1)
    e = np.where(ar < 2.0 ** -6, -6, k - 1)
    n = np.rint(ar / np.exp2(e - 3.0))                  # ties to even n = even mantissa
    mag = (8 * (e + 6) + n).astype(np.int64)
    mag = np.where(a >= E4M3_MAX, 0x7E, np.minimum(mag, 0x7E))
    code = np.where(np.signbit(x), 0x80 | mag, mag)
    code = np.where(np.isnan(x), 0x7F, code)
    return code.astype(np.uint8)


def pow2_scale(maxabs: float) -> float:
    """The least power of two s = 2^e, e in [-126, 127], with maxabs <= 448 s."""
    if maxabs == 0.0:
        return 1.0
    e = int(np.ceil(np.log2(maxabs / E4M3_MAX)))
    e = min(max(e, -126), 127)
    # log2 is rounded: settle e on the exact comparisons
    while e > -126 and maxabs <= E4M3_MAX * 2.0 ** (e - 1):
        e -= 1
    while e < 127 and maxabs > E4M3_MAX * 2.0 ** e:
        e += 1
    return float(2.0 ** e)


def quantize_rows(x2d: np.ndarray):
    """(codes, scales) of a matrix stored row by row with one scale per row."""
    x2d = np.asarray(x2d, dtype=np.float64)
    scales = np.array([pow2_scale(float(np.max(np.abs(row)))) if row.size else 1.0
                       for row in x2d])
    codes = e4m3_encode(x2d / scales[:, None])
    return codes, scales


def dequantize_rows(codes: np.ndarray, scales: np.ndarray) -> np.ndarray:
    return e4m3_decode(codes) * np.asarray(scales, dtype=np.float64)[:, None]


def fp8_inputs(t: np.ndarray, b_vv: np.ndarray):
    """The t and B values an FP8 context contracts: t quantized per (i, j) row,
    B per X slice, both returned dequantized in FP64 with their original shapes."""
    o, _, v, _ = t.shape
    nx = b_vv.shape[0]
    tq = dequantize_rows(*quantize_rows(t.reshape(o * o, v * v))).reshape(t.shape)
    bq = dequantize_rows(*quantize_rows(b_vv.reshape(nx, v * v))).reshape(b_vv.shape)
    return tq, bq
