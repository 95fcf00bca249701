"""Pins of the oracle's e4m3 numbers (oracle.fp8) against the OCP E4M3 format
definition: the table values the specification fixes, a brute-force search for
the nearest representable value, the tie rule, saturation, the relative error
bound 2^-4 of normal values, and the power-of-two scale definition."""
import numpy as np
import pytest

from oracle import fp8

FINITE = np.array([c for c in range(256) if c not in fp8.NAN_CODES], dtype=np.uint8)


def test_spec_values():
    # largest normal, smallest normal, largest and smallest subnormal, one, zero
    d = fp8.e4m3_decode
    assert d(0x7E) == 448.0 and d(0xFE) == -448.0
    assert d(0x08) == 2.0 ** -6
    assert d(0x07) == 0.875 * 2.0 ** -6
    assert d(0x01) == 2.0 ** -9
    assert d(0x38) == 1.0 and d(0xB8) == -1.0
    assert d(0x00) == 0.0 and np.signbit(d(0x80))
    assert d(0x77) == 240.0  # 1.875 * 2^7
    assert np.isnan(d(0x7F)) and np.isnan(d(0xFF))
    enc = fp8.e4m3_encode
    assert enc(448.0) == 0x7E and enc(1.0) == 0x38 and enc(2.0 ** -9) == 0x01
    assert enc(-2.0) == 0xC0 and enc(2.0 ** -6) == 0x08 and enc(0.0) == 0x00
    assert enc(-0.0) == 0x80 and enc(np.nan) == 0x7F


def test_round_trip_every_finite_code():
    np.testing.assert_array_equal(fp8.e4m3_encode(fp8.e4m3_decode(FINITE)), FINITE)


def test_values_are_monotone_in_the_code():
    pos = fp8.e4m3_decode(np.arange(0, 0x7F, dtype=np.uint8))
    assert np.all(np.diff(pos) > 0)


def test_nearest_value_by_brute_force():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-460, 460, 4000), rng.uniform(-0.05, 0.05, 4000),
                        rng.standard_normal(2000) * 2.0 ** rng.integers(-12, 8, 2000)])
    table = fp8.e4m3_decode(FINITE)
    got = fp8.e4m3_decode(fp8.e4m3_encode(x))
    best = np.min(np.abs(x[:, None] - table[None, :]), axis=1)
    np.testing.assert_array_equal(np.abs(x - got), best)
    assert np.all(np.sign(got) * np.sign(x) >= 0)


def test_ties_go_to_the_even_mantissa():
    pos = fp8.e4m3_decode(np.arange(0, 0x7F, dtype=np.uint8))
    mids = 0.5 * (pos[:-1] + pos[1:])        # exact in FP64
    codes = fp8.e4m3_encode(mids).astype(int)
    lo = np.arange(0, 0x7E)
    want = np.where(lo % 2 == 0, lo, lo + 1)  # the neighbour whose mantissa is even
    np.testing.assert_array_equal(codes, want)
    np.testing.assert_array_equal(fp8.e4m3_encode(-mids).astype(int), want | 0x80)


def test_saturation():
    for x in (448.0, 449.0, 463.99, 464.0, 480.0, 1e6, np.inf):
        assert fp8.e4m3_encode(x) == 0x7E
        assert fp8.e4m3_encode(-x) == 0xFE


def test_relative_error_bound_of_normals():
    rng = np.random.default_rng(1)
    x = np.exp(rng.uniform(np.log(2.0 ** -6), np.log(448.0), 20000))
    q = fp8.e4m3_decode(fp8.e4m3_encode(x))
    assert np.max(np.abs(q - x) / x) <= 2.0 ** -4
    # subnormal range: absolute error at most half the spacing 2^-9
    y = rng.uniform(0, 2.0 ** -6, 5000)
    assert np.max(np.abs(fp8.e4m3_decode(fp8.e4m3_encode(y)) - y)) <= 2.0 ** -10


@pytest.mark.parametrize("m", [1.0, 448.0, 448.0 * 2 ** 3, 448.0 * 2 ** -7 * 1.0000001, 0.75,
                               3.1e-30, 2.5e30, 1e-300])
def test_pow2_scale_is_the_least_power_of_two(m):
    s = fp8.pow2_scale(m)
    e = int(np.log2(s))
    assert s == 2.0 ** e
    assert m <= 448.0 * s or e == 127
    assert m > 448.0 * s / 2 or e == -126


def test_quantize_rows_range_and_error():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((6, 300)) * np.array([1e-8, 1e-3, 1.0, 7.0, 448.0, 1e5])[:, None]
    x[1, 5] = 0.0
    codes, scales = fp8.quantize_rows(x)
    q = fp8.dequantize_rows(codes, scales)
    for r in range(6):
        s = scales[r]
        assert np.max(np.abs(x[r])) <= 448.0 * s
        assert np.max(np.abs(x[r])) > 224.0 * s           # least power of two
        big = np.abs(x[r]) >= 2.0 ** -6 * s
        assert np.all(np.abs(q[r] - x[r])[big] <= 2.0 ** -4 * np.abs(x[r])[big])
        assert np.all(np.abs(q[r] - x[r])[~big] <= 2.0 ** -10 * s)
    assert np.all(fp8.quantize_rows(np.zeros((2, 4)))[1] == 1.0)


def test_fp8_inputs_shapes_and_slices():
    rng = np.random.default_rng(3)
    t = rng.standard_normal((3, 3, 8, 8))
    b = rng.standard_normal((5, 8, 8))
    b[2] *= 1e-3
    tq, bq = fp8.fp8_inputs(t, b)
    assert tq.shape == t.shape and bq.shape == b.shape
    # each X slice has its own scale: the small slice keeps its relative accuracy
    assert np.linalg.norm(bq[2] - b[2]) / np.linalg.norm(b[2]) < 2.0 ** -4
    assert np.linalg.norm(tq - t) / np.linalg.norm(t) < 2.0 ** -4
