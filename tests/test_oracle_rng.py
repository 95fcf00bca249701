"""Pins of the oracle's counter-based SplitMix64 and random guess: the
generator's published first outputs for seed 0, the exact [-1, 1) mapping,
and the layout of the draws over the four factors."""
import numpy as np

from oracle import rng


def test_splitmix64_published_outputs():
    # first three outputs of SplitMix64 from state 0 (reference implementation)
    got = rng.splitmix64(0, [0, 1, 2])
    assert [int(x) for x in got] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform_mapping_is_exact_and_in_range():
    z = rng.splitmix64(7, np.arange(1000, dtype=np.uint64))
    u = rng.uniform_pm1(7, np.arange(1000, dtype=np.uint64))
    assert np.all(u >= -1.0) and np.all(u < 1.0)
    np.testing.assert_array_equal((u + 1.0) * 2.0 ** 52, (z >> np.uint64(11)).astype(np.float64))
    big = rng.uniform_pm1(3, np.arange(200000, dtype=np.uint64))
    assert abs(big.mean()) < 0.01 and abs(big.var() - 1.0 / 3.0) < 0.01


def test_random_guess_layout():
    g, r, a, b = rng.random_guess(2, 3, 4, seed=11)
    assert g.shape == (2, 4) and r.shape == (2, 4) and a.shape == (3, 4) and b.shape == (3, 4)
    assert a[1, 2] == rng.uniform_pm1(11, [2 * 4 + 2 * 4 + 1 * 4 + 2])[0]
    assert g[0, 3] == rng.uniform_pm1(11, [3])[0]
    assert not np.array_equal(rng.random_guess(2, 3, 4, seed=12)[0], g)
