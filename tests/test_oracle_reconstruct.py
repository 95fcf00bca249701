"""Pins of the oracle's pair symmetrisation of a reconstructed tensor (Section
"The CPD approximation of the PPL tensor-network"): symmetry, idempotence,
fixed points, and the invariance of a contraction with a pair-symmetric t."""
import numpy as np

import oracle


def test_symmetrize_pairs_properties():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 3, 4, 4))
    s = oracle.symmetrize_pairs(x)
    np.testing.assert_array_equal(s, s.transpose(1, 0, 3, 2))
    np.testing.assert_array_equal(oracle.symmetrize_pairs(s), s)
    # entries by hand
    assert s[0, 2, 1, 3] == 0.5 * (x[0, 2, 1, 3] + x[2, 0, 3, 1])
    assert s[1, 1, 2, 2] == x[1, 1, 2, 2]
    # a contraction with a pair-symmetric t does not see the symmetrisation
    t = rng.standard_normal((3, 3, 4, 4))
    t = t + t.transpose(1, 0, 3, 2)
    assert np.sum(s * t) == np.sum(x * t) or abs(np.sum(s * t) - np.sum(x * t)) < 1e-12


def test_cp_full_by_hand():
    rng = np.random.default_rng(1)
    fs = [rng.standard_normal((n, 2)) for n in (2, 2, 3, 3)]
    lam = np.array([0.5, 2.0])
    cp = oracle.cp_full(fs, lam)
    i, j, a, b = 1, 0, 2, 1
    want = sum(lam[r] * fs[0][i, r] * fs[1][j, r] * fs[2][a, r] * fs[3][b, r] for r in range(2))
    assert abs(cp[i, j, a, b] - want) < 1e-14
