"""Pins of the oracle's singles-dressed PPL tensor (eq. B, eq. fulldfB, eq. dfB):
the Dbar route against the un-simplified four-index form, the t1 = 0 reduction,
the three MTTKRP routes, and the rank-one tau closed form."""
import numpy as np
import pytest

import oracle
import synth


def _problem(o, v, nx, seed):
    rng = np.random.default_rng(seed)
    n = o + v
    b = rng.standard_normal((nx, n, n))
    b = 0.5 * (b + b.transpose(0, 2, 1))
    t2 = rng.standard_normal((o, o, v, v))
    t2 = 0.5 * (t2 + t2.transpose(1, 0, 3, 2))
    t1 = 0.3 * rng.standard_normal((o, v))
    return b, t2, t1


def test_dbar_route_equals_four_index_form():
    b, t2, t1 = _problem(3, 5, 4, 0)
    tau, bvv, dbar = oracle.dress(t2, t1, b)
    r = oracle.form_r(tau, bvv, b_right=dbar)
    np.testing.assert_allclose(r, oracle.form_r_fulldf(t2, t1, b), rtol=0, atol=1e-12)
    np.testing.assert_allclose(r, oracle.form_r_einsum(tau, bvv, dbar), rtol=0, atol=1e-12)


def test_dressing_by_hand():
    b, t2, t1 = _problem(2, 3, 2, 1)
    tau, bvv, dbar = oracle.dress(t2, t1, b)
    o = 2
    for (i, j, c, d) in [(0, 1, 2, 0), (1, 1, 0, 2)]:
        assert tau[i, j, c, d] == pytest.approx(t2[i, j, c, d] + t1[i, c] * t1[j, d], abs=1e-15)
    for (x, bb, d) in [(0, 1, 2), (1, 2, 0)]:
        want = b[x, o + bb, o + d] - 2.0 * sum(b[x, o + bb, k] * t1[k, d] for k in range(o))
        assert dbar[x, bb, d] == pytest.approx(want, abs=1e-14)


def test_zero_singles_reduce_to_doubles():
    b, t2, _ = _problem(3, 4, 5, 2)
    tau, bvv, dbar = oracle.dress(t2, np.zeros((3, 4)), b)
    np.testing.assert_array_equal(tau, t2)
    np.testing.assert_array_equal(dbar, bvv)
    np.testing.assert_allclose(oracle.form_r(tau, bvv, b_right=dbar), oracle.form_r(t2, bvv),
                               rtol=0, atol=1e-13)


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_singles_mttkrp_three_routes(mode):
    b, t2, t1 = _problem(2, 3, 2, 3)
    tau, bvv, dbar = oracle.dress(t2, t1, b)
    rng = np.random.default_rng(4)
    fs = (rng.standard_normal((2, 3)), rng.standard_normal((2, 3)),
          rng.standard_normal((3, 3)), rng.standard_normal((3, 3)))
    r = oracle.form_r(tau, bvv, b_right=dbar)
    want = oracle.mttkrp(r, fs, mode)
    np.testing.assert_allclose(oracle.mttkrp_chain(tau, bvv, fs, mode, b_right=dbar), want,
                               rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.mttkrp_bruteforce(tau, bvv, fs, mode, b_right=dbar), want,
                               rtol=1e-12, atol=1e-12)


def test_rank_one_tau_closed_form():
    """t2 = 0 and t1 = u p^T make tau = u u p p, so R is the rank-X CP tensor
    (u, u, B p, Dbar p) of the closed form."""
    cfg = synth.custom_config(3, 5, 4, 2)
    rng = np.random.default_rng(5)
    b = rng.standard_normal((4, 8, 8))
    b = 0.5 * (b + b.transpose(0, 2, 1))
    t1, (u, p) = synth.rank1_singles(cfg)
    tau, bvv, dbar = oracle.dress(np.zeros((3, 3, 5, 5)), t1, b)
    r = oracle.form_r(tau, bvv, b_right=dbar)
    cf = oracle.rank1_closed_form(u, u, p, p, bvv, dbar)
    np.testing.assert_allclose(r, oracle.cp_full(cf), rtol=0, atol=1e-12)


def test_singles_break_pair_symmetry_only_through_dbar():
    """R_ijab = R_jiba holds without singles (t pair symmetric, B symmetric)
    and fails with them (Dbar is on the b side only): a property of eq. dfB
    the GPU path must not assume."""
    b, t2, t1 = _problem(3, 4, 3, 6)
    tau0, bvv, _ = oracle.dress(t2, np.zeros_like(t1), b)
    r0 = oracle.form_r(tau0, bvv)
    np.testing.assert_allclose(r0, r0.transpose(1, 0, 3, 2), rtol=0, atol=1e-12)
    tau, bvv, dbar = oracle.dress(t2, t1, b)
    r = oracle.form_r(tau, bvv, b_right=dbar)
    assert np.abs(r - r.transpose(1, 0, 3, 2)).max() > 1e-3
