"""Pins of the oracle's synthetic CCD-like iteration (oracle.ccd): the exact
ladder iteration converges to the direct solution of D t = w + s R(t), by at
least the contraction factor the scale guarantees; s = 0 gives the MP2
amplitudes; the symmetrised CP ladder keeps t pair-symmetric; the
near-optimal guess caches the iterate after sweep n - 5."""
import numpy as np
import pytest

import oracle
from oracle import ccd
import synth


@pytest.fixture(scope="module")
def c1():
    cfg = synth.CONFIGS["C1"]
    inp = synth.make_inputs(cfg)
    return cfg, inp, synth.exchange_integrals(inp), synth.ccd_scale(inp)


def test_mp2_limit(c1):
    """One Jacobi step without the ladder returns w / D, the MP2 amplitudes the
    input generator builds by its own route."""
    cfg, inp, w, s = c1
    t = ccd.jacobi_update(w, np.ones_like(w), inp.e_occ, inp.e_vir, 0.0)
    np.testing.assert_allclose(t, inp.t, rtol=1e-14, atol=0)
    d = ccd.denominators(inp.e_occ, inp.e_vir)
    assert d.max() <= -1.0  # the generator's energies keep every denominator <= -1


def test_exact_ladder_converges_to_direct_solve(c1):
    cfg, inp, w, s = c1
    t_star = ccd.exact_fixed_point(w, inp.b_vv, inp.e_occ, inp.e_vir, s)
    # the fixed point solves D t = w + s R(t) with R from the oracle's explicit route
    resid = ccd.denominators(inp.e_occ, inp.e_vir) * t_star - w - s * oracle.form_r(t_star, inp.b_vv)
    assert np.abs(resid).max() <= 1e-13 * np.abs(w).max()
    t, hist = ccd.ccd_loop(w, inp.b_vv, inp.e_occ, inp.e_vir, s, 60, cfg.rank, exact=True)
    np.testing.assert_allclose(t, t_star, rtol=0, atol=1e-13 * np.abs(t_star).max())
    # contraction by at least 1/2 per step (the scale's guarantee), checked on the step sizes
    dts = [h["dt_norm"] for h in hist[:10]]
    assert all(b <= 0.5 * a + 1e-15 for a, b in zip(dts, dts[1:]))
    assert dts[0] > 0.0


def test_ladder_changes_the_amplitudes(c1):
    """The ladder term is not negligible at this scale: the fixed point moves
    t away from MP2 by more than 1 % (so a CP error in it shows in t)."""
    cfg, inp, w, s = c1
    t_star = ccd.exact_fixed_point(w, inp.b_vv, inp.e_occ, inp.e_vir, s)
    assert np.linalg.norm(t_star - inp.t) > 1e-2 * np.linalg.norm(inp.t)


@pytest.mark.parametrize("guess", ["random", "optimal", "near_optimal"])
def test_cp_loop_keeps_pair_symmetry_and_follows_guess_rule(c1, guess):
    cfg, inp, w, s = c1
    t, hist = ccd.ccd_loop(w, inp.b_vv, inp.e_occ, inp.e_vir, s, 4, cfg.rank, guess=guess,
                           seed=3)
    np.testing.assert_allclose(t, t.transpose(1, 0, 3, 2), rtol=0, atol=1e-15 * np.abs(t).max())
    assert hist[0]["guess"] == "random"
    for h in hist[1:]:
        if guess == "near_optimal":
            assert h["guess"] in ("near_optimal", "optimal")
        else:
            assert h["guess"] == guess
    assert all(1 <= h["sweeps"] <= 100 for h in hist)


def test_near_optimal_cache_is_iterate_n_minus_5(c1):
    """With n > 5 ALS sweeps in CC step 1, step 2 starts from the iterate after
    sweep n - 5 of step 1 (rerun here sweep by sweep)."""
    cfg, inp, w, s = c1
    t0 = inp.t
    r = oracle.form_r(t0, inp.b_vv)
    init = oracle.rng.random_guess(cfg.o, cfg.v, cfg.rank, 3 + 1)
    its = []
    f, lam, h = oracle.cp_als(r, init, 100, tol=1e-3, stop_rule=1,
                              on_sweep=lambda fs, l: its.append(fs))
    n = len(h["fit"])
    assert n > 5
    # the iterate after sweep n - 5, reached by running n - 5 sweeps from the start
    f5, _, _ = oracle.cp_als(r, init, n - 5)
    for a, b in zip(its[n - 6], f5):
        np.testing.assert_array_equal(a, b)
    # the loop's second step starts there: its ALS from that cache gives step 2's fit
    _, hist = ccd.ccd_loop(w, inp.b_vv, inp.e_occ, inp.e_vir, s, 2, cfg.rank,
                           guess="near_optimal", seed=3)
    assert hist[0]["sweeps"] == n and hist[1]["guess"] == "near_optimal"
    t1 = ccd.jacobi_update(w, oracle.symmetrize_pairs(oracle.cp_full(f, lam)), inp.e_occ,
                           inp.e_vir, s)
    r1 = oracle.form_r(t1, inp.b_vv)
    _, _, h2 = oracle.cp_als(r1, f5, 100, tol=1e-3, stop_rule=1)
    assert hist[1]["sweeps"] == len(h2["fit"])
    assert hist[1]["fit"] == pytest.approx(h2["fit"][-1], abs=1e-14)
