"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

MTTKRPs are compared per mode for identical factors, element by element
(rtol 1e-10 with atol 1e-10 max|M|, the FP64 target; low-precision paths by
the bounds derived in bounds.py); ALS trajectories are compared sweep by sweep
from the same starting factors, including the C2 workload over 30 sweeps and a
rank-1024 problem whose W inverse takes 16 pivot blocks; ||R||^2, E_exact, E_CP
(final and per sweep) and the fit scalars against the oracle's explicit
tensors; the FP64 refinement of the BF16 and FP8 paths against the oracle's
sweeps from the same state.  Sizes span several GEMM tiles with ragged tails.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from bounds import (N_ROUND_BF16, abs_chain, assert_fp64, assert_lowp, chain_lengths)

pytestmark = pytest.mark.gpu

SMALL = {
    "C1": synth.CONFIGS["C1"],
    "ragged_xlt_v": synth.custom_config(3, 10, 7, 5, name="o3v10X7R5"),
    "ragged_tiles": synth.custom_config(5, 33, 70, 70, name="o5v33X70R70"),
    "odd": synth.custom_config(7, 19, 61, 131, name="o7v19X61R131"),
}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


_CACHE = {}


def _problem(cfg):
    if cfg.name not in _CACHE:
        inp = synth.make_inputs(cfg)
        r = oracle.form_r(inp.t, inp.b_vv)
        _CACHE[cfg.name] = (inp, r)
    return _CACHE[cfg.name]


def _ctx(lib, cfg, inp, precision="fp64"):
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, precision)
    ctx.load_t2(inp.t)
    ctx.load_df(inp.b_vv)
    return ctx


@pytest.mark.parametrize("name", list(SMALL))
def test_norm_r2_and_energy_exact(lib, name):
    cfg = SMALL[name]
    _say(f"norm_r2 {name}")
    inp, r = _problem(cfg)
    ctx = _ctx(lib, cfg, inp)
    n2, e = ctx.norm_r2()
    n2_o, e_o = oracle.norm_r2_and_energy(r, inp.t)
    assert n2 == pytest.approx(n2_o, rel=1e-12)
    assert e == pytest.approx(e_o, rel=1e-12)


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_mttkrp_fp64(lib, name, mode):
    cfg = SMALL[name]
    _say(f"mttkrp fp64 {name} mode {mode}")
    inp, r = _problem(cfg)
    fs = synth.init_factors(cfg)
    ctx = _ctx(lib, cfg, inp)
    ctx.set_factors(*fs)
    got = ctx.mttkrp(mode)
    want = oracle.mttkrp(r, fs, mode)
    assert_fp64(got, want)


def test_set_get_factors_roundtrip(lib):
    cfg = SMALL["odd"]
    inp, _ = _problem(cfg)
    fs = synth.init_factors(cfg)
    lam = np.linspace(0.5, 1.5, cfg.rank)
    ctx = _ctx(lib, cfg, inp)
    ctx.set_factors(*fs, lam)
    out = ctx.get_factors()
    for a, b in zip(out, (*fs, lam)):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("name", list(SMALL))
def test_fit_and_energy_at_given_factors(lib, name):
    cfg = SMALL[name]
    _say(f"fit/energy {name}")
    inp, r = _problem(cfg)
    fs = synth.init_factors(cfg)
    lam = np.linspace(0.5, 1.5, cfg.rank)
    ctx = _ctx(lib, cfg, inp)
    ctx.set_factors(*fs, lam)
    fit, inner, cp2 = ctx.fit()
    cp = oracle.cp_full(fs, lam)
    assert inner == pytest.approx(np.sum(r * cp), rel=1e-11)
    assert cp2 == pytest.approx(np.sum(cp * cp), rel=1e-11)
    want_fit = 1 - np.linalg.norm(r - cp) / np.linalg.norm(r)
    assert fit == pytest.approx(want_fit, rel=1e-9, abs=1e-9)
    assert ctx.energy() == pytest.approx(np.sum(cp * inp.t), rel=1e-11)


@pytest.mark.parametrize("name", list(SMALL))
def test_als_trajectory_fp64(lib, name):
    cfg = SMALL[name]
    _say(f"als trajectory {name}")
    inp, r = _problem(cfg)
    fs = synth.init_factors(cfg)
    n2 = float(np.sum(r * r))
    f_o, lam_o, hist = oracle.cp_als(r, fs, 10, norm_r2=n2, t=inp.t)
    ctx = _ctx(lib, cfg, inp)
    ctx.set_factors(*fs)
    rep = ctx.als(10, energy=True, eta=True)
    assert rep["sweeps"] == 10
    np.testing.assert_allclose(rep["fit_hist"], hist["fit"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(rep["eta_hist"], hist["eta"], rtol=1e-7, atol=1e-9)
    # without eta the sweeps are the same and eta is reported as NaN
    ctx.set_factors(*fs)
    rep2 = ctx.als(10)
    np.testing.assert_allclose(rep2["fit_hist"], rep["fit_hist"], rtol=0, atol=1e-12)
    assert np.all(np.isnan(rep2["eta_hist"]))
    assert rep["loss"] == pytest.approx(hist["loss"][-1], rel=1e-8)
    assert rep["energy_cp"] == pytest.approx(hist["energy"][-1], rel=1e-8)
    fi, fj, fa, fb, lam = ctx.get_factors()
    for g_, w_ in zip((fi, fj, fa, fb), f_o):
        assert _rel(g_, w_) <= 1e-7
    assert _rel(lam, lam_o) <= 1e-7


def test_als_stop_rule_fit(lib):
    cfg = SMALL["C1"]
    inp, r = _problem(cfg)
    fs = synth.init_factors(cfg)
    _, _, hist = oracle.cp_als(r, fs, 50, stop_rule=1, tol=1e-3)
    ctx = _ctx(lib, cfg, inp)
    ctx.set_factors(*fs)
    rep = ctx.als(50, stop_rule=1, tol=1e-3)
    assert rep["sweeps"] == len(hist["fit"])


def test_ridge_retry_matches_oracle(lib):
    cfg = SMALL["ragged_tiles"]
    _say("ridge retry")
    inp, r = _problem(cfg)
    fs = [np.array(f) for f in synth.init_factors(cfg)]
    fs[3][:, 0] = 0.0  # a zero beta column makes W of the first update singular
    _, _, hist = oracle.cp_als(r, fs, 3)
    assert hist["retries"] > 0
    ctx = _ctx(lib, cfg, inp)
    ctx.set_factors(*fs)
    rep = ctx.als(3)
    assert rep["ridge_retries"] == hist["retries"]
    np.testing.assert_allclose(rep["fit_hist"], hist["fit"], rtol=0, atol=1e-9)


def test_planted_cp_tensor(lib):
    cfg = synth.custom_config(6, 20, 30, 24, name="planted")
    _say("planted")
    pf = synth.planted_factors(cfg, 12)
    true, lamp = pf[:4], pf[4]
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank)
    ctx.load_planted(*true, lamp)
    r = oracle.cp_full(true, lamp)
    n2, e = ctx.norm_r2()
    assert n2 == pytest.approx(np.sum(r * r), rel=1e-12)
    assert np.isnan(e)
    fs = synth.init_factors(cfg)
    ctx.set_factors(*fs)
    for mode in range(4):
        assert_fp64(ctx.mttkrp(mode), oracle.mttkrp(r, fs, mode))
    _, _, hist = oracle.cp_als(r, fs, 5)
    rep = ctx.als(5)
    np.testing.assert_allclose(rep["fit_hist"], hist["fit"], rtol=0, atol=1e-9)


def test_planted_recovery_from_perturbed_start(lib):
    cfg = synth.custom_config(16, 128, 384, 512, name="C2planted")
    _say("planted C2 recovery")
    pf = synth.planted_factors(cfg, 512)
    true, lamp = pf[:4], pf[4]
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank)
    ctx.load_planted(*true, lamp)
    rng = np.random.default_rng(0)
    start = [f + 1e-3 * rng.standard_normal(f.shape) for f in true]
    ctx.set_factors(*start)
    rep = ctx.als(10)
    assert rep["fit"] >= 1 - 1e-7


@pytest.mark.slow
@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_mttkrp_fp64_c2(lib, mode):
    cfg = synth.CONFIGS["C2"]
    _say(f"mttkrp fp64 C2 mode {mode}")
    inp, r = _problem(cfg)
    fs = synth.init_factors(cfg)
    ctx = _ctx(lib, cfg, inp)
    ctx.set_factors(*fs)
    assert_fp64(ctx.mttkrp(mode), oracle.mttkrp(r, fs, mode))


@pytest.mark.parametrize("cfg_name", ["C3", "C5"])
def test_full_size_rank1_t2_closed_form(lib, cfg_name):
    """At the full workload sizes: T2 = u w p q makes R an exact rank-X CP tensor
    whose MTTKRPs have a closed form (no O(N^6) work), in FP64 and BF16."""
    cfg = synth.CONFIGS[cfg_name]
    _say(f"closed form {cfg_name}")
    rng = np.random.default_rng(cfg.cfg_id)
    b = rng.standard_normal((cfg.nx, cfg.v, cfg.v)) / np.sqrt(cfg.nx)
    t, (u, w, p, q) = synth.rank1_t2(cfg)
    cf = oracle.rank1_closed_form(u, w, p, q, b)
    # |t| = |u||w||p||q| is rank one too: the chain on absolute values in closed form
    cf_abs = oracle.rank1_closed_form(np.abs(u), np.abs(w), np.abs(p), np.abs(q), np.abs(b))
    fs = synth.init_factors(cfg)
    fs_abs = [np.abs(f) for f in fs]
    for prec in ("fp64", "bf16"):
        ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, prec)
        ctx.load_t2(t)
        ctx.load_df(b)
        ctx.set_factors(*fs)
        for mode in range(4):
            want = oracle.planted_mttkrp(cf, np.ones(cfg.nx), fs, mode)
            got = ctx.mttkrp(mode)
            _say(f"  {prec} mode {mode} rel err {_rel(got, want):.3e}")
            if prec == "fp64":
                assert_fp64(got, want)
            else:
                m_abs = oracle.planted_mttkrp(cf_abs, np.ones(cfg.nx), fs_abs, mode)
                assert_lowp(got, want, m_abs, N_ROUND_BF16,
                            chain_lengths(cfg.o, cfg.v, cfg.nx, mode), f"bf16 mode {mode}")
        ctx.close()
        del ctx


@pytest.mark.parametrize("name", ["C1", "ragged_tiles", "odd"])
def test_mttkrp_bf16_bounds(lib, name):
    """BF16 MTTKRP against the oracle's FP64 chain: element-wise within the
    rigorous rounding bound of the chain on absolute values, norm-wise within
    twice the statistical estimate (bounds.py)."""
    cfg = SMALL[name]
    _say(f"mttkrp bf16 bounds {name}")
    inp, r = _problem(cfg)
    fs = synth.init_factors(cfg)
    ctx = _ctx(lib, cfg, inp, "bf16")
    ctx.set_factors(*fs)
    for mode in range(4):
        want = oracle.mttkrp(r, fs, mode)
        m_abs = abs_chain(inp.t, inp.b_vv, fs, mode)
        err = assert_lowp(ctx.mttkrp(mode), want, m_abs, N_ROUND_BF16,
                          chain_lengths(cfg.o, cfg.v, cfg.nx, mode), f"{name} mode {mode}")
        _say(f"  mode {mode}: {err:.2e}")
    ctx.close()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_fp64_refinement_matches_oracle(lib, prec):
    """S13: from a state S reached by low-precision sweeps, the FP64 refinement
    sweeps of that context follow the oracle's textbook ALS from S: fit, energy
    and factors sweep by sweep; and they equal what an FP64 context gives from S."""
    cfg = synth.custom_config(5, 40, 70, 70, name="o5v40X70R70")
    _say(f"refinement vs oracle ({prec})")
    inp, r = _problem(cfg)
    clp = _ctx(lib, cfg, inp, prec)
    clp.set_factors(*synth.init_factors(cfg))
    clp.als(4)
    state = clp.get_factors()
    k = 4
    rl = clp.als(0, refine=k, energy_every=True, energy=True)
    assert rl["sweeps"] == k and rl["refine_sweeps"] == k
    f_o, lam_o, hist = oracle.cp_als(r, state[:4], k, norm_r2=float(np.sum(r * r)), t=inp.t)
    np.testing.assert_allclose(rl["fit_hist"], hist["fit"], rtol=0, atol=1e-10)
    np.testing.assert_allclose(rl["energy_hist"], hist["energy"], rtol=1e-10, atol=0)
    assert rl["energy_cp"] == pytest.approx(hist["energy"][-1], rel=1e-10)
    got = clp.get_factors()
    for g_, w_ in zip(got[:4], f_o):
        assert_fp64(g_, w_, rtol=1e-8)
    assert_fp64(got[4], lam_o, rtol=1e-8)
    c64 = _ctx(lib, cfg, inp, "fp64")
    c64.set_factors(*state)
    r64 = c64.als(k, energy_every=True)
    np.testing.assert_allclose(rl["fit_hist"], r64["fit_hist"], rtol=0, atol=1e-12)
    # same-init energy check of the mixed path: the refinement reproduces the
    # FP64 path's E_CP to 1e-8 Ha from identical factors
    assert np.abs(rl["energy_hist"] - r64["energy_hist"]).max() <= 1e-8
    for a, b in zip(clp.get_factors(), c64.get_factors()):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-10 * max(1.0, np.abs(b).max()))
    clp.close()
    c64.close()


def test_refinement_stop_rules(lib):
    """refine_tol stops the FP64 refinement once the fit changes by less than
    the tolerance; refine_etol once E_CP changes by less than it between two
    FP64 sweeps; with both set, both must hold."""
    cfg = SMALL["ragged_tiles"]
    _say("refinement stop rules")
    inp = synth.make_inputs(cfg)
    c16 = _ctx(lib, cfg, inp, "bf16")
    c16.set_factors(*synth.init_factors(cfg))
    c16.als(3)
    state = c16.get_factors()
    # BF16 sweeps to a stop rule, then refinement until |dfit| < 1e-4 (at most 40)
    c16.set_factors(*state)
    r = c16.als(20, stop_rule=1, tol=1e-3, refine=40, refine_tol=1e-4)
    n_bf = r["sweeps"] - r["refine_sweeps"]
    assert 1 <= n_bf <= 20 and 1 <= r["refine_sweeps"] <= 40
    h = r["fit_hist"]
    if r["refine_sweeps"] < 40:
        assert abs(h[-1] - h[-2]) < 1e-4
    if r["refine_sweeps"] > 1:
        assert all(abs(h[k] - h[k - 1]) >= 1e-4 for k in range(n_bf, len(h) - 1))
    # energy criterion: the reference run records E_CP of 40 FP64 sweeps
    c16.set_factors(*state)
    full = c16.als(0, refine=40, energy_every=True)["energy_hist"]
    etol = float(np.median(np.abs(np.diff(full))))
    want = next((n for n in range(1, 40) if abs(full[n] - full[n - 1]) < etol), None)
    c16.set_factors(*state)
    r = c16.als(0, refine=40, refine_etol=etol)
    assert r["refine_sweeps"] == (40 if want is None else want + 1)
    np.testing.assert_allclose(r["energy_hist"], full[:r["sweeps"]], rtol=1e-13, atol=0)
    # both criteria: the later of the two stops
    c16.set_factors(*state)
    fits = c16.als(0, refine=40)["fit_hist"]
    ftol = float(np.median(np.abs(np.diff(fits))))
    both = next((n for n in range(1, 40) if abs(full[n] - full[n - 1]) < etol
                 and abs(fits[n] - fits[n - 1]) < ftol), None)
    c16.set_factors(*state)
    r = c16.als(0, refine=40, refine_etol=etol, refine_tol=ftol)
    assert r["refine_sweeps"] == (40 if both is None else both + 1)
    c16.close()


def test_energy_every_sweep_and_energy_stop(lib):
    """E_CP after every sweep (formed from the tau the next sweep reuses)
    against the oracle's explicit sum per sweep; stop_rule 3 stops at the first
    sweep whose energy change is below tol; the trajectory is unchanged by
    evaluating the energy."""
    cfg = SMALL["odd"]
    _say("energy every sweep")
    inp, r = _problem(cfg)
    fs = synth.init_factors(cfg)
    _, _, hist = oracle.cp_als(r, fs, 12, norm_r2=float(np.sum(r * r)), t=inp.t)
    ctx = _ctx(lib, cfg, inp)
    ctx.set_factors(*fs)
    rep = ctx.als(12, energy_every=True)
    np.testing.assert_allclose(rep["energy_hist"], hist["energy"], rtol=1e-9, atol=0)
    np.testing.assert_allclose(rep["fit_hist"], hist["fit"], rtol=0, atol=1e-9)
    ctx.set_factors(*fs)
    plain = ctx.als(12)
    np.testing.assert_allclose(plain["fit_hist"], rep["fit_hist"], rtol=0, atol=1e-13)
    assert np.all(np.isnan(plain["energy_hist"]))
    e = np.asarray(hist["energy"])
    tol = float(np.median(np.abs(np.diff(e))))
    want = next(n for n in range(1, 12) if abs(e[n] - e[n - 1]) < tol)
    ctx.set_factors(*fs)
    r3 = ctx.als(12, stop_rule=3, tol=tol)
    assert r3["sweeps"] == want + 1
    np.testing.assert_allclose(r3["energy_hist"], e[:want + 1], rtol=1e-9, atol=0)
    # a BF16 context evaluates it from its bfloat16 tau: close, not exact
    c16 = _ctx(lib, cfg, inp, "bf16")
    c16.set_factors(*fs)
    r16 = c16.als(3, energy_every=True)
    assert np.all(np.isfinite(r16["energy_hist"]))
    assert abs(r16["energy_hist"][0] - e[0]) <= 2e-2 * abs(e[0])
    ctx.close()
    c16.close()


@pytest.mark.parametrize("sweep", [2, 3])
def test_early_alpha_fork_failure_recovery(lib, sweep):
    """The W_alpha inverse forked during sweep s-1 for sweep s reports a failed
    pivot (forced from the host through the test hook, so no kernel faults):
    the sweep issued ahead is dropped, sweep s is redone from its snapshot with
    the ridge rule, and the trajectory is the oracle's (status words 2 and 3
    alternate with the sweep parity, hence two sweeps)."""
    cfg = SMALL["ragged_tiles"]
    _say(f"early alpha fork failure at sweep {sweep}")
    inp, r = _problem(cfg)
    fs = synth.init_factors(cfg)
    _, _, hist = oracle.cp_als(r, fs, 6, norm_r2=float(np.sum(r * r)))
    ctx = _ctx(lib, cfg, inp)
    ctx.set_factors(*fs)
    ctx.inject_alpha_fault(sweep)
    rep = ctx.als(6)
    assert rep["careful_sweeps"] == 1
    assert rep["ridge_retries"] == 0  # the redo finds W positive definite
    np.testing.assert_allclose(rep["fit_hist"], hist["fit"], rtol=0, atol=1e-9)
    # the flag is consumed by that call
    ctx.set_factors(*fs)
    rep2 = ctx.als(6)
    assert rep2["careful_sweeps"] == 0
    np.testing.assert_allclose(rep2["fit_hist"], rep["fit_hist"], rtol=0, atol=1e-13)
    ctx.close()


@pytest.mark.timeout(600)
def test_als_trajectory_c2_30_sweeps(lib):
    """The C2 workload (o 16, v 128, X 384, R 512; R has 8 pivot blocks of W)
    over its 30 FP64 sweeps against the oracle's textbook ALS on the explicit R."""
    cfg = synth.CONFIGS["C2"]
    _say("C2 30-sweep trajectory")
    inp, r = _problem(cfg)
    fs = synth.init_factors(cfg)
    f_o, lam_o, hist = oracle.cp_als(r, fs, 30, norm_r2=float(np.sum(r * r)), t=inp.t)
    ctx = _ctx(lib, cfg, inp)
    ctx.set_factors(*fs)
    rep = ctx.als(30, energy_every=True)
    _say(f"  fit {rep['fit']:.10f} oracle {hist['fit'][-1]:.10f}")
    np.testing.assert_allclose(rep["fit_hist"], hist["fit"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(rep["energy_hist"], hist["energy"], rtol=1e-8, atol=0)
    got = ctx.get_factors()
    for g_, w_ in zip(got[:4], f_o):
        assert _rel(g_, w_) <= 1e-6
    assert _rel(got[4], lam_o) <= 1e-6
    ctx.close()


def test_als_trajectory_rank_1024(lib):
    """R = 1024: W and its inverse span 16 pivot blocks of 64; ten FP64 sweeps
    against the oracle on an explicit R (o 10, v 48, X 96)."""
    cfg = synth.custom_config(10, 48, 96, 1024, name="o10v48X96R1024")
    _say("rank 1024 trajectory")
    inp, r = _problem(cfg)
    fs = synth.init_factors(cfg)
    f_o, lam_o, hist = oracle.cp_als(r, fs, 10, norm_r2=float(np.sum(r * r)))
    ctx = _ctx(lib, cfg, inp)
    ctx.set_factors(*fs)
    rep = ctx.als(10)
    assert rep["ridge_retries"] == hist["retries"]
    np.testing.assert_allclose(rep["fit_hist"], hist["fit"], rtol=0, atol=1e-9)
    got = ctx.get_factors()
    for g_, w_ in zip(got[:4], f_o):
        assert _rel(g_, w_) <= 1e-6
    ctx.close()


def test_windowed_stop_rule(lib):
    """stop_window w: the main sweeps stop at the first n with
    |fit_n - fit_{n-w}| / w < tol, checked on the returned history."""
    cfg = SMALL["ragged_tiles"]
    _say("windowed stop rule")
    inp = synth.make_inputs(cfg)
    ctx = _ctx(lib, cfg, inp, "fp64")
    fs = synth.init_factors(cfg)
    ctx.set_factors(*fs)
    full = ctx.als(60)["fit_hist"]
    w, tol = 4, 2e-3
    want = next((n for n in range(w, 60) if abs(full[n] - full[n - w]) / w < tol), None)
    ctx.set_factors(*fs)
    r = ctx.als(60, stop_rule=1, tol=tol, stop_window=w)
    if want is None:
        assert r["sweeps"] == 60
    else:
        assert r["sweeps"] == want + 1
        np.testing.assert_allclose(r["fit_hist"], full[:want + 1], rtol=0, atol=1e-12)


def test_eta_stop_rule(lib):
    """stop_rule 2 (eq. N3_stopping): the sweeps stop at the first n with
    eta_n < tol, eta taken from a full run with eta evaluation switched on."""
    cfg = SMALL["odd"]
    _say("eta stop rule")
    inp = synth.make_inputs(cfg)
    ctx = _ctx(lib, cfg, inp, "fp64")
    fs = synth.init_factors(cfg)
    ctx.set_factors(*fs)
    eta = ctx.als(40, eta=True)["eta_hist"]
    tol = float(np.quantile(eta, 0.5))
    want = next(n for n in range(40) if eta[n] < tol)
    ctx.set_factors(*fs)
    r = ctx.als(40, stop_rule=2, tol=tol)
    assert r["sweeps"] == want + 1
    np.testing.assert_allclose(r["eta_hist"], eta[:want + 1], rtol=1e-12, atol=0)


def test_init_random_matches_oracle_generator(lib):
    """cpppl_init_random draws the paper's U[-1, 1] guess from counter-based
    SplitMix64: bitwise the oracle's draws, lambda = 1, and ALS from it follows
    the oracle's trajectory."""
    from oracle import rng
    cfg = SMALL["ragged_tiles"]
    _say("init_random")
    inp, r = _problem(cfg)
    ctx = _ctx(lib, cfg, inp)
    for seed in (0, 12345, 2 ** 63 + 5):
        ctx.init_random(seed)
        got = ctx.get_factors()
        want = rng.random_guess(cfg.o, cfg.v, cfg.rank, seed)
        for g, w in zip(got[:4], want):
            np.testing.assert_array_equal(g, w)
        np.testing.assert_array_equal(got[4], np.ones(cfg.rank))
    rep = ctx.als(5)
    _, _, hist = oracle.cp_als(r, want, 5, norm_r2=float(np.sum(r * r)))
    np.testing.assert_allclose(rep["fit_hist"], hist["fit"], rtol=0, atol=1e-9)
    ctx.close()


def test_bf16_sampled_columns_full_size(lib):
    """C3 sizes (o 32, v 256, X 768, R 1024) on the MP2-shaped inputs: sampled
    columns r of the BF16 MTTKRP (Y and Z on the B-resident kernel, tau, M, G
    and H on the tiled one) against the oracle's FP64 chain, within the derived
    element-wise and norm-wise bounds (a column of the MTTKRP depends on column
    r of the factors only)."""
    cfg = synth.CONFIGS["C3"]
    _say("bf16 sampled columns C3")
    inp = synth.make_inputs(cfg)
    fs = synth.init_factors(cfg)
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "bf16")
    ctx.load_t2(inp.t)
    ctx.load_df(inp.b_vv)
    ctx.set_factors(*fs)
    cols = [0, 377, cfg.rank - 1]
    sub = [f[:, cols] for f in fs]
    for mode in range(4):
        got = ctx.mttkrp(mode)[:, cols]
        want = oracle.mttkrp_chain(inp.t, inp.b_vv, sub, mode)
        err = assert_lowp(got, want, abs_chain(inp.t, inp.b_vv, sub, mode), N_ROUND_BF16,
                          chain_lengths(cfg.o, cfg.v, cfg.nx, mode), f"C3 mode {mode}")
        _say(f"  mode {mode}: rel err {err:.2e}")
    ctx.close()


def test_bf16_sampled_columns_full_size_c5(lib):
    """C5 sizes (o 48, v 384, X 1152, R 2048) on the MP2-shaped inputs: sampled
    columns r of the BF16 MTTKRP for one occupied and one virtual mode (Y and Z
    on the B-resident kernel's four-wave, 128-column work-groups at K = v = 384)
    against the oracle's FP64 chain, within the derived bounds."""
    cfg = synth.CONFIGS["C5"]
    _say("bf16 sampled columns C5")
    inp = synth.make_inputs(cfg)
    fs = synth.init_factors(cfg)
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "bf16")
    ctx.load_t2(inp.t)
    ctx.load_df(inp.b_vv)
    ctx.set_factors(*fs)
    cols = [0, 1023, cfg.rank - 1]
    sub = [f[:, cols] for f in fs]
    for mode in (0, 2):
        got = ctx.mttkrp(mode)[:, cols]
        want = oracle.mttkrp_chain(inp.t, inp.b_vv, sub, mode)
        err = assert_lowp(got, want, abs_chain(inp.t, inp.b_vv, sub, mode), N_ROUND_BF16,
                          chain_lengths(cfg.o, cfg.v, cfg.nx, mode), f"C5 mode {mode}")
        _say(f"  mode {mode}: rel err {err:.2e}")
    ctx.close()
