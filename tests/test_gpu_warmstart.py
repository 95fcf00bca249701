"""Warm starts across a CCSD-like amplitude sequence, through the C ABI.

Pinned against the oracle: the amplitude update t <- t + dt, the features
(previous factor columns and the first-order change M(dR) W^{-1} / lambda of
each factor, with M(dR) the textbook MTTKRP of the explicitly formed PPL
tensor of dt), the training targets, and the judge (a non-plain candidate is
kept only when ||CP||^2 - 2 <R, CP> is lower).  The size of the learned
network's gain is reported; it is not a pinned quantity.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from bounds import assert_fp64

pytestmark = pytest.mark.gpu

CFG = synth.custom_config(6, 24, 72, 40, name="ws_small")


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _ctx(lib, cfg, t, b, precision="fp64"):
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, precision)
    ctx.load_t2(t)
    ctx.load_df(b)
    return ctx


def _gram_w(fs, mode):
    return oracle.gram_hadamard(fs, mode)


def test_plain_warm_start_advances_t_and_keeps_factors(lib):
    cfg = CFG
    inp = synth.make_inputs(cfg)
    fs = synth.init_factors(cfg)
    dt = synth.perturbation(cfg, 0, inp.t)
    ctx = _ctx(lib, cfg, inp.t, inp.b_vv)
    ctx.set_factors(*fs)
    assert ctx.warm_start(dt, lib.WS_PLAIN) == lib.WS_PLAIN
    got = ctx.get_factors()
    for a, b in zip(got[:4], fs):
        np.testing.assert_array_equal(a, b)
    r_new = oracle.form_r(inp.t + dt, inp.b_vv)
    for mode in range(4):
        want = oracle.mttkrp(r_new, fs, mode)
        assert_fp64(ctx.mttkrp(mode), want)
    n2, e = ctx.norm_r2()
    assert n2 == pytest.approx(float(np.sum(r_new * r_new)), rel=1e-12)


def test_features_and_targets_match_oracle(lib):
    cfg = CFG
    _say("warm-start features")
    inp = synth.make_inputs(cfg)
    r0 = oracle.form_r(inp.t, inp.b_vv)
    f0, lam0, _ = oracle.cp_als(r0, synth.init_factors(cfg), 8)
    dt = synth.perturbation(cfg, 1, inp.t)
    ctx = _ctx(lib, cfg, inp.t, inp.b_vv)
    ctx.set_factors(*f0, lam0)
    net = lib.MLP(ctx.ws_in_dim, ctx.ws_out_dim, capacity=cfg.rank)
    ctx.warm_start(dt, lib.WS_PLAIN)
    rep = ctx.als(5)
    ctx.training_rows(net)
    x, y = net.get_rows()
    assert x.shape == (cfg.rank, ctx.ws_in_dim)
    # previous columns, mode order (i, j, a, b)
    prev = np.concatenate([f.T for f in f0], axis=1)
    np.testing.assert_allclose(x[:, :ctx.ws_out_dim], prev, rtol=1e-6, atol=1e-7)
    # first-order change of every factor from the MTTKRP of dR
    rd = oracle.form_r(dt, inp.b_vv)
    d = []
    for mode in range(4):
        m = oracle.mttkrp(rd, f0, mode)
        d.append((m @ np.linalg.inv(_gram_w(f0, mode))) / lam0)
    d = np.concatenate([q.T for q in d], axis=1)
    nd = ctx.ws_out_dim
    got = x[:, nd:2 * nd]
    assert np.abs(got - d).max() <= 1e-5 * np.abs(d).max()
    # the last feature: log10 of the relative step ||dt|| / ||t||
    np.testing.assert_allclose(x[:, -1], np.log10(np.linalg.norm(dt) / np.linalg.norm(inp.t)),
                               rtol=1e-6)
    # targets: sign-aligned converged column - previous column - first-order change
    fi, fj, fa, fb, _ = ctx.get_factors()
    new = [fi, fj, fa, fb]
    tgt = []
    for f1, f0m in zip(new, f0):
        sg = np.sign(np.sum(f1 * f0m, axis=0))
        sg[sg == 0] = 1
        tgt.append((f1 * sg - f0m).T)
    tgt = np.concatenate(tgt, axis=1) - d
    assert np.abs(y - tgt).max() <= 1e-5 * max(1e-3, np.abs(tgt).max())
    assert rep["sweeps"] == 5
    # standardisation: per-column mean / std of x and rms of y, applied to the rows
    xr, yr = x.astype(np.float64), y.astype(np.float64)
    net.standardize()
    mu, inv, sc = net.standardization()
    sd = xr.std(axis=0)
    flat = ~(sd > 1e-30 * (1 + np.abs(xr.mean(axis=0))))
    np.testing.assert_allclose(mu, xr.mean(axis=0), rtol=1e-5, atol=1e-7 * np.abs(xr).max())
    np.testing.assert_allclose(inv[~flat], 1.0 / sd[~flat], rtol=1e-4)
    assert np.all(inv[flat] == 1.0)
    rms = np.sqrt(np.mean(yr * yr, axis=0))
    np.testing.assert_allclose(sc, np.where(rms > 0, rms, 1.0), rtol=1e-4)
    xs, ys = net.get_rows()
    np.testing.assert_allclose(xs, (xr - mu) * inv, rtol=1e-4, atol=1e-4)
    np.testing.assert_allclose(ys, yr / sc, rtol=1e-4, atol=1e-5)
    with pytest.raises(lib.CppplError):
        net.standardize()


def test_first_order_candidate_is_judged(lib):
    cfg = CFG
    _say("first-order judge")
    inp = synth.make_inputs(cfg)
    r0 = oracle.form_r(inp.t, inp.b_vv)
    f0, lam0, _ = oracle.cp_als(r0, synth.init_factors(cfg), 30)
    dt = synth.perturbation(cfg, 2, inp.t)
    r1 = oracle.form_r(inp.t + dt, inp.b_vv)
    ctx = _ctx(lib, cfg, inp.t, inp.b_vv)
    ctx.set_factors(*f0, lam0)
    chosen = ctx.warm_start(dt, lib.WS_FIRST_ORDER)
    fi, fj, fa, fb, lam = ctx.get_factors()
    cand = oracle.cp_full((fi, fj, fa, fb), lam)
    plain = oracle.cp_full(f0, lam0)
    l_cand = np.sum(cand * cand) - 2 * np.sum(r1 * cand)
    l_plain = np.sum(plain * plain) - 2 * np.sum(r1 * plain)
    assert l_cand <= l_plain + 1e-9 * abs(l_plain)
    if chosen == lib.WS_PLAIN:
        for a, b in zip((fi, fj, fa, fb), f0):
            np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)
    _say(f"  chosen={chosen} L_plain={l_plain:.6e} L_cand={l_cand:.6e}")


def _sweeps_to(fits, target, rel=1e-4):
    for k, f in enumerate(fits):
        if abs(f - target) <= rel * abs(target):
            return k + 1
    return len(fits) + 1


def test_learned_warm_start_sequence(lib):
    """Train on the warm starts of steps 1-6 of an amplitude sequence, evaluate
    plain / first-order / learned on steps 7-10 from the same converged start."""
    cfg = CFG
    _say("learned warm-start sequence")
    inp = synth.make_inputs(cfg)
    ts = [inp.t] + list(synth.amplitude_sequence(cfg, inp.t, 10, period=6))
    ctx = _ctx(lib, cfg, ts[0], inp.b_vv)
    ctx.set_factors(*synth.init_factors(cfg))
    ctx.als(400, stop_rule=1, tol=1e-9)
    net = lib.MLP(ctx.ws_in_dim, ctx.ws_out_dim, capacity=10 * cfg.rank, seed=5)
    for k in range(1, 7):
        ctx.warm_start(ts[k] - ts[k - 1], lib.WS_PLAIN)
        ctx.als(400, stop_rule=1, tol=1e-9)
        ctx.training_rows(net)
    net.standardize()
    hist = net.train(300, lr=1e-3, batch=64, seed=1)
    assert hist[-1] < hist[0]
    report = []
    for k in range(7, 11):
        state = ctx.get_factors()
        res = {}
        for name, strat in (("plain", lib.WS_PLAIN), ("first_order", lib.WS_FIRST_ORDER),
                            ("learned", lib.WS_LEARNED)):
            ctx.load_t2(ts[k - 1])
            ctx.set_factors(*state)
            chosen = ctx.warm_start(ts[k] - ts[k - 1], strat, net if strat == lib.WS_LEARNED else None)
            rep = ctx.als(400, stop_rule=1, tol=1e-9)
            res[name] = (chosen, rep["fit_hist"])
        target = res["plain"][1][-1]
        # (chosen, sweeps to within 1e-4 of the plain converged fit, sweeps to
        #  |dfit| < 1e-9, gap of the first-sweep fit, final fit)
        row = {n: (c, _sweeps_to(h, target), len(h), abs(h[0] - target) / abs(target), h[-1])
               for n, (c, h) in res.items()}
        report.append(row)
        _say(f"  step {k}: " + ", ".join(
            f"{n}: chosen={c} to1e-4={s} converged={nc} gap1={g:.2e}"
            for n, (c, s, nc, g, f) in row.items()))
        # every warm start converges to the same fit within the stopping noise
        for n, (c, s, nc, g, f) in row.items():
            assert abs(f - target) <= 1e-4 * abs(target)
        ctx.load_t2(ts[k - 1])
        ctx.set_factors(*state)
        ctx.warm_start(ts[k] - ts[k - 1], lib.WS_PLAIN)
        ctx.als(400, stop_rule=1, tol=1e-9)
    for idx, what in ((1, "sweeps to within 1e-4"), (2, "sweeps to |dfit|<1e-9"),
                      (3, "first-sweep fit gap")):
        mean = {n: float(np.mean([r[n][idx] for r in report])) for n in report[0]}
        _say(f"  mean {what}: {mean}")


def test_near_optimal_cache(lib):
    """The near-optimal guess: an ALS call of n > 5 sweeps caches its (n-5)th
    iterate; a call of n <= 5 sweeps keeps the old cache; the warm start
    NEAR_OPTIMAL installs the cache (PLAIN while none exists)."""
    cfg = CFG
    _say("near-optimal cache")
    inp = synth.make_inputs(cfg)
    fs = synth.init_factors(cfg)
    zero = np.zeros_like(inp.t)
    ctx = _ctx(lib, cfg, inp.t, inp.b_vv)
    ctx.set_factors(*fs)
    assert ctx.warm_start(zero, lib.WS_NEAR_OPTIMAL) == lib.WS_PLAIN
    for a, b in zip(ctx.get_factors()[:4], fs):
        np.testing.assert_array_equal(a, b)
    ctx.als(3)
    f3 = ctx.get_factors()
    ctx.set_factors(*fs)
    ctx.als(8, near_cache=True)
    assert ctx.warm_start(zero, lib.WS_NEAR_OPTIMAL) == lib.WS_NEAR_OPTIMAL
    for a, b in zip(ctx.get_factors(), f3):
        np.testing.assert_array_equal(a, b)
    ctx.als(4, near_cache=True)  # too short: the cache stays the 3rd iterate
    assert ctx.warm_start(zero, lib.WS_NEAR_OPTIMAL) == lib.WS_NEAR_OPTIMAL
    for a, b in zip(ctx.get_factors(), f3):
        np.testing.assert_array_equal(a, b)


def _judge_loss(ctx):
    _, inner, cp2 = ctx.fit()
    return cp2 - 2.0 * inner


def test_learned_warm_start_gain(lib):
    """What the trained network gains over the warm start without it, on an
    amplitude sequence whose step sizes repeat with period 5 (0.3^(k mod 5)
    times 1e-2 ||t||): trained on steps 1-8 (ALS converged to |dfit| < 1e-7 from
    the plain start), its standardised training loss falls at least 10x; on
    steps 9-12 the start the judge keeps is never worse than the plain one
    (nor, for the learned strategy, than the first-order one), and the
    reduction of the initial loss gap (L_plain - L) / (L_plain - L*), with L*
    the loss of the converged plain run, is reported for both strategies."""
    cfg = CFG
    _say("learned warm-start gain")
    inp = synth.make_inputs(cfg)
    ts = [inp.t] + list(synth.amplitude_sequence(cfg, inp.t, 12, period=5))
    ctx = _ctx(lib, cfg, ts[0], inp.b_vv)
    ctx.set_factors(*synth.init_factors(cfg))
    ctx.als(400, stop_rule=1, tol=1e-8)
    net = lib.MLP(ctx.ws_in_dim, ctx.ws_out_dim, capacity=8 * cfg.rank, seed=5)
    for k in range(1, 9):
        ctx.warm_start(ts[k] - ts[k - 1], lib.WS_PLAIN)
        ctx.als(300, stop_rule=1, tol=1e-7)
        ctx.training_rows(net)
    net.standardize()
    hist = net.train(400, lr=1e-3, batch=64, seed=1)
    _say(f"  training loss {hist[0]:.4e} -> {hist[-1]:.4e} ({hist[0] / hist[-1]:.1f}x)")
    assert hist[-1] <= 0.1 * hist[0]
    gains = {"learned": [], "first_order": []}
    picks = []
    for k in range(9, 13):
        state = ctx.get_factors()
        ctx.load_t2(ts[k - 1])
        ctx.set_factors(*state)
        ctx.warm_start(ts[k] - ts[k - 1], lib.WS_PLAIN)
        l_plain = _judge_loss(ctx)
        ctx.als(300, stop_rule=1, tol=1e-7)
        l_star = _judge_loss(ctx)
        converged = ctx.get_factors()
        l_start = {}
        for name, strat in (("first_order", lib.WS_FIRST_ORDER), ("learned", lib.WS_LEARNED)):
            ctx.load_t2(ts[k - 1])
            ctx.set_factors(*state)
            chosen = ctx.warm_start(ts[k] - ts[k - 1], strat, net if strat == lib.WS_LEARNED else None)
            l_start[name] = _judge_loss(ctx)
            # the judge never keeps a worse start than the plain one ...
            assert l_start[name] <= l_plain + 1e-12 * abs(l_plain)
            gains[name].append((l_plain - l_start[name]) / max(l_plain - l_star, 1e-300))
            if strat == lib.WS_LEARNED:
                picks.append(chosen)
            _say(f"  step {k} {name}: chosen={chosen} gap reduction {gains[name][-1]:.3e}")
        # ... and the learned one never a worse start than the first-order one
        assert l_start["learned"] <= l_start["first_order"] + 1e-12 * abs(l_plain)
        # continue the sequence from the converged plain run
        ctx.load_t2(ts[k])
        ctx.set_factors(*converged)
    for name, g in gains.items():
        _say(f"  {name}: mean reduction of the initial loss gap {np.mean(g):.3e}")
    _say(f"  learned strategy kept: {picks} (0 plain, 2 first order, 1 network)")
