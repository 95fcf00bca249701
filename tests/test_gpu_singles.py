"""GPU parity of the singles-dressed PPL tensor (eq. B, eq. fulldfB, eq. dfB):
tau = t + t1 t1 in place of t and Dbar = D - 2 D_vo t1 on the b side, through
the C ABI (cpppl_load_singles), against the oracle's dressed R."""
import sys

import numpy as np
import pytest

import oracle
from oracle import fp8
import synth
from bounds import (N_ROUND_BF16, N_ROUND_FP8, abs_chain, assert_fp64, assert_lowp,
                    chain_lengths)

pytestmark = pytest.mark.gpu

SMALL = {
    "C1": synth.CONFIGS["C1"],
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
        t1, b_vo = synth.make_singles(inp)
        tau, bvv, dbar = oracle.dress(inp.t, t1, inp.b_full)
        r = oracle.form_r(tau, bvv, b_right=dbar)
        _CACHE[cfg.name] = (inp, t1, b_vo, tau, dbar, r)
    return _CACHE[cfg.name]


def _ctx(lib, cfg, inp, t1, b_vo, precision="fp64"):
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, precision, singles=True)
    ctx.load_t2(inp.t)
    ctx.load_df(inp.b_vv)
    ctx.load_singles(t1, b_vo)
    return ctx


@pytest.mark.parametrize("name", list(SMALL))
def test_singles_mttkrp_fp64(lib, name):
    cfg = SMALL[name]
    _say(f"singles mttkrp {name}")
    inp, t1, b_vo, tau, dbar, r = _problem(cfg)
    fs = synth.init_factors(cfg)
    ctx = _ctx(lib, cfg, inp, t1, b_vo)
    ctx.set_factors(*fs)
    for mode in range(4):
        assert_fp64(ctx.mttkrp(mode), oracle.mttkrp(r, fs, mode))
    n2, e = ctx.norm_r2()
    n2_o, e_o = oracle.norm_r2_and_energy(r, tau)
    assert n2 == pytest.approx(n2_o, rel=1e-12)
    assert e == pytest.approx(e_o, rel=1e-12)
    ctx.close()


@pytest.mark.parametrize("name", ["ragged_tiles", "odd"])
def test_singles_als_trajectory(lib, name):
    cfg = SMALL[name]
    _say(f"singles als {name}")
    inp, t1, b_vo, tau, dbar, r = _problem(cfg)
    fs = synth.init_factors(cfg)
    f_o, lam_o, hist = oracle.cp_als(r, fs, 8, norm_r2=float(np.sum(r * r)), t=tau)
    ctx = _ctx(lib, cfg, inp, t1, b_vo)
    ctx.set_factors(*fs)
    rep = ctx.als(8, energy=True)
    np.testing.assert_allclose(rep["fit_hist"], hist["fit"], rtol=0, atol=1e-9)
    assert rep["energy_cp"] == pytest.approx(hist["energy"][-1], rel=1e-8)
    fi, fj, fa, fb, lam = ctx.get_factors()
    for g_, w_ in zip((fi, fj, fa, fb), f_o):
        assert _rel(g_, w_) <= 1e-7
    ctx.close()


def test_singles_low_precision(lib):
    cfg = synth.custom_config(5, 40, 70, 70, name="o5v40X70R70")
    _say("singles bf16 / fp8")
    inp = synth.make_inputs(cfg)
    t1, b_vo = synth.make_singles(inp)
    tau, bvv, dbar = oracle.dress(inp.t, t1, inp.b_full)
    fs = synth.init_factors(cfg)
    tq, bq = fp8.fp8_inputs(tau, bvv)
    dq = fp8.dequantize_rows(*fp8.quantize_rows(dbar.reshape(cfg.nx, -1))).reshape(dbar.shape)
    for prec in ("bf16", "fp8"):
        ctx = _ctx(lib, cfg, inp, t1, b_vo, prec)
        ctx.set_factors(*fs)
        for mode in range(4):
            got = ctx.mttkrp(mode)
            ks = chain_lengths(cfg.o, cfg.v, cfg.nx, mode)
            if prec == "bf16":
                want = oracle.mttkrp_chain(tau, bvv, fs, mode, b_right=dbar)
                err = assert_lowp(got, want, abs_chain(tau, bvv, fs, mode, b_right=dbar),
                                  N_ROUND_BF16, ks, f"bf16 mode {mode}")
            else:
                want = oracle.mttkrp_chain(tq, bq, fs, mode, b_right=dq)
                err = assert_lowp(got, want, abs_chain(tq, bq, fs, mode, b_right=dq),
                                  N_ROUND_FP8, ks, f"fp8 mode {mode}")
            _say(f"  {prec} mode {mode}: {err:.2e}")
            assert_fp64(ctx.mttkrp(mode, "fp64"),
                        oracle.mttkrp_chain(tau, bvv, fs, mode, b_right=dbar))
        ctx.close()


def test_singles_removed_and_reloaded(lib):
    cfg = SMALL["ragged_tiles"]
    inp, t1, b_vo, tau, dbar, r = _problem(cfg)
    fs = synth.init_factors(cfg)
    ctx = _ctx(lib, cfg, inp, t1, b_vo)
    ctx.set_factors(*fs)
    dressed = [ctx.mttkrp(m) for m in range(4)]
    plain_ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "fp64")
    plain_ctx.load_t2(inp.t)
    plain_ctx.load_df(inp.b_vv)
    plain_ctx.set_factors(*fs)
    ctx.load_singles(None, None)
    for m in range(4):
        np.testing.assert_allclose(ctx.mttkrp(m), plain_ctx.mttkrp(m), rtol=1e-13, atol=1e-13)
    ctx.load_singles(t1, b_vo)
    ctx.load_t2(inp.t)       # the dressing stays with the context
    ctx.load_df(inp.b_vv)
    for m in range(4):
        np.testing.assert_allclose(ctx.mttkrp(m), dressed[m], rtol=1e-13, atol=1e-13)
    # a warm start adds dt to the doubles part: tau = (t + dt) + t1 t1
    dt = 1e-2 * synth.perturbation(cfg, 0, inp.t)
    ctx.warm_start(dt)
    r2 = oracle.form_r(tau + dt, inp.b_vv, b_right=dbar)
    for m in range(4):
        assert_fp64(ctx.mttkrp(m), oracle.mttkrp(r2, fs, m))
    ctx.close()
    plain_ctx.close()


def test_singles_errors(lib):
    cfg = SMALL["C1"]
    inp, t1, b_vo, *_ = _problem(cfg)
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "fp64")
    ctx.load_t2(inp.t)
    ctx.load_df(inp.b_vv)
    with pytest.raises(lib.CppplError) as e:
        ctx.load_singles(t1, b_vo)
    assert e.value.status == -7
    ctx.close()
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "fp64", singles=True)
    with pytest.raises(lib.CppplError) as e:
        ctx.load_singles(t1, b_vo)
    assert e.value.status == -2
    ctx.close()


@pytest.mark.parametrize("cfg_name", ["C3"])
def test_singles_full_size_rank1_tau_closed_form(lib, cfg_name):
    """At full size: t2 = 0 and t1 = u p^T make tau = u u p p, so R is the
    rank-X CP tensor (u, u, B p, Dbar p): closed-form MTTKRPs, FP64 and BF16."""
    cfg = synth.CONFIGS[cfg_name]
    _say(f"singles closed form {cfg_name}")
    rng = np.random.default_rng(cfg.cfg_id)
    n = cfg.o + cfg.v
    b = rng.standard_normal((cfg.nx, n, n)) / np.sqrt(cfg.nx)
    b = 0.5 * (b + b.transpose(0, 2, 1))
    t1, (u, p) = synth.rank1_singles(cfg)
    t2 = np.zeros((cfg.o, cfg.o, cfg.v, cfg.v))
    _, bvv, dbar = oracle.dress(t2[:1, :1], t1, b)  # Dbar only (tau is not formed here)
    cf = oracle.rank1_closed_form(u, u, p, p, bvv, dbar)
    cf_abs = oracle.rank1_closed_form(np.abs(u), np.abs(u), np.abs(p), np.abs(p), np.abs(bvv),
                                      np.abs(dbar))
    fs = synth.init_factors(cfg)
    fs_abs = [np.abs(f) for f in fs]
    b_vo = np.ascontiguousarray(b[:, cfg.o:, :cfg.o])
    for prec in ("fp64", "bf16"):
        ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, prec, singles=True)
        ctx.load_t2(t2)
        ctx.load_df(np.ascontiguousarray(bvv))
        ctx.load_singles(t1, b_vo)
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
