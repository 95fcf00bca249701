"""The synthetic CCD-like Jacobi iteration on the GPU (cpppl_jacobi_step with
ALS and the warm starts between CC steps) against the oracle's loop
(oracle.ccd) at C1, for the paper's three initial guesses: per CC step the
ALS sweep count, the fit and the amplitude change dt, element by element."""
import sys

import numpy as np
import pytest

import oracle
from oracle import ccd
import synth
from bounds import assert_fp64

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def c1():
    cfg = synth.CONFIGS["C1"]
    inp = synth.make_inputs(cfg)
    return cfg, inp, synth.exchange_integrals(inp), synth.ccd_scale(inp)


def test_jacobi_step_matches_oracle(lib, c1):
    """One step from given factors: dt = (w + s sym(CP)) / D - t, host and device."""
    import torch
    cfg, inp, w, s = c1
    fs = synth.init_factors(cfg)
    lam = np.linspace(0.5, 1.5, cfg.rank)
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "fp64")
    ctx.load_t2(inp.t)
    ctx.load_df(inp.b_vv)
    ctx.set_factors(*fs, lam)
    want = ccd.jacobi_update(w, oracle.symmetrize_pairs(oracle.cp_full(fs, lam)), inp.e_occ,
                             inp.e_vir, s) - inp.t
    assert_fp64(ctx.jacobi_step(w, inp.e_occ, inp.e_vir, s), want, rtol=1e-12)
    dev = [torch.tensor(x, device="cuda") for x in (w, inp.e_occ, inp.e_vir)]
    got = ctx.jacobi_step(*dev, s)
    assert_fp64(got.cpu().numpy(), want, rtol=1e-12)
    # scale 0: the MP2 amplitudes minus t, i.e. zero at t = w / D
    np.testing.assert_allclose(ctx.jacobi_step(w, inp.e_occ, inp.e_vir, 0.0), 0.0, atol=1e-15)
    ctx.close()


@pytest.mark.parametrize("guess", ["random", "optimal", "near_optimal"])
def test_ccd_loop_matches_oracle(lib, c1, guess):
    import torch
    cfg, inp, w, s = c1
    _say(f"ccd loop {guess}")
    steps, seed = 5, 3
    t_o, hist_o = ccd.ccd_loop(w, inp.b_vv, inp.e_occ, inp.e_vir, s, steps, cfg.rank, guess=guess,
                               seed=seed)
    ts = [w / ccd.denominators(inp.e_occ, inp.e_vir)]
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "fp64")
    ctx.load_t2(ts[0])
    ctx.load_df(inp.b_vv)
    dev = [torch.tensor(x, device="cuda") for x in (w, inp.e_occ, inp.e_vir)]
    dts = []
    hist = lib.ccd_loop(ctx, *dev, s, steps, guess=guess, seed=seed,
                        on_step=lambda k, dt, rec: dts.append(dt.cpu().numpy()))
    t_gpu = ts[0] + np.sum(dts, axis=0)
    for k, (h, ho) in enumerate(zip(hist, hist_o)):
        _say(f"  step {k + 1}: sweeps {h['sweeps']} / {ho['sweeps']}, fit {h['fit']:.10f} / "
             f"{ho['fit']:.10f}, guess {h['guess']} / {ho['guess']}")
        assert h["guess"] == ho["guess"]
        assert h["sweeps"] == ho["sweeps"]
        assert abs(h["fit"] - ho["fit"]) <= 1e-8
        assert ho["dt_norm"] == pytest.approx(float(np.linalg.norm(dts[k])), rel=1e-6)
    np.testing.assert_allclose(t_gpu, t_o, rtol=0, atol=1e-7 * np.abs(t_o).max())
    ctx.close()
