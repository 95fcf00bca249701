"""GPU reconstruction of the CP tensor and its pair symmetrisation
(cpppl_reconstruct) against the oracle's explicit CP tensor."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("shape", [(4, 16, 48, 32), (5, 33, 70, 70), (7, 19, 61, 131)])
def test_reconstruct_small(lib, shape):
    import torch
    o, v, nx, rank = shape
    cfg = synth.custom_config(o, v, nx, rank)
    _say(f"reconstruct {cfg.name}")
    inp = synth.make_inputs(cfg)
    ctx = lib.Context(o, v, nx, rank, "fp64")
    ctx.load_t2(inp.t)
    ctx.load_df(inp.b_vv)
    ctx.set_factors(*synth.init_factors(cfg))
    ctx.als(3)
    fi, fj, fa, fb, lam = ctx.get_factors()
    want = oracle.cp_full((fi, fj, fa, fb), lam)
    got = ctx.reconstruct()
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    sym = ctx.reconstruct(symmetrize=True)
    np.testing.assert_allclose(sym, oracle.symmetrize_pairs(want), rtol=0,
                               atol=1e-12 * np.abs(want).max())
    np.testing.assert_array_equal(sym, sym.transpose(1, 0, 3, 2))
    # device output
    dev = torch.empty((o, o, v, v), dtype=torch.float64, device="cuda")
    ctx.reconstruct(symmetrize=True, out=dev)
    np.testing.assert_array_equal(dev.cpu().numpy(), sym)
    # E_CP does not see the symmetrisation (t is pair symmetric)
    assert np.sum(sym * inp.t) == pytest.approx(ctx.energy(), rel=1e-10)
    ctx.close()


def test_reconstruct_full_size_sampled(lib):
    """C3 sizes: sampled entries against sum_r lambda_r gamma rho alpha beta."""
    cfg = synth.CONFIGS["C3"]
    _say("reconstruct C3 sampled")
    fs = synth.planted_factors(cfg, 64)
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "fp64")
    ctx.load_planted(*fs)
    init = synth.init_factors(cfg)
    lam = np.linspace(0.5, 1.5, cfg.rank)
    ctx.set_factors(*init, lam)
    full = ctx.reconstruct()
    sym = ctx.reconstruct(symmetrize=True)
    rng = np.random.default_rng(3)
    idx = [tuple(int(rng.integers(0, n)) for n in (cfg.o, cfg.o, cfg.v, cfg.v)) for _ in range(200)]
    g, r, a, b = init
    for (i, j, x, y) in idx:
        want = float(np.sum(lam * g[i] * r[j] * a[x] * b[y]))
        want_t = float(np.sum(lam * g[j] * r[i] * a[y] * b[x]))
        assert abs(full[i, j, x, y] - want) <= 1e-12 * (1 + abs(want))
        assert abs(sym[i, j, x, y] - 0.5 * (want + want_t)) <= 1e-12 * (1 + abs(want) + abs(want_t))
    ctx.close()
