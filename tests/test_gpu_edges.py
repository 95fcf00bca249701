"""Edge cases of the HIP path against the oracle: degenerate mode sizes (one
occupied orbital, one virtual orbital, one auxiliary function), rank one, the
largest rank the library accepts, and an all-zero amplitude tensor (for which
the fit is undefined and the call must fail cleanly)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from bounds import N_ROUND_BF16, abs_chain, assert_fp64, assert_lowp, chain_lengths

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


EDGES = {
    "o1": (1, 12, 9, 6),
    "v1": (3, 1, 5, 4),
    "x1": (3, 7, 1, 5),
    "rank1": (4, 9, 11, 1),
    "tiny": (1, 1, 1, 1),
}


@pytest.mark.parametrize("name", list(EDGES))
def test_edge_shapes(lib, name):
    o, v, nx, rank = EDGES[name]
    cfg = synth.custom_config(o, v, nx, rank, name=name)
    _say(f"edge {name} {EDGES[name]}")
    inp = synth.make_inputs(cfg)
    r = oracle.form_r(inp.t, inp.b_vv)
    fs = synth.init_factors(cfg)
    for prec in ("fp64", "bf16"):
        ctx = lib.Context(o, v, nx, rank, prec)
        ctx.load_t2(inp.t)
        ctx.load_df(inp.b_vv)
        ctx.set_factors(*fs)
        for mode in range(4):
            got, want = ctx.mttkrp(mode), oracle.mttkrp(r, fs, mode)
            if prec == "fp64":
                assert_fp64(got, want)
            else:
                assert_lowp(got, want, abs_chain(inp.t, inp.b_vv, fs, mode), N_ROUND_BF16,
                            chain_lengths(o, v, nx, mode), f"{name} mode {mode}",
                            normwise_check=False)
        n2, e = ctx.norm_r2()
        assert n2 == pytest.approx(float(np.sum(r * r)), rel=1e-12)
        if prec == "fp64" and rank <= max(o, v):
            rep = ctx.als(3)
            _, _, hist = oracle.cp_als(r, fs, 3)
            # an exact fit (here the 1 x 1 x 1 x 1 case) is resolved by the
            # residual identity only to ~sqrt(eps): 1e-7 there (reading P4)
            atol = 1e-7 if max(hist["fit"]) > 1 - 1e-6 else 1e-9
            np.testing.assert_allclose(rep["fit_hist"], hist["fit"], rtol=0, atol=atol)
        ctx.close()


def test_max_rank_mttkrp(lib):
    """R = 4096, the largest rank accepted: the MTTKRP chain of every mode; 4097 is refused."""
    cfg = synth.custom_config(3, 8, 10, 4096, name="o3v8X10R4096")
    _say("rank 4096")
    inp = synth.make_inputs(cfg)
    r = oracle.form_r(inp.t, inp.b_vv)
    fs = synth.init_factors(cfg)
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "fp64")
    ctx.load_t2(inp.t)
    ctx.load_df(inp.b_vv)
    ctx.set_factors(*fs)
    for mode in range(4):
        assert_fp64(ctx.mttkrp(mode), oracle.mttkrp(r, fs, mode))
    with pytest.raises(lib.CppplError):
        lib.Context(cfg.o, cfg.v, cfg.nx, 4097, "fp64")
    ctx.close()


def test_zero_amplitudes_fail_cleanly(lib):
    """t = 0 makes R = 0: ||R|| = 0 leaves the fit undefined and W singular;
    the library reports an error instead of returning numbers."""
    cfg = synth.custom_config(3, 8, 10, 4, name="zero")
    inp = synth.make_inputs(cfg)
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "fp64")
    ctx.load_t2(np.zeros_like(inp.t))
    ctx.load_df(inp.b_vv)
    ctx.set_factors(*synth.init_factors(cfg))
    assert ctx.norm_r2() == (0.0, 0.0)
    for mode in range(4):
        assert not np.any(ctx.mttkrp(mode))
    with pytest.raises(lib.CppplError) as e:
        ctx.als(2)
    assert e.value.status in (-5, -6)  # E_NOT_SPD or E_NONFINITE
    ctx.close()
