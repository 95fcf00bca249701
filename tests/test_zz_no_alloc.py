"""cpppl_mttkrp_noalloc (the entry point for callers that cannot allocate)
against cpppl_mttkrp of a context, through the C ABI: two calls in a row on
the same device array, the second with a smaller problem, every mode, element
by element; a problem larger than the array is refused before any work."""
import sys

import numpy as np
import pytest

import synth
from bounds import assert_fp64

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(lib, cfg, torch):
    inp = synth.make_inputs(cfg)
    fs = synth.init_factors(cfg)
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "fp64")
    ctx.load_t2(inp.t)
    ctx.load_df(inp.b_vv)
    ctx.set_factors(*fs)
    dev = [torch.tensor(x, device="cuda") for x in (inp.t, inp.b_vv, *fs)]
    for mode in range(4):
        want = ctx.mttkrp(mode)
        got = lib.mttkrp_noalloc(*dev, mode)
        torch.cuda.synchronize()
        assert_fp64(got.cpu().numpy(), want, rtol=1e-12)
    ctx.close()


def test_noalloc_matches_context_twice(lib):
    import torch
    big = synth.custom_config(6, 40, 90, 70, name="o6v40X90R70")
    small = synth.custom_config(3, 10, 7, 5, name="o3v10X7R5")
    for cfg in (big, small):
        _say(f"noalloc {cfg.name}")
        _run(lib, cfg, torch)


def test_noalloc_refuses_oversized_problem(lib):
    import ctypes as C
    import torch
    L = lib.load_library()
    d = lib.Dims(32, 256, 768, 1024, 0)   # tau alone is 512 MiB
    x = torch.zeros(8, dtype=torch.float64, device="cuda")
    p = C.c_void_p(x.data_ptr())
    st = L.cpppl_mttkrp_noalloc(C.byref(d), p, p, p, p, p, p, 2, p, None)
    assert st == -4  # CPPPL_E_NOMEM, nothing enqueued
    assert L.cpppl_mttkrp_noalloc(C.byref(d), p, p, p, p, p, p, 7, p, None) == -1
