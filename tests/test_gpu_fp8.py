"""GPU checks of the FP8 (OCP e4m3) ablation path against the oracle's e4m3
definition (oracle.fp8) and the FP64 oracle:
 * the loader's conversion of every finite code times power-of-two scales (exact);
 * row quantisation with power-of-two scales (codes and scales bit-exact);
 * the BF16 GEMM with an e4m3 B operand in every scale mode, with ragged tiles,
   batches, split-K and both K-slice variants, against numpy in FP64 on the
   dequantised values;
 * the FP8 MTTKRP of every mode against the oracle's chain on the dequantised t
   and B (the BF16-path tolerance) and against the exact MTTKRP;
 * FP64 refinement sweeps of an FP8 context against an FP64 context.
"""
import ctypes as C
import sys

import numpy as np
import pytest

import zlib

import oracle
from oracle import fp8
import synth
from bounds import N_ROUND_FP8, abs_chain, assert_fp64, assert_lowp, chain_lengths, normwise

pytestmark = pytest.mark.gpu

FINITE = np.array([c for c in range(256) if c not in fp8.NAN_CODES], dtype=np.uint8)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def env(lib):
    import torch
    L = lib.load_library()
    L.cpppl_test_gemm_e4m3b.restype = C.c_int
    L.cpppl_test_gemm_e4m3b.argtypes = [C.c_int64] * 4 + [C.c_void_p] + [C.c_int64] * 3 + \
        [C.c_void_p] + [C.c_int64] * 2 + [C.c_void_p, C.c_int, C.c_void_p] + [C.c_int64] * 2 + \
        [C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    L.cpppl_test_quantize_e4m3.restype = C.c_int
    L.cpppl_test_quantize_e4m3.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                           C.c_void_p]
    L.cpppl_test_dequant_e4m3.restype = C.c_int
    L.cpppl_test_dequant_e4m3.argtypes = [C.c_void_p, C.c_int64, C.c_float, C.c_void_p, C.c_void_p]
    return L, torch


def _stream(torch):
    return torch.cuda.current_stream().cuda_stream


@pytest.mark.parametrize("scale", [1.0, 2.0 ** -5, 2.0 ** 10, 2.0 ** -100, 2.0 ** 100])
def test_dequant_every_code(env, scale):
    L, torch = env
    _say(f"dequant scale {scale}")
    codes = np.zeros(256, dtype=np.uint8)
    codes[:len(FINITE)] = FINITE
    tq = torch.tensor(codes, dtype=torch.uint8).cuda()
    out = torch.zeros(256, dtype=torch.bfloat16, device="cuda")
    assert L.cpppl_test_dequant_e4m3(tq.data_ptr(), 256, scale, out.data_ptr(), _stream(torch)) == 0
    got = out.cpu().to(torch.float64).numpy()[:len(FINITE)]
    want = fp8.e4m3_decode(FINITE) * scale
    np.testing.assert_array_equal(got, want)


def _quantize_gpu(L, torch, x):
    rows, n = x.shape
    tx = torch.tensor(x.reshape(-1)).cuda()
    tq = torch.zeros(rows * n, dtype=torch.uint8, device="cuda")
    ts = torch.zeros(rows, dtype=torch.float32, device="cuda")
    assert L.cpppl_test_quantize_e4m3(tx.data_ptr(), rows, n, tq.data_ptr(), ts.data_ptr(),
                                      _stream(torch)) == 0
    return tq.cpu().numpy().reshape(rows, n), ts.cpu().numpy().astype(np.float64)


def test_quantize_rows_bit_exact(env):
    L, torch = env
    _say("quantize rows")
    cfg = synth.custom_config(5, 16, 40, 8, name="o5v16")
    inp = synth.make_inputs(cfg)
    t_rows = inp.t.reshape(25, 256)
    pos = fp8.e4m3_decode(np.arange(0, 0x7F, dtype=np.uint8))
    mids = 0.5 * (pos[:-1] + pos[1:])
    special = np.zeros((6, 256))
    special[0, :126] = mids * 2.0 ** -3          # exact ties, scale 2^-3 (max below)
    special[0, 200] = 448.0 * 2.0 ** -3
    special[0, 201:] = -mids[:55] * 2.0 ** -3
    special[1, :] = 0.0                           # all zero: scale 1
    special[2, :] = np.linspace(-1e-200, 1e-200, 256)   # scale clamped at 2^-126
    special[3, :] = np.linspace(-3e38, 1e42, 256)       # scale clamped at 2^127, saturation
    special[4, :] = np.linspace(-448.0, 447.0, 256)
    special[5, :] = np.random.default_rng(5).standard_normal(256) * 1e-3
    for x in (t_rows, special, inp.b_vv.reshape(cfg.nx, -1)):
        q, s = _quantize_gpu(L, torch, x)
        q_o, s_o = fp8.quantize_rows(x)
        np.testing.assert_array_equal(s, s_o)
        np.testing.assert_array_equal(q, q_o)


GEMM_CASES = [
    # (M, N, K, batch, splits, pad)
    (70, 45, 37, 1, 1, 3),
    (129, 131, 200, 2, 1, 8),
    (33, 257, 300, 1, 4, 0),
    (130, 200, 4104, 1, 1, 8),     # K slice of 64
    (5, 3, 1, 3, 1, 1),
    (64, 128, 64, 1, 1, 0),
]


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("ak", [True, False])
@pytest.mark.parametrize("ctype", [0, 1])
@pytest.mark.parametrize("case", GEMM_CASES)
def test_gemm_e4m3_b(env, mode, ak, ctype, case):
    L, torch = env
    M, N, K, batch, splits, pad = case
    _say(f"gemm e4m3 mode={mode} ak={ak} ctype={ctype} case={case}")
    rng = np.random.default_rng(zlib.crc32(repr((M, N, K, batch, mode, ak)).encode()))
    a = rng.standard_normal((batch, M, K))
    a = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    if ak:
        sam, sak = K + pad, 1
        store_a = np.zeros((batch, M, K + pad))
        store_a[:, :, :K] = a
    else:
        sam, sak = 1, M + pad
        store_a = np.zeros((batch, K, M + pad))
        store_a[:, :, :M] = a.transpose(0, 2, 1)
    sab = store_a.shape[1] * store_a.shape[2]
    ta = torch.tensor(store_a.reshape(-1)).to(torch.bfloat16).cuda()
    # B(k, n) at n * sbn + k: codes of random finite values
    sbn = K + pad
    codes = FINITE[rng.integers(0, len(FINITE), size=(batch, N, sbn))]
    sbb = N * sbn
    tb = torch.tensor(codes.reshape(-1), dtype=torch.uint8).cuda()
    if mode == 1:
        scale = 2.0 ** rng.integers(-8, 4, size=N)
        bmul = np.broadcast_to(scale[None, :, None], (batch, N, K))
    elif mode == 2:
        scale = np.repeat(2.0 ** rng.integers(-8, 4, size=(K + 7) // 8), 8)[:K]
        bmul = np.broadcast_to(scale[None, None, :], (batch, N, K))
    else:
        scale = np.ones(1)
        bmul = np.ones((batch, N, K))
    tsc = torch.tensor(scale, dtype=torch.float32).cuda()
    b = fp8.e4m3_decode(codes[:, :, :K]) * bmul                 # batch x N x K
    want = np.einsum("bmk,bnk->bmn", a, b)
    out_t = torch.float64 if ctype == 0 else torch.float32
    tc = torch.zeros(batch * M * N, dtype=out_t, device="cuda")
    part = torch.zeros(max(1, splits * batch * M * N), dtype=torch.float64, device="cuda")
    st = L.cpppl_test_gemm_e4m3b(M, N, K, batch, ta.data_ptr(), sam, sak, sab, tb.data_ptr(), sbn,
                                 sbb, tsc.data_ptr(), mode, tc.data_ptr(), N, M * N, ctype, splits,
                                 part.data_ptr(), _stream(torch))
    assert st == 0
    got = tc.cpu().to(torch.float64).numpy().reshape(batch, M, N)
    err = np.abs(got - want).max() / max(1e-300, np.abs(want).max())
    assert err <= 5e-5, err


FP8_SMALL = {
    "C1": synth.CONFIGS["C1"],
    "ragged": synth.custom_config(5, 40, 70, 70, name="o5v40X70R70"),
    "odd": synth.custom_config(7, 24, 61, 131, name="o7v24X61R131"),
}


@pytest.mark.parametrize("name", list(FP8_SMALL))
def test_fp8_mttkrp(lib, name):
    cfg = FP8_SMALL[name]
    _say(f"fp8 mttkrp {name}")
    inp = synth.make_inputs(cfg)
    fs = synth.init_factors(cfg)
    tq, bq = fp8.fp8_inputs(inp.t, inp.b_vv)
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "fp8")
    ctx.load_t2(inp.t)
    ctx.load_df(inp.b_vv)
    ctx.set_factors(*fs)
    for mode in range(4):
        got = ctx.mttkrp(mode)
        want_q = oracle.mttkrp_chain(tq, bq, fs, mode)
        want = oracle.mttkrp_chain(inp.t, inp.b_vv, fs, mode)
        e_x, e_oq = _rel(got, want), _rel(want_q, want)
        # against the oracle's chain on the dequantised inputs: the 5 bfloat16
        # roundings of the factors and intermediates (bounds.py)
        e_q = assert_lowp(got, want_q, abs_chain(tq, bq, fs, mode), N_ROUND_FP8,
                          chain_lengths(cfg.o, cfg.v, cfg.nx, mode), f"{name} mode {mode}")
        _say(f"  mode {mode}: vs quantised inputs {e_q:.2e}, vs exact {e_x:.2e} "
             f"(oracle quantisation error {e_oq:.2e})")
        # against the exact MTTKRP: the quantisation error plus at most that bound
        assert e_x <= e_oq + normwise(N_ROUND_FP8)
        # FP64 MTTKRP of the same context uses the FP64 masters
        assert_fp64(ctx.mttkrp(mode, "fp64"), want)
    with pytest.raises(lib.CppplError):
        ctx.mttkrp(0, "bf16")
    ctx.close()


def test_fp8_needs_v_multiple_of_8(lib):
    with pytest.raises(lib.CppplError):
        lib.Context(3, 10, 7, 5, "fp8")


def test_fp8_refinement_is_fp64(lib):
    cfg = FP8_SMALL["ragged"]
    _say("fp8 refinement = FP64 sweeps")
    inp = synth.make_inputs(cfg)
    c8 = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "fp8")
    c8.load_t2(inp.t)
    c8.load_df(inp.b_vv)
    c8.set_factors(*synth.init_factors(cfg))
    r = c8.als(6)
    assert np.all(np.isfinite(r["fit_hist"]))
    assert r["fit_hist"][-1] > r["fit_hist"][0]
    state = c8.get_factors()
    r8 = c8.als(0, refine=2)
    assert r8["sweeps"] == 2 and r8["refine_sweeps"] == 2
    c64 = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "fp64")
    c64.load_t2(inp.t)
    c64.load_df(inp.b_vv)
    c64.set_factors(*state)
    r64 = c64.als(2)
    np.testing.assert_allclose(r8["fit_hist"], r64["fit_hist"], rtol=0, atol=1e-12)
    c8.close()
    c64.close()


def test_fp8_sampled_columns_full_size(lib):
    """C3 sizes (o 32, v 256, X 768, R 1024): sampled columns r of the FP8
    MTTKRP against the oracle's chain on the dequantised inputs (a column of
    the MTTKRP depends on column r of the factors only)."""
    cfg = synth.CONFIGS["C3"]
    _say("fp8 sampled columns C3")
    inp = synth.make_inputs(cfg)
    fs = synth.init_factors(cfg)
    ctx = lib.Context(cfg.o, cfg.v, cfg.nx, cfg.rank, "fp8")
    ctx.load_t2(inp.t)
    ctx.load_df(inp.b_vv)
    ctx.set_factors(*fs)
    cols = [0, 511, cfg.rank - 1]
    tq, bq = fp8.fp8_inputs(inp.t, inp.b_vv)
    sub = [f[:, cols] for f in fs]
    for mode in (0, 2):
        got = ctx.mttkrp(mode)[:, cols]
        want = oracle.mttkrp_chain(tq, bq, sub, mode)
        err = assert_lowp(got, want, abs_chain(tq, bq, sub, mode), N_ROUND_FP8,
                          chain_lengths(cfg.o, cfg.v, cfg.nx, mode), f"C3 mode {mode}")
        _say(f"  mode {mode}: rel err {err:.2e}")
    ctx.close()


RESIDENT_E4M3 = [
    # (M, N, K, pad): shapes of Y = F^T B with an e4m3 B (batch 1, BF16 result),
    # which go to the B-resident kernel
    (300, 4096, 256, 8),     # ragged last row block
    (256, 2304, 384, 0),     # K = 384: four-wave work-groups of 128 columns
    (200, 4096, 128, 8),     # K = 128
]


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("case", RESIDENT_E4M3)
def test_gemm_e4m3_b_resident(env, mode, case):
    """e4m3 B in the B-resident kernel (fragments decoded once per work-group):
    against the decoded product in numpy, and bit for bit against the tiled
    kernel (the same product written with a C row stride that is not a multiple
    of 8 goes there)."""
    L, torch = env
    M, N, K, pad = case
    _say(f"gemm e4m3 B resident mode={mode} case={case}")
    rng = np.random.default_rng(zlib.crc32(repr(("resident-e4m3", M, N, K, mode)).encode()))
    a = rng.standard_normal((M, K))
    a = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    sam = K + pad
    store_a = np.zeros((M, sam))
    store_a[:, :K] = a
    ta = torch.tensor(store_a.reshape(-1)).to(torch.bfloat16).cuda()
    sbn = K + pad
    codes = FINITE[rng.integers(0, len(FINITE), size=(N, sbn))]
    tb = torch.tensor(codes.reshape(-1), dtype=torch.uint8).cuda()
    if mode == 1:
        scale = 2.0 ** rng.integers(-8, 4, size=N)
        bmul = np.broadcast_to(scale[:, None], (N, K))
    elif mode == 2:
        scale = np.repeat(2.0 ** rng.integers(-8, 4, size=K // 8), 8)
        bmul = np.broadcast_to(scale[None, :], (N, K))
    else:
        scale = np.ones(1)
        bmul = np.ones((N, K))
    tsc = torch.tensor(scale, dtype=torch.float32).cuda()
    want = a @ (fp8.e4m3_decode(codes[:, :K]) * bmul).T
    out = {}
    for scm in (N, N + 4):
        tc = torch.full((M * scm,), 7.0, dtype=torch.bfloat16, device="cuda")
        st = L.cpppl_test_gemm_e4m3b(M, N, K, 1, ta.data_ptr(), sam, 1, 0, tb.data_ptr(), sbn, 0,
                                     tsc.data_ptr(), mode, tc.data_ptr(), scm, 0, 2, 1, None,
                                     _stream(torch))
        assert st == 0
        full = tc.view(M, scm)
        if scm > N:
            assert torch.all(full[:, N:].float() == 7.0)
        out[scm] = full[:, :N].contiguous()
    torch.cuda.synchronize()
    assert torch.equal(out[N].view(torch.int16), out[N + 4].view(torch.int16))
    got = out[N].to(torch.float64).cpu().numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err <= 8e-3, err
