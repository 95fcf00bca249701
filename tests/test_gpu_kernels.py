"""GPU checks of the kernel layer through the test hooks: the matrix-core GEMM
in both precisions and every operand layout (ragged tiles, batches, split-K),
and the blocked Cholesky solve, against numpy in FP64."""
import ctypes as C
import sys
import zlib

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env(lib):
    import torch
    L = lib.load_library()
    L.cpppl_test_gemm.restype = C.c_int
    L.cpppl_test_gemm.argtypes = [C.c_int] + [C.c_int64] * 4 + [C.c_void_p] + [C.c_int64] * 3 + \
        [C.c_void_p] + [C.c_int64] * 3 + [C.c_void_p] + [C.c_int64] * 2 + \
        [C.c_int, C.c_double, C.c_double, C.c_int, C.c_void_p, C.c_void_p]
    L.cpppl_test_spd_solve.restype = C.c_int
    L.cpppl_test_spd_solve.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                                       C.c_void_p, C.c_void_p, C.c_void_p]
    return L, torch


def _operand(torch, rng, batch, rows, cols, unit_dim, dtype, pad=3):
    """Logical X[b][rows][cols] stored with unit stride along `unit_dim`."""
    x = rng.standard_normal((batch, rows, cols))
    if dtype == "bf16":
        x = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    if unit_dim == 1:
        ld = cols + pad
        store = np.zeros((batch, rows, ld))
        store[:, :, :cols] = x
        s_row, s_col = ld, 1
    else:
        ld = rows + pad
        store = np.zeros((batch, cols, ld))
        store[:, :, :rows] = x.transpose(0, 2, 1)
        s_row, s_col = 1, ld
    sb = store.shape[1] * store.shape[2]
    t = torch.tensor(store.reshape(-1))
    if dtype == "bf16":
        t = t.to(torch.bfloat16)
    return x, t.cuda(), s_row, s_col, sb


CASES = [
    # (M, N, K, batch, splits)
    (70, 45, 37, 1, 1),
    (129, 131, 200, 2, 1),
    (64, 64, 16, 1, 1),
    (33, 257, 300, 1, 4),
    (5, 3, 1, 3, 1),
    (130, 200, 4104, 1, 1),     # BF16: K slices of 64, odd slice count
    (257, 129, 9000, 2, 2),     # BF16: K slices of 64 per split, ragged tail
    (512, 130, 1100, 1, 1),     # BF16 k-contiguous: 256-row tiles, ragged K tail
    (2100, 70, 1040, 2, 1),     # BF16 k-contiguous: 256-row tiles, ragged last tile row
    (200, 136, 256, 2, 1),      # BF16 unchecked loads: whole K slices, ragged rows (multiples of 8)
    (200, 136, 4096, 1, 1),     # the same with K slices of 64
    (264, 72, 8192, 1, 2),      # the same, split-K
    (136, 200, 2112, 1, 1),     # unchecked loads, two-stage prefetch over an odd number of 64-deep slices
    (200, 136, 96, 1, 1),       # unchecked loads, three 32-deep slices (two-stage where the layout runs at three waves)
    (200, 136, 32, 2, 1),       # unchecked loads, a single slice
]


@pytest.mark.parametrize("dtype", ["f64", "bf16"])
@pytest.mark.parametrize("ak", [True, False])
@pytest.mark.parametrize("bk", [True, False])
@pytest.mark.parametrize("case", CASES)
def test_gemm_layouts(env, dtype, ak, bk, case):
    L, torch = env
    M, N, K, batch, splits = case
    _say(f"gemm {dtype} ak={ak} bk={bk} case={case}")
    rng = np.random.default_rng(zlib.crc32(repr((M, N, K, batch, ak, bk)).encode()))
    a, ta, sam, sak, sab = _operand(torch, rng, batch, M, K, 1 if ak else 0, dtype)
    b, tb, sbk, sbn, sbb = _operand(torch, rng, batch, K, N, 0 if bk else 1, dtype)
    c0 = rng.standard_normal((batch, M, N))
    beta = 0.5 if dtype == "f64" else 0.0
    alpha = -1.25 if dtype == "f64" else 1.0
    tc = torch.tensor(c0.reshape(-1)).cuda()
    part = torch.zeros(max(1, splits * batch * M * N), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    st = L.cpppl_test_gemm(0 if dtype == "f64" else 1, M, N, K, batch,
                           ta.data_ptr(), sam, sak, sab, tb.data_ptr(), sbk, sbn, sbb,
                           tc.data_ptr(), N, M * N, 0, alpha, beta, splits, part.data_ptr(), stream)
    assert st == 0
    want = alpha * np.einsum("bmk,bkn->bmn", a, b) + beta * c0
    got = tc.cpu().numpy().reshape(batch, M, N)
    err = np.abs(got - want).max() / max(1e-300, np.abs(want).max())
    tol = 1e-13 if dtype == "f64" else 5e-5
    assert err <= tol, err


STAGED = [
    # (M, N, K, batch, splits), both operands k-contiguous
    (512, 200, 1024, 2, 1),     # 256-row tiles
    (768, 256, 1100, 1, 1),     # 256-row tiles, ragged K tail
    (2100, 130, 1030, 1, 1),    # 256-row tiles, ragged last tile row
    (512, 200, 96, 2, 1),       # 128-row tiles, short K
    (512, 136, 1056, 1, 1),     # 256-row tiles, two-stage prefetch over an odd number of slices
    (1024, 64, 3000, 1, 4),     # 128-row tiles, split-K
]


@pytest.mark.parametrize("out", ["f32", "bf16"])
@pytest.mark.parametrize("case", STAGED)
def test_gemm_bf16_outputs(env, out, case):
    """FP32 and BF16 results (the LDS-staged epilogue), split-K included."""
    L, torch = env
    M, N, K, batch, splits = case
    _say(f"gemm bf16 -> {out} case={case}")
    rng = np.random.default_rng(zlib.crc32(repr((M, N, K, batch, out)).encode()))
    a, ta, sam, sak, sab = _operand(torch, rng, batch, M, K, 1, "bf16")
    b, tb, sbk, sbn, sbb = _operand(torch, rng, batch, K, N, 0, "bf16")
    tdt = torch.float32 if out == "f32" else torch.bfloat16
    tc = torch.full((batch * M * N,), 7.0, dtype=tdt, device="cuda")
    part = torch.zeros(max(1, splits * batch * M * N), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    st = L.cpppl_test_gemm(1, M, N, K, batch, ta.data_ptr(), sam, sak, sab, tb.data_ptr(), sbk,
                           sbn, sbb, tc.data_ptr(), N, M * N, 1 if out == "f32" else 2, 0.75, 0.0,
                           splits, part.data_ptr(), stream)
    assert st == 0
    want = 0.75 * np.einsum("bmk,bkn->bmn", a, b)
    got = tc.to(torch.float64).cpu().numpy().reshape(batch, M, N)
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err <= (5e-5 if out == "f32" else 8e-3), err


CHAINED = [
    # (M, N, K, batch, splits): 2048 to 4096 tiles of 128 x 128 with K per
    # split at most 512, so work-groups run two tiles in turn
    (136, 264, 64, 400, 1),      # ragged last tile row and column (multiples of 8)
    (200, 136, 32, 900, 1),      # a single K slice per tile
    (128, 128, 64, 2101, 1),     # an odd tile count: the last work-group has one tile
    (1024, 2048, 1248, 1, 20),   # split-K, the last split one slice shorter than the rest
]


@pytest.mark.parametrize("layout", ["kk", "rr"])
@pytest.mark.parametrize("out", ["f32", "bf16"])
@pytest.mark.parametrize("case", CHAINED)
def test_gemm_bf16_chained(env, layout, out, case):
    """Unchecked short-K products of 2048 to 4096 tiles at four waves per SIMD (two
    k-contiguous or two row-contiguous operands) run two tiles per work-group,
    the second tile's first slice loading before the first tile's results are
    stored.  Every tile is checked against numpy."""
    L, torch = env
    M, N, K, batch, splits = case
    ak = bk = layout == "kk"
    _say(f"gemm bf16 chained {layout} -> {out} case={case}")
    rng = np.random.default_rng(zlib.crc32(repr((M, N, K, batch, layout, out)).encode()))
    a, ta, sam, sak, sab = _operand(torch, rng, batch, M, K, 1 if ak else 0, "bf16", pad=8)
    b, tb, sbk, sbn, sbb = _operand(torch, rng, batch, K, N, 0 if bk else 1, "bf16", pad=8)
    tdt = torch.float32 if out == "f32" else torch.bfloat16
    tc = torch.full((batch * M * N,), 7.0, dtype=tdt, device="cuda")
    part = torch.zeros(max(1, splits * batch * M * N), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    st = L.cpppl_test_gemm(1, M, N, K, batch, ta.data_ptr(), sam, sak, sab, tb.data_ptr(), sbk,
                           sbn, sbb, tc.data_ptr(), N, M * N, 1 if out == "f32" else 2, 1.0, 0.0,
                           splits, part.data_ptr(), stream)
    assert st == 0
    want = np.matmul(a, b)
    got = tc.to(torch.float64).cpu().numpy().reshape(batch, M, N)
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err <= (5e-5 if out == "f32" else 8e-3), err


RESIDENT = [
    # (M, N, K, batch, pad): K of 128, 256 or 384, N a multiple of the
    # work-group's columns (256, or 128 at K = 384), at least 16 column blocks
    # over the batches, at least 128 rows, a BF16 result
    (1024, 4096, 256, 1, 0),   # row blocks and row ranges divide evenly
    (1000, 8192, 256, 1, 8),   # ragged last row block, padded operand rows
    (300, 4608, 128, 1, 0),    # K = 128: half the lanes load each row block
    (128, 4096, 256, 1, 0),    # eight row blocks, one row range
    (200, 256, 256, 20, 8),    # batched (the shape of Z = Y tau per r), ragged rows
    (768, 512, 128, 9, 0),     # batched, two column blocks per batch, K = 128
    (300, 2304, 384, 1, 8),    # K = 384: four-wave work-groups of 128 columns
    (200, 384, 384, 8, 0),     # K = 384, batched (the shape of Z at v = 384)
]


@pytest.mark.parametrize("bk", [True, False])
@pytest.mark.parametrize("case", RESIDENT)
def test_gemm_bf16_b_resident(env, case, bk):
    """Short-K products of a k-contiguous A over many columns with a BF16
    result (the shapes of Y = F^T B and of Z = Y tau per r, B k- or
    n-contiguous) keep B in registers and stream A.  Checked against numpy, and
    bit for bit against the tiled kernel: the same product written with a C row
    stride that is not a multiple of 8 goes there (the padding columns must
    stay untouched)."""
    L, torch = env
    M, N, K, batch, pad = case
    _say(f"gemm bf16 B resident bk={bk} case={case}")
    rng = np.random.default_rng(zlib.crc32(repr(("resident", M, N, K, batch, pad, bk)).encode()))
    a, ta, sam, sak, sab = _operand(torch, rng, batch, M, K, 1, "bf16", pad=pad)
    b, tb, sbk, sbn, sbb = _operand(torch, rng, batch, K, N, 0 if bk else 1, "bf16", pad=pad)
    stream = torch.cuda.current_stream().cuda_stream
    out = {}
    for scm in (N, N + 4):
        tc = torch.full((batch * M * scm,), 7.0, dtype=torch.bfloat16, device="cuda")
        st = L.cpppl_test_gemm(1, M, N, K, batch, ta.data_ptr(), sam, sak, sab, tb.data_ptr(), sbk,
                               sbn, sbb, tc.data_ptr(), scm, M * scm, 2, 0.5, 0.0, 1, None, stream)
        assert st == 0
        full = tc.view(batch, M, scm)
        if scm > N:
            assert torch.all(full[:, :, N:].float() == 7.0)
        out[scm] = full[:, :, :N].contiguous()
    torch.cuda.synchronize()
    assert torch.equal(out[N].view(torch.int16), out[N + 4].view(torch.int16))
    want = 0.5 * np.matmul(a, b)
    got = out[N].to(torch.float64).cpu().numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err <= 8e-3, err


@pytest.mark.parametrize("which", ["Y", "Z"])
def test_gemm_bf16_chained_bitwise(env, which):
    """At o = 32, v = 256, X = 768, R = 1024 the ALS sweep may cut Y = F^T B and
    Z = Y tau (per r) into launches along N or the batch, which changes each
    launch's grid (tiles per work-group, row ranges per column block) but not
    the arithmetic of an element, so a whole product and one cut into four must
    agree bit for bit."""
    L, torch = env
    v, X, R = 256, 768, 1024
    _say(f"gemm bf16 chained vs whole, {which} at v={v} X={X} R={R}")
    g = torch.Generator(device="cuda").manual_seed(7)
    stream = torch.cuda.current_stream().cuda_stream

    def call(M, N, K, batch, A, sam, sak, sab, B, sbk, sbn, sbb, C, scm, scb):
        st = L.cpppl_test_gemm(1, M, N, K, batch, A, sam, sak, sab, B, sbk, sbn, sbb, C, scm, scb,
                               2, 1.0, 0.0, 1, 0, stream)
        assert st == 0

    if which == "Y":
        M, N, K = R, X * v, v
        a = torch.randn(M * K, device="cuda", generator=g).to(torch.bfloat16)   # [r][p]
        b = torch.randn(N * K, device="cuda", generator=g).to(torch.bfloat16)   # [(X, q)][p]
        whole = torch.empty(M * N, dtype=torch.bfloat16, device="cuda")
        cut = torch.full((M * N,), 3.0, dtype=torch.bfloat16, device="cuda")
        call(M, N, K, 1, a.data_ptr(), K, 1, 0, b.data_ptr(), 1, K, 0, whole.data_ptr(), N, 0)
        n4 = N // 4
        for c in range(4):
            call(M, n4, K, 1, a.data_ptr(), K, 1, 0, b[c * n4 * K:].data_ptr(), 1, K, 0,
                 cut[c * n4:].data_ptr(), N, 0)
    else:
        M, N, K, batch = X, v, v, R
        a = torch.randn(batch * M * K, device="cuda", generator=g).to(torch.bfloat16)  # [r][X][c]
        b = torch.randn(batch * N * K, device="cuda", generator=g).to(torch.bfloat16)  # [r][d][c]
        whole = torch.empty(batch * M * N, dtype=torch.bfloat16, device="cuda")
        cut = torch.full((batch * M * N,), 3.0, dtype=torch.bfloat16, device="cuda")
        call(M, N, K, batch, a.data_ptr(), K, 1, M * K, b.data_ptr(), 1, K, N * K,
             whole.data_ptr(), N, M * N)
        b4 = batch // 4
        for c in range(4):
            call(M, N, K, b4, a[c * b4 * M * K:].data_ptr(), K, 1, M * K, b[c * b4 * N * K:].data_ptr(),
                 1, K, N * K, cut[c * b4 * M * N:].data_ptr(), N, M * N)
    torch.cuda.synchronize()
    assert torch.isfinite(whole.float()).all()
    assert torch.equal(whole.view(torch.int16), cut.view(torch.int16))


@pytest.mark.parametrize("which", ["Y", "Z"])
def test_gemm_bf16_b_resident_full_size(env, which):
    """The C3 shapes of Y = F^T B (1024 x 196608, K = 256) and Z = Y tau per r
    (1024 batches of 768 x 256, K = 256) on the B-resident kernel, with its
    register ring and padded trips exactly as the sweep launches them: bit for
    bit against the tiled kernel (reached through a C row stride that is not a
    multiple of 8), and sampled columns against float64 products."""
    L, torch = env
    v, X, R = 256, 768, 1024
    _say(f"gemm bf16 B resident full size {which}")
    g = torch.Generator(device="cuda").manual_seed(11)
    stream = torch.cuda.current_stream().cuda_stream
    if which == "Y":
        M, N, K, batch = R, X * v, v, 1
    else:
        M, N, K, batch = X, v, v, R
    a = torch.randn(batch * M * K, device="cuda", generator=g).to(torch.bfloat16)
    b = torch.randn(batch * N * K, device="cuda", generator=g).to(torch.bfloat16)
    out = {}
    for scm in (N, N + 4):
        c = torch.full((batch * M * scm,), 7.0, dtype=torch.bfloat16, device="cuda")
        st = L.cpppl_test_gemm(1, M, N, K, batch, a.data_ptr(), K, 1, M * K, b.data_ptr(), 1, K,
                               N * K, c.data_ptr(), scm, M * scm, 2, 1.0, 0.0, 1, 0, stream)
        assert st == 0
        full = c.view(batch, M, scm)
        if scm > N:
            assert torch.all(full[:, :, N:].float() == 7.0)
        out[scm] = full[:, :, :N].contiguous()
        del c, full
    torch.cuda.synchronize()
    assert torch.equal(out[N].view(torch.int16), out[N + 4].view(torch.int16))
    a3 = a.view(batch, M, K).double()
    b3 = b.view(batch, N, K).double()
    for bi in sorted({0, batch // 2, batch - 1}):
        for col in sorted({0, N // 3, N - 1}):
            want = (a3[bi] @ b3[bi, col]).cpu().numpy()
            got = out[N][bi, :, col].double().cpu().numpy()
            err = np.abs(got - want).max() / np.abs(want).max()
            assert err <= 8e-3, (which, bi, col, err)


@pytest.mark.parametrize("R,n", [(1, 3), (17, 5), (64, 64), (65, 7), (300, 130), (1024, 256),
                                 (2048, 32)])
def test_spd_inverse_solve(env, R, n):
    L, torch = env
    _say(f"spd_solve R={R} n={n}")
    rng = np.random.default_rng(R)
    f = rng.standard_normal((R + 5, R))
    w = f.T @ f + 0.1 * np.eye(R)
    x = rng.standard_normal((R, n))
    tw = torch.tensor(w).cuda()
    tx = torch.tensor(x).cuda()
    ty = torch.zeros((R, n), dtype=torch.float64, device="cuda")
    work = torch.zeros(R * R + 8192, dtype=torch.float64, device="cuda")
    status = torch.zeros(4, dtype=torch.int32, device="cuda")
    st = L.cpppl_test_spd_solve(tw.data_ptr(), R, tx.data_ptr(), ty.data_ptr(), n, work.data_ptr(),
                                status.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert st == 0 and int(status[0]) == 0
    want = np.linalg.solve(w, x)
    got = ty.cpu().numpy()
    cond = np.linalg.cond(w)
    assert np.abs(got - want).max() <= 1e-14 * cond * np.abs(want).max() * 10


def test_spd_inverse_flags_indefinite(env):
    L, torch = env
    R = 70
    w = np.eye(R)
    w[40, 40] = -1.0
    tw = torch.tensor(w).cuda()
    tx = torch.ones((R, 2), dtype=torch.float64, device="cuda")
    ty = torch.zeros((R, 2), dtype=torch.float64, device="cuda")
    work = torch.zeros(R * R + 8192, dtype=torch.float64, device="cuda")
    status = torch.zeros(4, dtype=torch.int32, device="cuda")
    st = L.cpppl_test_spd_solve(tw.data_ptr(), R, tx.data_ptr(), ty.data_ptr(), 2, work.data_ptr(),
                                status.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert st == 0 and int(status[0]) == 1
    assert torch.isfinite(ty).all()

