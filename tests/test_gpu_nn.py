"""GPU tests of the surrogate building blocks (include/sbr_nn.h) against plain
FP64 numpy and the CPU surrogate reference.

GEMM cases use small integers (exact in bfloat16, every partial sum exact in
FP32) so the matrix-core result must equal the FP64 product bit for bit in
every operand layout; random-valued cases then check rounding behaviour.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import surrogate_ref as R


@pytest.fixture(scope="module")
def env():
    """Tensors and kernels share one stream (temporaries passed to the
    asynchronous calls are recycled by torch only in that stream's order)."""
    import torch
    from paper_2208_10006_amd import sbr, nn
    from paper_2208_10006_amd.surrogate import Runtime
    rt = Runtime(0)
    with rt:
        yield torch, sbr, nn, rt.ctx
    rt.synchronize()


def banner(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(torch, a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    if str(t.dtype) == "torch.bfloat16":
        return t.float().cpu().numpy().astype(np.float64)
    return t.cpu().numpy()


def sync(torch):
    torch.cuda.synchronize()


def run_gemm(env, A, B, layout, bias=None, flags=0, C0=None, out_bf16=False):
    """A [M][K], B [K][N] (numpy); `layout` chooses the strides the kernel sees."""
    torch, S, nn, ctx = env
    M, K = A.shape
    N = B.shape[1]
    if layout in ("fwd", "bwd_data"):
        Ad = dev(torch, A, torch.bfloat16)
        a_si, a_sk = K, 1
    else:  # A stored transposed ([K][M], "bwd_weight")
        Ad = dev(torch, A.T, torch.bfloat16)
        a_si, a_sk = 1, M
    if layout in ("fwd", "bwd_weight"):
        Bd = dev(torch, B, torch.bfloat16)
        b_sk, b_sj = N, 1
    else:  # B stored transposed ([N][K], "bwd_data")
        Bd = dev(torch, B.T, torch.bfloat16)
        b_sk, b_sj = 1, K
    dt = torch.bfloat16 if out_bf16 else torch.float32
    Cd = dev(torch, C0, dt) if C0 is not None else torch.full((M, N), 7.0, dtype=dt, device="cuda")
    bd = dev(torch, bias, torch.float32) if bias is not None else None
    f = flags | (nn.OUT_BF16 if out_bf16 else 0)
    nn.sbr_nn_gemm_bf16(ctx, M, N, K, Ad, a_si, a_sk, Bd, b_sk, b_sj, bd, Cd, N, f)
    sync(torch)
    return host(Cd)


# covers 64- and 128-wide tiles, split-K (long K, few tiles), ragged edges and
# every operand load mode (k-contiguous, row-contiguous, general strides)
SHAPES = [(1, 1, 1), (16, 16, 32), (64, 64, 32), (64, 64, 64), (100, 70, 45), (130, 257, 300), (5, 3, 1000),
          (300, 2, 17), (65536, 128, 64), (65600, 136, 72), (9, 16, 409600), (256, 256, 4096)]


@pytest.mark.parametrize("layout", ["fwd", "bwd_data", "bwd_weight"])
@pytest.mark.parametrize("shape", SHAPES)
def test_gemm_exact_integers(env, layout, shape):
    M, N, K = shape
    banner("gemm exact", layout, M, N, K)
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    A = rng.integers(-4, 5, (M, K)).astype(np.float64)
    B = rng.integers(-4, 5, (K, N)).astype(np.float64)
    C = run_gemm(env, A, B, layout)
    assert np.array_equal(C, A @ B)


def test_gemm_operand_positions(env):
    """One-hot operands: C[i][j] = A[i][k] B[k][j] for a single k isolates the
    lane layout of each operand (a wrong row/column/k mapping moves the 1)."""
    M, N, K = 48, 40, 96
    banner("gemm positions", M, N, K)
    rng = np.random.default_rng(5)
    for layout in ["fwd", "bwd_data", "bwd_weight"]:
        for _ in range(3):
            k = int(rng.integers(0, K))
            A = np.zeros((M, K))
            B = np.zeros((K, N))
            A[:, k] = np.arange(M) + 1
            B[k, :] = (np.arange(N) + 1) * 64
            C = run_gemm(env, A, B, layout)
            assert np.array_equal(C, A @ B), (layout, k)


def test_gemm_k_zero_gives_bias(env):
    torch, S, nn, ctx = env
    banner("gemm K=0")
    bias = np.arange(9, dtype=np.float32)
    A = np.zeros((5, 0))
    B = np.zeros((0, 9))
    C = run_gemm(env, A, B, "fwd", bias=bias)
    assert np.array_equal(C, np.tile(bias, (5, 1)))


@pytest.mark.parametrize("layout", ["fwd", "bwd_data", "bwd_weight"])
def test_gemm_random_values_and_flags(env, layout):
    M, N, K = 197, 131, 259
    banner("gemm flags", layout, M, N, K)
    rng = np.random.default_rng(11)
    A = R.bf16(rng.standard_normal((M, K)))
    B = R.bf16(rng.standard_normal((K, N)))
    bias = rng.standard_normal(N).astype(np.float32)
    ref = A @ B + bias.astype(np.float64)
    tol = 2e-6 * (np.abs(A) @ np.abs(B) + np.abs(bias)) + 1e-30
    C = run_gemm(env, A, B, layout, bias=bias)
    assert np.all(np.abs(C - ref) <= tol)
    Cr = run_gemm(env, A, B, layout, bias=bias, flags=1)
    assert np.all(np.abs(Cr - np.maximum(ref, 0)) <= tol)
    assert np.all(Cr >= 0)
    # bf16 output: the FP32 result rounded once
    Cb = run_gemm(env, A, B, layout, bias=bias, flags=1, out_bf16=True)
    assert np.array_equal(Cb, R.bf16(np.maximum(C, 0).astype(np.float32)))
    # accumulate into an existing FP32 C
    C0 = rng.standard_normal((M, N)).astype(np.float32)
    Ca = run_gemm(env, A, B, layout, bias=bias, flags=4, C0=C0)
    assert np.all(np.abs(Ca - (ref + C0)) <= tol + 1e-6 * np.abs(C0))


def run_gemm_ex(env, A, B, layout, mask=None, with_bsum=False, bsum0=None, flags=0, out_bf16=False):
    """sbr_nn_gemm_bf16_ex; returns (C, bsum) on the host (bsum None unless asked)."""
    torch, S, nn, ctx = env
    M, K = A.shape
    N = B.shape[1]
    if layout == "bwd_weight":  # A stored transposed ([K][M])
        Ad = dev(torch, A.T, torch.bfloat16) if M else None
        a_si, a_sk = 1, M
    else:
        Ad = dev(torch, A, torch.bfloat16) if M else None
        a_si, a_sk = K, 1
    if layout == "bwd_data":  # B stored transposed ([N][K])
        Bd = dev(torch, B.T, torch.bfloat16)
        b_sk, b_sj = 1, K
    else:
        Bd = dev(torch, B, torch.bfloat16)
        b_sk, b_sj = N, 1
    dt = torch.bfloat16 if out_bf16 else torch.float32
    Cd = torch.full((max(M, 1), N), 7.0, dtype=dt, device="cuda")
    md = dev(torch, mask, torch.bfloat16) if mask is not None else None
    bs = None
    if with_bsum:
        bs = dev(torch, bsum0, torch.float32) if bsum0 is not None else torch.full((N,), 7.0, device="cuda")
    f = flags | (nn.OUT_BF16 if out_bf16 else 0)
    nn.sbr_nn_gemm_bf16_ex(ctx, M, N, K, Ad, a_si, a_sk, Bd, b_sk, b_sj, None, Cd if M else None, N, f, md, N, bs)
    sync(torch)
    return host(Cd)[:M], (host(bs) if bs is not None else None)


# the column-sum row lands in its own tile row (M = 64, 256), in the last
# partial tile (M = 9, 100) or alone (M = 0); long K with few tiles splits K
EX_SHAPES = [(1, 1, 1), (0, 16, 5000), (9, 16, 409600), (64, 64, 64), (100, 70, 45), (256, 256, 4096),
             (257, 130, 3000), (3, 257, 70000)]


@pytest.mark.parametrize("shape", EX_SHAPES)
@pytest.mark.parametrize("layout", ["bwd_weight", "fwd"])
def test_gemm_column_sums_exact(env, layout, shape):
    """bsum = column sums of B from the same products: exact on small integers
    (every partial sum is an integer below 2^24), C unchanged by it."""
    M, N, K = shape
    banner("gemm column sums", layout, M, N, K)
    rng = np.random.default_rng(M * 7 + N * 11 + K)
    A = rng.integers(-4, 5, (M, K)).astype(np.float64)
    B = rng.integers(-4, 5, (K, N)).astype(np.float64)
    C, bs = run_gemm_ex(env, A, B, layout, with_bsum=True)
    assert np.array_equal(bs, B.sum(0))
    assert np.array_equal(C, A @ B)
    b0 = rng.integers(-100, 100, N).astype(np.float32)
    _, bs2 = run_gemm_ex(env, A, B, layout, with_bsum=True, bsum0=b0, flags=nn_accumulate(env))
    assert np.array_equal(bs2, B.sum(0) + b0)


def nn_accumulate(env):
    return env[2].ACCUMULATE


@pytest.mark.parametrize("shape", [(1, 1, 1), (197, 131, 259), (4096, 256, 256), (300, 128, 2), (5, 3, 100000)])
@pytest.mark.parametrize("layout", ["bwd_data", "fwd"])
def test_gemm_relu_mask(env, layout, shape):
    """C = (A B) * (mask > 0): exact on integers, FP32 and bf16 outputs; zero,
    negative and positive mask values (and -0) all occur."""
    M, N, K = shape
    banner("gemm relu mask", layout, M, N, K)
    rng = np.random.default_rng(M + 3 * N + 5 * K)
    A = rng.integers(-4, 5, (M, K)).astype(np.float64)
    B = rng.integers(-4, 5, (K, N)).astype(np.float64)
    mask = R.bf16(rng.choice([-1.5, -0.0, 0.0, 1e-30, 0.25, 3.0], (M, N)))
    want = (A @ B) * (mask > 0)
    C, _ = run_gemm_ex(env, A, B, layout, mask=mask)
    assert np.array_equal(C, want)
    Cb, _ = run_gemm_ex(env, A, B, layout, mask=mask, out_bf16=True)
    assert np.array_equal(Cb, R.bf16(want.astype(np.float32)))


def test_gemm_ex_matches_plain_and_deterministic(env):
    """Random bf16 values with a long K (split-K): the extended product equals
    the plain one bit for bit, and repeated calls give identical bits."""
    M, N, K = 144, 32, 200000
    banner("gemm ex determinism", M, N, K)
    rng = np.random.default_rng(21)
    A = R.bf16(rng.standard_normal((M, K)))
    B = R.bf16(rng.standard_normal((K, N)))
    C0 = run_gemm(env, A, B, "bwd_weight")
    C1, b1 = run_gemm_ex(env, A, B, "bwd_weight", with_bsum=True)
    C2, b2 = run_gemm_ex(env, A, B, "bwd_weight", with_bsum=True)
    assert np.array_equal(C0, C1) and np.array_equal(C1, C2) and np.array_equal(b1, b2)
    tol = (K + 2) * 2.0 ** -24 * np.abs(B).sum(0)
    assert np.all(np.abs(b1 - B.sum(0)) <= tol)


def test_gemm_rejects_bad_arguments(env):
    torch, S, nn, ctx = env
    banner("gemm errors")
    x = torch.zeros(16, dtype=torch.bfloat16, device="cuda")
    with pytest.raises(Exception):
        nn.sbr_nn_gemm_bf16(ctx, 4, 4, 4, x, 4, 1, x, 4, 1, None, x, 4, 0x10)
    with pytest.raises(Exception):
        nn.sbr_nn_gemm_bf16(ctx, -1, 4, 4, x, 4, 1, x, 4, 1, None, x, 4, 0)
    with pytest.raises(Exception):
        nn.sbr_nn_im2col(ctx, x, 1, 3, 4, 1, x)
    with pytest.raises(Exception):  # mask leading dimension below N
        nn.sbr_nn_gemm_bf16_ex(ctx, 4, 4, 4, x, 4, 1, x, 4, 1, None, x, 4, 0, x, 3, None)
    with pytest.raises(Exception):  # column sums without B
        nn.sbr_nn_gemm_bf16_ex(ctx, 0, 4, 4, None, 1, 0, None, 4, 1, None, None, 4, 0, None, 0, x.float())
    with pytest.raises(Exception):
        nn.sbr_nn_col2im_relu_backward(ctx, x.float(), 1, 3, 4, 1, x, x)


@pytest.mark.parametrize("shape", [(1, 2, 2, 1), (2, 8, 6, 3), (3, 16, 16, 16), (1, 128, 128, 1)])
def test_im2col_col2im(env, shape):
    torch, S, nn, ctx = env
    n, H, W, C = shape
    banner("im2col/col2im", shape)
    rng = np.random.default_rng(H * W + C)
    x = R.bf16(rng.standard_normal(shape))
    xd = dev(torch, x, torch.bfloat16)
    col = torch.empty((n * (H // 2) * (W // 2), 9 * C), dtype=torch.bfloat16, device="cuda")
    nn.sbr_nn_im2col(ctx, xd, n, H, W, C, col)
    d = rng.standard_normal(col.shape).astype(np.float32)
    dx = torch.empty(shape, dtype=torch.float32, device="cuda")
    nn.sbr_nn_col2im(ctx, dev(torch, d, torch.float32), n, H, W, C, dx)
    sync(torch)
    assert np.array_equal(host(col), R.conv_patches(x))
    ref = R.conv_patches_adjoint(d.astype(np.float64), n, H, W, C)
    assert np.allclose(host(dx), ref, rtol=1e-6, atol=1e-6)
    # fused with the ReLU backward of the layer whose output is y: the same
    # FP32 sums, zeroed where y <= 0, rounded to bf16 once
    y = R.bf16(rng.choice([-1.0, 0.0, 0.5, 2.0], shape))
    dz = torch.empty(shape, dtype=torch.bfloat16, device="cuda")
    nn.sbr_nn_col2im_relu_backward(ctx, dev(torch, d, torch.float32), n, H, W, C, dev(torch, y, torch.bfloat16), dz)
    sync(torch)
    assert np.array_equal(host(dz), R.bf16((host(dx) * (y > 0)).astype(np.float32)))


def test_fourier_features(env):
    torch, S, nn, ctx = env
    n, D, L, E, F, Sn = 777, 7, 8, 16, 144, 3
    banner("fourier", n, D, L, E, F)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (n, D)).astype(np.float32)
    x[0, :] = 0.0
    x[1, :] = 0.5
    emb = R.bf16(rng.standard_normal((Sn, E)))
    scene = rng.integers(0, Sn, n).astype(np.int32)
    X = 2
    extra = rng.normal(size=(n, X)).astype(np.float32)
    out = torch.empty((n, F), dtype=torch.bfloat16, device="cuda")
    nn.sbr_nn_fourier(ctx, dev(torch, x, torch.float32), n, D, L, dev(torch, emb, torch.bfloat16), E,
                      dev(torch, scene, torch.int32), F, out, dev(torch, extra, torch.float32), X)
    sync(torch)
    g = host(out)
    arch = R.Arch(E=E, D=D, L=L, F=F, X=X)
    ref = R.features(arch, emb, x.astype(np.float64), scene, lambda a: a, extra.astype(np.float64))
    fe = E + D + 2 * D * L
    assert np.array_equal(g[:, :E + D], R.bf16(ref[:, :E + D]))
    assert np.array_equal(g[:, fe:fe + X], R.bf16(extra))
    assert np.all(g[:, fe + X:] == 0)
    fr, fg = ref[:, E + D:E + D + 2 * D * L], g[:, E + D:E + D + 2 * D * L]
    assert np.all(np.abs(fg - fr) <= 2.0 ** -8 * np.abs(fr) + 1e-7)


def test_elementwise_kernels(env):
    torch, S, nn, ctx = env
    banner("relu_backward/cast/colsum/gather/onehot")
    rng = np.random.default_rng(4)
    n = 10007
    g = rng.standard_normal(n).astype(np.float32)
    y = R.bf16(rng.standard_normal(n))
    y[::7] = 0.0
    gout = torch.empty(n, dtype=torch.float32, device="cuda")
    gbf = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    nn.sbr_nn_relu_backward(ctx, dev(torch, g, torch.float32), dev(torch, y, torch.bfloat16), n, gout, gbf)
    cast = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    nn.sbr_nn_cast_bf16(ctx, dev(torch, g, torch.float32), n, cast)
    M, N, ld = 3001, 37, 40
    m = rng.standard_normal((M, ld)).astype(np.float32)
    cs = torch.full((N,), 1.5, dtype=torch.float32, device="cuda")
    nn.sbr_nn_colsum(ctx, dev(torch, m, torch.float32), M, N, ld, cs, 1)
    src = rng.standard_normal((50, 12)).astype(np.float32)
    idx = rng.integers(0, 50, 333).astype(np.int64)
    dst = torch.empty((333, 12), dtype=torch.float32, device="cuda")
    nn.sbr_nn_gather_rows(ctx, dev(torch, src, torch.float32), 48, dev(torch, idx, torch.int64), 333, dst)
    sc = rng.integers(0, 9, 100).astype(np.int32)
    oh = torch.empty((100, 9), dtype=torch.bfloat16, device="cuda")
    nn.sbr_nn_onehot_bf16(ctx, dev(torch, sc, torch.int32), 100, 9, oh)
    sync(torch)
    want = np.where(y > 0, g, 0.0).astype(np.float32)
    assert np.array_equal(host(gout), want)
    assert np.array_equal(host(gbf), R.bf16(want))
    assert np.array_equal(host(cast), R.bf16(g))
    assert np.allclose(host(cs), 1.5 + m[:, :N].astype(np.float64).sum(0), rtol=1e-6, atol=1e-5)
    assert np.array_equal(host(dst), src[idx])
    assert np.array_equal(host(oh), (sc[:, None] == np.arange(9)[None, :]).astype(np.float64))


@pytest.mark.parametrize("M,N", [(1, 1), (3001, 2), (5000, 16), (777, 37), (20011, 64), (4096, 128), (999, 200),
                                 (3333, 256)])
def test_relu_backward_colsum(env, M, N):
    """The fused ReLU backward returns the masked gradient exactly and its
    column sums within FP32 rounding of the FP64 sums (the sums are FP64 in a
    fixed order); ragged row counts across the 1,024-row blocks."""
    torch, S, nn, ctx = env
    banner("relu_backward_colsum", M, N)
    rng = np.random.default_rng(M + N)
    g = rng.standard_normal((M, N)).astype(np.float32)
    y = R.bf16(rng.standard_normal((M, N)))
    y[::3, ::2] = 0.0
    gout = torch.empty((M, N), dtype=torch.float32, device="cuda")
    gbf = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")
    cs = torch.full((N,), np.nan, dtype=torch.float32, device="cuda")
    nn.sbr_nn_relu_backward_colsum(ctx, dev(torch, g, torch.float32), dev(torch, y, torch.bfloat16), M, N, cs, gout, gbf)
    cs2 = torch.full((N,), np.nan, dtype=torch.float32, device="cuda")
    nn.sbr_nn_relu_backward_colsum(ctx, dev(torch, g, torch.float32), dev(torch, y, torch.bfloat16), M, N, cs2, None, gbf)
    sync(torch)
    want = np.where(y > 0, g, 0.0).astype(np.float32)
    assert np.array_equal(host(gout), want)
    assert np.array_equal(host(gbf), R.bf16(want))
    ref = want.astype(np.float64).sum(0)
    assert np.all(np.abs(host(cs) - ref) <= 2.0 ** -24 * np.abs(ref) + 1e-12 * np.abs(want).sum(0) + 1e-30)
    assert np.array_equal(host(cs), host(cs2))
    with pytest.raises(S.SbrError):
        nn.sbr_nn_relu_backward_colsum(ctx, dev(torch, g, torch.float32), dev(torch, y, torch.bfloat16), M, 257, cs)


def test_mse_adam_ensemble(env):
    torch, S, nn, ctx = env
    banner("mse/adam/ensemble")
    rng = np.random.default_rng(6)
    n, T, ldp = 5003, 2, 3
    pred = rng.standard_normal((n, ldp)).astype(np.float32)
    tgt = rng.standard_normal((n, T)).astype(np.float32)
    w = (rng.random((n, T)) < 0.8).astype(np.float32)
    dpred = torch.zeros((n, T), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    scale = 1.0 / w.sum()
    nn.sbr_nn_mse(ctx, dev(torch, pred, torch.float32), ldp, dev(torch, tgt, torch.float32),
                  dev(torch, w, torch.float32), n, T, scale, dpred, T, loss)
    sync(torch)
    L, dL = R.mse(pred[:, :T].astype(np.float64), tgt.astype(np.float64), w.astype(np.float64))
    assert abs(loss.item() - L) <= 1e-6 * L
    assert np.allclose(host(dpred), dL, rtol=1e-5, atol=1e-9)

    m = 4099
    W0 = rng.standard_normal(m).astype(np.float32)
    wd = dev(torch, W0, torch.float32)
    md = torch.zeros(m, dtype=torch.float32, device="cuda")
    vd = torch.zeros(m, dtype=torch.float32, device="cuda")
    wb = torch.empty(m, dtype=torch.bfloat16, device="cuda")
    Wr, Mr, Vr = W0.astype(np.float64), np.zeros(m), np.zeros(m)
    lr, b1, b2, eps, dec = 1e-3, 0.9, 0.999, 1e-8, 1e-4
    for step in range(1, 4):
        G = rng.standard_normal(m).astype(np.float32)
        nn.sbr_nn_adam(ctx, wd, dev(torch, G, torch.float32), md, vd, m, lr, b1, b2, eps, dec, step, wb)
        gg = G + dec * Wr
        Mr = b1 * Mr + (1 - b1) * gg
        Vr = b2 * Vr + (1 - b2) * gg * gg
        Wr = Wr - lr * (Mr / (1 - b1 ** step)) / (np.sqrt(Vr / (1 - b2 ** step)) + eps)
    sync(torch)
    assert np.allclose(host(wd), Wr, rtol=1e-5, atol=1e-6)
    assert np.array_equal(host(wb), R.bf16(host(wd)))

    E, nn_, ld = 4, 1001, 2
    outs = rng.standard_normal((E, nn_, ld)).astype(np.float32)
    mean = torch.empty(nn_, dtype=torch.float32, device="cuda")
    spread = torch.empty(nn_, dtype=torch.float32, device="cuda")
    mask = torch.empty(nn_, dtype=torch.uint8, device="cuda")
    nn.sbr_nn_ensemble(ctx, dev(torch, outs, torch.float32), E, nn_ * ld, nn_, ld, 0, 1.0, mean, spread, mask)
    sync(torch)
    o = outs[:, :, 0].astype(np.float64)
    assert np.allclose(host(mean), o.mean(0), rtol=1e-6, atol=1e-6)
    sd = o.std(0)
    assert np.allclose(host(spread), sd, rtol=1e-5, atol=1e-6)
    far = np.abs(sd - 1.0) > 1e-5
    assert np.array_equal(host(mask)[far].astype(bool), (sd > 1.0)[far])


def test_transpose_bf16(env):
    torch, S, nn, ctx = env
    banner("transpose")
    rng = np.random.default_rng(8)
    a = R.bf16(rng.standard_normal((37, 300)))
    out = torch.empty((300, 37), dtype=torch.bfloat16, device="cuda")
    nn.sbr_nn_transpose_bf16(ctx, dev(torch, a, torch.bfloat16), 37, 300, out)
    sync(torch)
    assert np.array_equal(host(out), a.T)


@pytest.mark.parametrize("n", [1, 95, 96, 1000, 20011])
def test_mlp_fused_exact(env, n):
    """Fused inference against the plain definition, on values where every
    sum is exact in FP32 and every layer output is a bfloat16 number: inputs
    on a 2^-6 grid in [-2, 2], eight non-zero weights of +-1/8 per output
    column, biases on the 2^-6 grid in [-1/4, 0], output weights on a 2^-3
    grid.  Then GPU and reference must agree bit for bit."""
    torch, S, nn, ctx = env
    banner("mlp fused exact", n)
    rng = np.random.default_rng(n)
    Sn, depth, T = 5, 6, 2
    emb = rng.integers(-127, 128, (Sn, 128)) / 64.0
    shared = rng.integers(-127, 128, (n, 128)) / 64.0
    scene = rng.integers(0, Sn, n).astype(np.int32)
    W = np.zeros((depth, 256, 256))
    for l in range(depth):
        for j in range(256):
            rows = rng.choice(256, 8, replace=False)
            W[l, rows, j] = rng.choice([-0.125, 0.125], 8)
    b = -rng.integers(0, 17, (depth, 256)) / 64.0
    ow = rng.integers(-8, 9, (256, T)) / 8.0
    ob = rng.standard_normal(T).astype(np.float32)
    # reference: the definition, in FP64 (exact here), bf16 rounding between layers
    h = np.concatenate([emb[scene], shared], axis=1)
    for l in range(depth):
        h = R.bf16(np.maximum(h @ W[l] + b[l], 0.0))
    ref = h @ ow + ob.astype(np.float64)
    wt = np.ascontiguousarray(np.transpose(W, (0, 2, 1)))
    out = torch.empty((n, T), dtype=torch.float32, device="cuda")
    nn.sbr_nn_mlp_infer(ctx, n, dev(torch, shared, torch.bfloat16), dev(torch, emb, torch.bfloat16),
                        dev(torch, scene, torch.int32), dev(torch, wt, torch.bfloat16),
                        dev(torch, b, torch.float32), depth, dev(torch, ow, torch.bfloat16),
                        dev(torch, ob, torch.float32), T, out)
    sync(torch)
    assert np.array_equal(host(out), ref.astype(np.float32))
