"""Pins of the surrogate's CPU FP64 reference (test infrastructure): finite
differences for every parameter gradient, the convolution patches against
the direct definition, their adjoint identity, Fourier features at closed-form
points, and bfloat16 rounding."""
import numpy as np
import pytest

from oracle import surrogate_ref as R

SMALL = R.Arch(H=16, chans=(1, 2, 3, 4, 5), E=4, D=3, L=2, F=24, width=6, depth=2, T=2, X=2)


def small_problem(seed=0):
    rng = np.random.default_rng(seed)
    P = R.init_params(SMALL, seed)
    for k in P:  # non-zero biases so that their gradients are exercised
        if k.endswith("_b"):
            P[k] = rng.normal(0, 0.1, P[k].shape)
    hm = rng.uniform(0, 1, (3, 16, 16))
    x = rng.uniform(-1, 1, (11, 3))
    scene = rng.integers(0, 3, 11)
    t = rng.normal(size=(11, 2))
    w = (rng.uniform(size=(11, 2)) > 0.2).astype(float)
    extra = rng.normal(size=(11, 2))
    return P, hm, x, scene, t, w, extra


def test_gradients_match_finite_differences():
    P, hm, x, scene, t, w, ex = small_problem()
    out, cache = R.forward(SMALL, P, hm, x, scene, extra=ex)
    _, dout = R.mse(out, t, w)
    G = R.backward(SMALL, P, cache, dout)
    eps = 1e-6
    for k, v in P.items():
        flat = v.reshape(-1)
        for i in range(flat.size):
            old = flat[i]
            flat[i] = old + eps
            lp = R.loss_of(SMALL, P, hm, x, scene, t, w, ex)
            flat[i] = old - eps
            lm = R.loss_of(SMALL, P, hm, x, scene, t, w, ex)
            flat[i] = old
            fd = (lp - lm) / (2 * eps)
            an = G[k].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, i, fd, an)


def test_conv_patches_match_direct_convolution():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 10, 12, 3))
    Wc = rng.normal(size=(3, 3, 3, 4))  # ky, kx, ci, co
    col = R.conv_patches(x)
    got = (col @ Wc.reshape(27, 4)).reshape(2, 5, 6, 4)
    ref = np.zeros((2, 5, 6, 4))
    for b in range(2):
        for oy in range(5):
            for ox in range(6):
                for ky in range(3):
                    for kx in range(3):
                        iy, ix = 2 * oy - 1 + ky, 2 * ox - 1 + kx
                        if 0 <= iy < 10 and 0 <= ix < 12:
                            ref[b, oy, ox] += x[b, iy, ix] @ Wc[ky, kx]
    assert np.allclose(got, ref, atol=1e-12)


def test_conv_adjoint_identity():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 8, 6, 3))
    y = rng.normal(size=(2 * 4 * 3, 27))
    lhs = np.sum(R.conv_patches(x) * y)
    rhs = np.sum(x * R.conv_patches_adjoint(y, 2, 8, 6, 3))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_fourier_closed_form():
    f = R.fourier(np.array([[0.5, 0.25]]), 2)
    # d = 0: sin(pi/2)=1, cos(pi/2)=0, sin(pi)=0, cos(pi)=-1
    assert np.allclose(f[0, :4], [1, 0, 0, -1], atol=1e-15)
    s2 = np.sqrt(0.5)
    assert np.allclose(f[0, 4:], [s2, s2, 1, 0], atol=1e-15)


def test_bf16_rounding():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -3.0, 2 ** -130, 65504.0])
    exp = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -3.0, 2 ** -130, 65536.0])
    assert np.array_equal(R.bf16(vals), exp)


def test_bf16_emulation_is_close_to_fp64():
    P, hm, x, scene, t, w, ex = small_problem(3)
    a, _ = R.forward(SMALL, P, hm, x, scene, extra=ex)
    b, _ = R.forward(SMALL, P, hm, x, scene, use_bf16=True, extra=ex)
    assert np.max(np.abs(a - b)) < 0.05 * max(1.0, np.max(np.abs(a)))


# ---------------------------------------------------------------- link features
def test_link_features_closed_forms():
    """Flat ground: clearance is the lowest sample height and nothing obstructs;
    a uniform plateau of height c lowers the clearance by c and obstructs by the
    mean depth below c; the free-space term is Friis' loss; log f maps the
    frequency range onto [-1, 1]."""
    S = 128
    half = 250.0
    t = (np.arange(S) + 0.5) / S
    raw = np.array([[-100.0, 20.0, 25.0, 150.0, -60.0, 1.5, 28e9],
                    [10.0, 10.0, 5.0, 10.0, 60.0, 30.0, 300e9]])
    flat = np.zeros((1, 32, 32))
    x, ex = R.link_features(raw, [0, 0], flat, half, S)
    z0 = raw[:, 2][:, None] + t[None, :] * (raw[:, 5] - raw[:, 2])[:, None]
    assert np.allclose(ex[:, 1], z0.min(1) / 60.0, atol=1e-13)
    assert np.all(ex[:, 2] == 0.0)
    d = np.linalg.norm(raw[:, 3:6] - raw[:, 0:3], axis=1)
    friis_db = -20 * np.log10(R.C0 / (4 * np.pi * d * raw[:, 6]))
    assert np.allclose(ex[:, 0], (120.0 - friis_db) / 20.0, atol=1e-12)
    assert np.allclose(x[:, 6], [-1.0, 1.0], atol=1e-12)
    assert np.allclose(x[0, :6], [-0.4, 0.08, 25 / 60, 0.6, -0.24, 1.5 / 60], atol=1e-15)
    c = 0.5  # 30 m plateau
    x2, ex2 = R.link_features(raw, [0, 0], np.full((1, 32, 32), c), half, S)
    assert np.allclose(ex2[:, 1], (z0.min(1) - 30.0) / 60.0, atol=1e-13)
    assert np.allclose(ex2[:, 2], np.maximum(30.0 - z0, 0).mean(1) / 60.0, atol=1e-13)


def test_terrain_bilinear_reproduces_linear_maps_and_pixel_centres():
    H, half = 16, 250.0
    pix = 2 * half / H
    cc = -half + (np.arange(H) + 0.5) * pix
    m = 0.3 + 0.01 * cc[None, :] - 0.02 * cc[:, None]  # linear in x and y, row = y
    rng = np.random.default_rng(3)
    px = rng.uniform(cc[0], cc[-1], 200)
    py = rng.uniform(cc[0], cc[-1], 200)
    assert np.allclose(R.terrain(m, px, py, half), 0.3 + 0.01 * px - 0.02 * py, atol=1e-12)
    r, c = rng.integers(0, H, 50), rng.integers(0, H, 50)
    q = rng.uniform(0, 1, (H, H))
    assert np.allclose(R.terrain(q, cc[c], cc[r], half), q[r, c], atol=1e-12)
    # outside the pixel-centre hull the value is clamped to the edge pixel
    assert np.isclose(R.terrain(q, np.array([-half]), np.array([-half]), half)[0], q[0, 0])


def test_link_features_wall_blocks_and_its_depth():
    """A single wall of pixels across the segment: clearance is the segment
    height minus the wall there, obstruction is non-zero only if the wall is
    higher than the segment."""
    H, half = 64, 250.0
    m = np.zeros((1, H, H))
    m[0, :, 32] = 1.0  # 60 m wall along the column whose centre is x = 3.90625 m
    raw = np.array([[-100.0, 0.0, 10.0, 100.0, 0.0, 10.0, 1e11]])
    x, ex = R.link_features(raw, [0], m, half, 1024)
    assert ex[0, 1] < -0.8  # the wall rises about 50 m above the segment
    assert ex[0, 2] > 0.0
    raw2 = np.array([[-100.0, 0.0, 80.0, 100.0, 0.0, 80.0, 1e11]])
    x2, ex2 = R.link_features(raw2, [0], m, half, 1024)
    assert ex2[0, 2] == 0.0
    # the nearest sample lies within half a sample spacing (0.098 m) of the
    # wall's pixel centre, where the bilinear tent (7.8 m pixels) is 60 m high
    step, pix = 200.0 / 1024, 500.0 / 64
    assert (80.0 - 60.0) / 60.0 <= ex2[0, 1] <= (80.0 - 60.0 * (1 - 0.5 * step / pix)) / 60.0 + 1e-12
