"""Pins of the surrogate's CPU FP64 reference (test infrastructure): finite
differences for every parameter gradient, the convolution patches against
the direct definition, their adjoint identity, Fourier features at closed-form
points, and bfloat16 rounding."""
import numpy as np
import pytest

from oracle import surrogate_ref as R

SMALL = R.Arch(H=16, chans=(1, 2, 3, 4, 5), E=4, D=3, L=2, F=20, width=6, depth=2, T=2)


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
    return P, hm, x, scene, t, w


def test_gradients_match_finite_differences():
    P, hm, x, scene, t, w = small_problem()
    out, cache = R.forward(SMALL, P, hm, x, scene)
    _, dout = R.mse(out, t, w)
    G = R.backward(SMALL, P, cache, dout)
    eps = 1e-6
    for k, v in P.items():
        flat = v.reshape(-1)
        for i in range(flat.size):
            old = flat[i]
            flat[i] = old + eps
            lp = R.loss_of(SMALL, P, hm, x, scene, t, w)
            flat[i] = old - eps
            lm = R.loss_of(SMALL, P, hm, x, scene, t, w)
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
    P, hm, x, scene, t, w = small_problem(3)
    a, _ = R.forward(SMALL, P, hm, x, scene)
    b, _ = R.forward(SMALL, P, hm, x, scene, use_bf16=True)
    assert np.max(np.abs(a - b)) < 0.05 * max(1.0, np.max(np.abs(a)))
