"""CPU FP64 reference of the radio-map surrogate (test infrastructure only).

Network (the learned part that predicts SBR outputs):
  stem   : four 3x3 / stride-2 / pad-1 convolutions with ReLU on a height
           map [H][W][1] (channels last), then a linear layer with ReLU to an
           embedding of width E, once per scene;
  inputs : per point the embedding of its scene, D raw scalars, their
           Fourier features sin(2^l pi x), cos(2^l pi x), l < L, and X link
           features (free-space gain, terrain clearance and obstruction along
           the Tx-Rx segment over the height map), zero padded to width F;
  MLP    : `depth` hidden linear layers of width Wd with ReLU, then a linear
           layer to T outputs;
  loss   : weighted mean squared error.
Written as plain loops / matrix products in FP64.  With ``bf16=True`` the
values the GPU stores in bfloat16 (weights, activations, GEMM inputs) are
rounded to bfloat16 at the same places; accumulation stays FP64.
Only the test-suite and the benchmark's CPU baseline may import this module.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def bf16(x):
    """Round to bfloat16 (round to nearest even), returned as float64."""
    a = np.asarray(x, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@dataclass
class Arch:
    H: int = 128
    chans: tuple = (1, 16, 32, 64, 128)
    E: int = 128
    D: int = 7
    L: int = 8
    F: int = 256
    width: int = 256
    depth: int = 6
    T: int = 2
    X: int = 3

    @property
    def stem_hw(self):
        return self.H // 2 ** (len(self.chans) - 1)

    @property
    def flat(self):
        return self.stem_hw ** 2 * self.chans[-1]


def conv_patches(x):
    """3x3 stride-2 pad-1 patches: x [n][H][W][C] -> [n*Ho*Wo][9*C], column (ky*3+kx)*C + c."""
    n, H, W, C = x.shape
    Ho, Wo = H // 2, W // 2
    xp = np.zeros((n, H + 2, W + 2, C))
    xp[:, 1:H + 1, 1:W + 1, :] = x
    out = np.zeros((n, Ho, Wo, 9, C))
    for ky in range(3):
        for kx in range(3):
            out[:, :, :, ky * 3 + kx, :] = xp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :]
    return out.reshape(n * Ho * Wo, 9 * C)


def conv_patches_adjoint(dcol, n, H, W, C):
    Ho, Wo = H // 2, W // 2
    d = dcol.reshape(n, Ho, Wo, 9, C)
    dxp = np.zeros((n, H + 2, W + 2, C))
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :] += d[:, :, :, ky * 3 + kx, :]
    return dxp[:, 1:H + 1, 1:W + 1, :]


def fourier(x, L):
    """[n][D] -> [n][2*D*L]: for each d: sin(2^0 pi x), cos(2^0 pi x), sin(2^1 pi x), ..."""
    n, D = x.shape
    out = np.zeros((n, 2 * D * L))
    for d in range(D):
        for l in range(L):
            a = np.pi * (2.0 ** l) * x[:, d]
            out[:, d * 2 * L + 2 * l] = np.sin(a)
            out[:, d * 2 * L + 2 * l + 1] = np.cos(a)
    return out


C0 = 299_792_458.0


def terrain(hmap2d, px, py, half):
    """Bilinear (edge-clamped) interpolation of a height map [H][H] whose pixel
    (r, c) is centred at (-half + (c + 0.5) * 2 half / H, -half + (r + 0.5) * 2 half / H)."""
    H = hmap2d.shape[0]
    pix = 2.0 * half / H
    u = (np.asarray(px, float) + half) / pix - 0.5
    w = (np.asarray(py, float) + half) / pix - 0.5
    c0 = np.clip(np.floor(u).astype(int), 0, H - 2)
    r0 = np.clip(np.floor(w).astype(int), 0, H - 2)
    fu = np.clip(u - c0, 0.0, 1.0)
    fw = np.clip(w - r0, 0.0, 1.0)
    h00, h01 = hmap2d[r0, c0], hmap2d[r0, c0 + 1]
    h10, h11 = hmap2d[r0 + 1, c0], hmap2d[r0 + 1, c0 + 1]
    return (1 - fw) * ((1 - fu) * h00 + fu * h01) + fw * ((1 - fu) * h10 + fu * h11)


def link_features(raw, scene, hmap, half=250.0, samples=128):
    """raw [n][7] = (Tx xyz, Rx xyz in m, f in Hz), hmap [S][H][H] (height / 60)
    -> x [n][7] normalised scalars, extra [n][3] link features:
    free-space path gain (120 - 20 log10(4 pi d f / c)) / 20 (d >= 1 m),
    min over the Tx-Rx segment of (segment height - terrain) / 60, and the
    mean of max(0, terrain - segment height) / 60, terrain sampled at
    (k + 0.5) / samples along the segment."""
    raw = np.asarray(raw, np.float64)
    n = len(raw)
    tx, rx, f = raw[:, 0:3], raw[:, 3:6], raw[:, 6]
    x = np.zeros((n, 7))
    x[:, 0:2] = tx[:, 0:2] / half
    x[:, 2] = tx[:, 2] / 60.0
    x[:, 3:5] = rx[:, 0:2] / half
    x[:, 5] = rx[:, 2] / 60.0
    x[:, 6] = 2.0 * (np.log(f) - np.log(28e9)) / (np.log(300e9) - np.log(28e9)) - 1.0
    d = np.maximum(np.linalg.norm(rx - tx, axis=1), 1.0)
    extra = np.zeros((n, 3))
    extra[:, 0] = (120.0 - 20.0 * np.log10(4.0 * np.pi * d * f / C0)) / 20.0
    for i in range(n):
        t = (np.arange(samples) + 0.5) / samples
        p = tx[i][None, :] + t[:, None] * (rx[i] - tx[i])[None, :]
        h = 60.0 * terrain(np.asarray(hmap[scene[i]], np.float64), p[:, 0], p[:, 1], half)
        extra[i, 1] = np.min(p[:, 2] - h) / 60.0
        extra[i, 2] = np.mean(np.maximum(h - p[:, 2], 0.0)) / 60.0
    return x, extra


def init_params(arch: Arch, seed: int):
    """He-uniform weights, zero biases (the GPU driver uses the same recipe)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = {}
    for i in range(len(arch.chans) - 1):
        fan = 9 * arch.chans[i]
        lim = np.sqrt(6.0 / fan)
        P[f"conv{i}_w"] = rng.uniform(-lim, lim, (fan, arch.chans[i + 1]))
        P[f"conv{i}_b"] = np.zeros(arch.chans[i + 1])
    lim = np.sqrt(6.0 / arch.flat)
    P["emb_w"] = rng.uniform(-lim, lim, (arch.flat, arch.E))
    P["emb_b"] = np.zeros(arch.E)
    fin = arch.F
    for i in range(arch.depth):
        lim = np.sqrt(6.0 / fin)
        P[f"mlp{i}_w"] = rng.uniform(-lim, lim, (fin, arch.width))
        P[f"mlp{i}_b"] = np.zeros(arch.width)
        fin = arch.width
    lim = np.sqrt(6.0 / fin)
    P["out_w"] = rng.uniform(-lim, lim, (fin, arch.T)) * 0.1
    P["out_b"] = np.zeros(arch.T)
    return P


def features(arch, emb, x, scene, r, extra=None):
    f = np.zeros((len(x), arch.F))
    f[:, :arch.E] = emb[scene]
    f[:, arch.E:arch.E + arch.D] = x
    fe = arch.E + arch.D + 2 * arch.D * arch.L
    f[:, arch.E + arch.D:fe] = r(fourier(x, arch.L))
    if arch.X:
        f[:, fe:fe + arch.X] = extra
    return f


def forward(arch: Arch, P, hmap, x, scene, use_bf16=False, extra=None):
    """hmap [S][H][W] (normalised heights), x [n][D], scene [n], extra [n][X] -> out [n][T], cache."""
    r = bf16 if use_bf16 else (lambda a: np.asarray(a, np.float64))
    W = {k: r(v) if k.endswith("_w") else np.asarray(v, np.float64) for k, v in P.items()}
    cache = {"x": x, "scene": scene}
    a = r(hmap[..., None])
    S = a.shape[0]
    hw = arch.H
    for i in range(len(arch.chans) - 1):
        col = conv_patches(a)
        z = col @ W[f"conv{i}_w"] + W[f"conv{i}_b"]
        a_new = r(np.maximum(z, 0.0))
        cache[f"conv{i}"] = (col, a_new, a.shape)
        hw //= 2
        a = a_new.reshape(S, hw, hw, arch.chans[i + 1])
    flat = a.reshape(S, -1)
    emb = r(np.maximum(flat @ W["emb_w"] + W["emb_b"], 0.0))
    cache["flat"], cache["emb"] = flat, emb
    h = r(features(arch, emb, x, scene, r, extra))
    cache["feat"] = h
    for i in range(arch.depth):
        hn = r(np.maximum(h @ W[f"mlp{i}_w"] + W[f"mlp{i}_b"], 0.0))
        cache[f"mlp{i}"] = (h, hn)
        h = hn
    out = h @ W["out_w"] + W["out_b"]
    cache["last"] = h
    cache["W"] = W
    return out, cache


def mse(out, target, weight):
    """loss = sum w (out - t)^2 / sum w, and its gradient."""
    cnt = max(float(np.sum(weight)), 1.0)
    rres = out - target
    return float(np.sum(weight * rres * rres) / cnt), 2.0 * weight * rres / cnt


def backward(arch: Arch, P, cache, dout, use_bf16=False):
    """Gradients of all parameters for d loss / d out = dout.  use_bf16: each
    layer's output gradient is rounded to bfloat16 once and both its weight
    and its bias gradient are formed from the rounded value."""
    r = bf16 if use_bf16 else (lambda a: np.asarray(a, np.float64))
    W = cache["W"]
    G = {}
    g = r(dout)
    G["out_w"] = cache["last"].T @ g
    G["out_b"] = g.sum(axis=0)
    dh = g @ W["out_w"].T
    for i in reversed(range(arch.depth)):
        h_in, h_out = cache[f"mlp{i}"]
        dzr = r(dh * (h_out > 0))
        G[f"mlp{i}_b"] = dzr.sum(axis=0)
        G[f"mlp{i}_w"] = h_in.T @ dzr
        dh = dzr @ W[f"mlp{i}_w"].T
    S = cache["emb"].shape[0]
    demb = np.zeros((S, arch.E))
    np.add.at(demb, cache["scene"], r(dh[:, :arch.E]))
    dzr = r(demb * (cache["emb"] > 0))
    G["emb_b"] = dzr.sum(axis=0)
    G["emb_w"] = cache["flat"].T @ dzr
    da = dzr @ W["emb_w"].T
    for i in reversed(range(len(arch.chans) - 1)):
        col, a_out, in_shape = cache[f"conv{i}"]
        dzr = r(da.reshape(a_out.shape) * (a_out > 0))
        G[f"conv{i}_b"] = dzr.sum(axis=0)
        G[f"conv{i}_w"] = col.T @ dzr
        if i > 0:
            dcol = dzr @ W[f"conv{i}_w"].T
            n, H, Wd, C = in_shape
            da = conv_patches_adjoint(dcol, n, H, Wd, C)
    return G


def loss_of(arch, P, hmap, x, scene, target, weight, extra=None):
    out, _ = forward(arch, P, hmap, x, scene, extra=extra)
    return mse(out, target, weight)[0]
