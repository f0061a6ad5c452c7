"""What the FP64 parts of the path buy, measured on the CPU from the oracle's
paths of a reduced urban canyon (200 Rx, 16 subcarriers at 300 GHz, up to six
reflections at up to 500 m):

* every valid path's chain of specular points re-propagated with an FP32 ray
  state (origin, direction and plane in FP32, one step per reflection) drifts
  from the FP64 chain by a fraction of the oracle's FP32-resolution ambiguity
  band 4e-6 (|P - centre| + t) that grows with the bounce (the FP64 state
  keeps it at rounding level);
* the phase 2 pi frac(f d / c) evaluated with f d / c in FP32 (about 5e5
  cycles) breaks the H tolerance (1e-5 per entry, floor 1e-6 max|H|) on a
  large share of the entries, so the phase must be FP64;
* path amplitudes rounded to complex64 (FP64 phase and FP64 sum) stay well
  inside the H tolerance.
The measured values are printed (pytest -s) and recorded with the design."""
import math

import numpy as np

from oracle import oracle as O
from paper_2208_10006_amd import workloads as W

C0 = 299792458.0


def _case():
    w = W.urban_canyon(N=48, n_rx=200, nf=16)
    return w, O.run(w)


def _planes(w):
    g, _, ng = O.scene_groups(w)
    tri = np.asarray(w.tri)
    n = np.zeros((ng, 3))
    c = np.zeros(ng)
    for G in range(ng):
        t = int(np.where(g == G)[0][0])
        v = np.cross(tri[t, 1] - tri[t, 0], tri[t, 2] - tri[t, 0])
        n[G] = v / np.linalg.norm(v)
        c[G] = n[G] @ tri[t, 0]
    pts = tri.reshape(-1, 3)
    return n, c, 0.5 * (pts.min(0) + pts.max(0))


def _chain(w, key, n, c):
    """Specular points of a valid key by the image method (FP64)."""
    p, q, k = (int(x) for x in key[:3])
    gs = [int(x) for x in key[3:3 + k]]
    imgs = [np.asarray(w.tx[p], float)]
    for G in gs:
        x = imgs[-1]
        imgs.append(x - 2 * (n[G] @ x - c[G]) * n[G])
    X = [None] * (k + 2)
    X[0], X[k + 1] = imgs[0], np.asarray(w.rx[q], float)
    for j in range(k, 0, -1):
        a, b, G = imgs[j], X[j + 1], gs[j - 1]
        da, db = n[G] @ a - c[G], n[G] @ b - c[G]
        X[j] = a + (b - a) * (da / (da - db))
    return gs, X


def test_fp32_ray_state_drift_against_the_band():
    w, r = _case()
    n, c, ctr = _planes(w)
    worst = {}
    for key in r.keys[r.valid]:
        if key[2] == 0:
            continue
        gs, X = _chain(w, key, n, c)
        o = (X[0] - ctr).astype(np.float32)
        d = X[1] - X[0]
        d = (d / np.linalg.norm(d)).astype(np.float32)
        for j, G in enumerate(gs, start=1):
            n32 = n[G].astype(np.float32)
            c32 = np.float32(c[G] - n[G] @ ctr)
            t = (c32 - n32 @ o) / (n32 @ d)
            o = (o + d * t).astype(np.float32)
            d = (d - np.float32(2) * (n32 @ d) * n32).astype(np.float32)
            ex = X[j] - ctr
            ratio = np.linalg.norm(o.astype(float) - ex) / (4e-6 * (np.linalg.norm(ex) + float(t)))
            worst[j] = max(worst.get(j, 0.0), ratio)
    print("FP32 ray state: worst drift / ambiguity band per bounce", {j: round(v, 3) for j, v in worst.items()})
    assert len(worst) == 6
    assert worst[6] > 5 * worst[1]          # the drift accumulates with the bounces
    assert max(worst.values()) > 0.1        # and reaches a sizeable share of the band


def test_fp32_phase_breaks_h_and_complex64_amplitudes_do_not():
    w, r = _case()
    keys, a64, H64 = r.keys[r.valid], r.a, r.H
    length = r.rec[r.valid][:, 1]
    cyc64 = np.outer(length, w.freq) / C0
    cyc32 = (np.outer(length.astype(np.float32), w.freq.astype(np.float32)) / np.float32(C0)).astype(np.float64)
    mx = np.abs(H64).max()
    den = np.maximum(np.abs(H64), 1e-6 * mx)

    def herr(a):
        H = O.channel_matrix(keys, a, len(w.tx), len(w.rx))
        return np.abs(H - H64) / den

    e_ph = herr(a64 * np.exp(-2j * math.pi * (cyc32 - cyc64)))
    e_c64 = herr(a64.astype(np.complex64).astype(np.complex128))
    print(f"FP32 phase: max per-entry H error {e_ph.max():.3g}, entries above 1e-5 {np.mean(e_ph > 1e-5):.3f}; "
          f"complex64 amplitudes: max {e_c64.max():.3g}")
    assert e_ph.max() > 1e-2 and np.mean(e_ph > 1e-5) > 0.1
    assert e_c64.max() < 1e-5
