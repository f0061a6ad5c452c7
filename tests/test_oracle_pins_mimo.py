"""Pins of the oracle's per-port received power (eq. (14), Sec. IV-C, Fig. 7)
and of the n x n MIMO office arrays, against closed forms that do not share
the oracle's formula."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_10006_amd import workloads as W

C0 = 299792458.0
EPS0 = 8.8541878128e-12


def exhaustive_coeff(N):
    m, lo, hi = O.edge_stats(N)
    return 1.05 * hi / m


def test_port_power_two_tones_dirichlet():
    """H_f = A e^{-j 2 pi f t1} + B e^{-j 2 pi f t2} on f_k = f0 + k df: the band
    mean of |H|^2 is A^2 + B^2 + (2AB / Nf) sum_k cos(x0 + k x), and that sum is
    the Dirichlet-kernel closed form sin(Nf x / 2) / sin(x / 2) cos(x0 + (Nf-1) x / 2)
    with x0 = 2 pi f0 dt, x = 2 pi df dt, dt = t2 - t1."""
    rng = np.random.default_rng(3)
    for Nf in (1, 2, 7, 64, 1000):
        A, B = rng.uniform(0.1, 2.0, 2)
        t1, t2 = rng.uniform(1e-9, 50e-9, 2)
        f0, df = 28e9, 1.7e6
        f = f0 + df * np.arange(Nf)
        H = (A * np.exp(-2j * np.pi * f * t1) + B * np.exp(-2j * np.pi * f * t2))[:, None, None]
        dt = t2 - t1
        x0, x = 2 * np.pi * f0 * dt, 2 * np.pi * df * dt
        dirichlet = math.sin(Nf * x / 2) / math.sin(x / 2) * math.cos(x0 + (Nf - 1) * x / 2)
        want = A * A + B * B + 2 * A * B * dirichlet / Nf
        got = O.port_power(H)[0, 0]
        assert abs(got - want) <= 1e-9 * (A + B) ** 2, (Nf, got, want)


def test_port_power_free_space_arrays_friis():
    """Free space, 2 Tx x 3 Rx points, three frequencies: one line-of-sight path
    per pair, so P[q][p] = band mean of (lambda_f / (4 pi d_qp))^2 (Friis)."""
    tx = np.array([[0.0, 0.0, 1.5], [0.0, 0.7, 1.5]])
    rx = np.array([[5.0, 3.0, 1.5], [6.0, -2.0, 1.0], [3.0, 1.0, 2.5]])
    freq = np.array([28e9, 60e9, 100e9])
    tri, e, s, r = W._pack([], [], [], [])
    w = W.Workload("free_space_arrays", tri, e, s, r, tx, rx, freq, geodesic_N=8, max_bounces=1)
    res = O.run(w, coeff=exhaustive_coeff(8))
    P = O.port_power(res.H)
    assert P.shape == (3, 2)
    for q in range(3):
        for p in range(2):
            d = float(np.linalg.norm(rx[q] - tx[p]))
            want = np.mean((C0 / freq / (4 * np.pi * d)) ** 2)
            assert abs(P[q, p] / want - 1) < 1e-12, (q, p)


def test_port_power_line_of_sight_plus_wall_reflection():
    """Tx and Rx on one normal of a wall, 3 m apart, the wall 2 m behind the Tx:
    line of sight (3 m) plus the normal-incidence reflection (7 m).  Per
    frequency h = lambda/(4 pi) (e^{-jk 3}/3 + Gamma e^{-jk 7}/7) with the
    closed-form normal-incidence Fresnel coefficient; the band mean of |h|^2
    depends on the relative phase of the two paths (combined with phase, not
    in power: the incoherent sum differs by up to 2 |a1 a2|)."""
    freq = np.linspace(28e9, 28.3e9, 9)
    w = W.one_plane(tx=(2.0, 0.3, 0.2), rx=(5.0, 0.3, 0.2), freq=freq, K=1, N=32)
    res = O.run(w, coeff=exhaustive_coeff(32))
    er, sg = (float(np.float32(x)) for x in (5.31, 0.0326))
    vals = []
    for f in freq:
        ec = er - 1j * sg / (2 * math.pi * f * EPS0)
        gam = (1 - np.sqrt(ec)) / (1 + np.sqrt(ec))
        lam = C0 / f
        h = lam / (4 * math.pi) * (np.exp(-2j * math.pi * ((f * 3.0 / C0) % 1)) / 3.0
                                   + gam * np.exp(-2j * math.pi * ((f * 7.0 / C0) % 1)) / 7.0)
        vals.append(abs(h) ** 2)
    want = float(np.mean(vals))
    P = O.port_power(res.H)
    assert abs(P[0, 0] / want - 1) < 1e-9
    incoherent = float(np.mean(np.sum(np.abs(res.a) ** 2, axis=0)))
    assert abs(incoherent / want - 1) > 1e-3  # the phase matters on this band


def test_port_power_sums_to_band_mean_frobenius():
    """sum over ports of P equals Q, the band mean of ||H_f||_F^2 that the
    capacity normalisation uses (eq. (15)-(17) reading), for any H."""
    rng = np.random.default_rng(9)
    H = rng.standard_normal((5, 4, 3)) + 1j * rng.standard_normal((5, 4, 3))
    Q = np.mean([np.linalg.norm(H[f], "fro") ** 2 for f in range(5)])
    assert abs(O.port_power(H).sum() / Q - 1) < 1e-13


@pytest.mark.parametrize("n,shape", [(16, (4, 4)), (32, (4, 8)), (64, (8, 8)), (128, (8, 16))])
def test_mimo_office_arrays(n, shape):
    """n x n MIMO: n Tx and n Rx elements in UPAs of the stated shape at
    lambda/2 (1.5 mm at 100 GHz), centred on the office's array positions."""
    w = W.mimo_office(n, nf=4)
    assert w.meta["upa"] == shape and len(w.tx) == n and len(w.rx) == n
    lam = C0 / 100e9
    for arr, c in ((w.tx, W.OFFICE_TX), (w.rx, W.OFFICE_RX)):
        assert np.allclose(arr.mean(0), c, atol=1e-12)
        d = np.linalg.norm(arr[:, None] - arr[None], axis=2) + np.eye(n) * 1e9
        assert abs(d.min() - lam / 2) < 1e-12
        assert np.all(arr[:, 0] == c[0])  # the y-z plane
    assert w.T == W.massive_mimo_office(nf=4).T
