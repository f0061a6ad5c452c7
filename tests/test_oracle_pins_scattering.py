"""Pins of the oracle's first-order directive scattering (reading R25: the
effective-roughness single-lobe model with the Kirchhoff roughness factor
deciding the scattered share) against closed forms and against the
reflection oracle: the lobe normalisation's closed forms, the tiling, the
same-side rule, and the specular direction, where the scattered field must
be the reflected field scaled by the ratio of the two models' magnitudes."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import scattering as SC
from paper_2208_10006_amd import workloads as W


@pytest.mark.parametrize("cos_i", [1.0, 0.8, 0.3, 0.01])
def test_lobe_norm_closed_forms(cos_i):
    """alpha = 0: the half-space, 2 pi; alpha = 1: (2 pi + pi cos theta_i) / 2
    (the half-space mean of s is n / 2); alpha = 2: adds the second moment
    2 pi / 3 of s s^T over the half-space."""
    assert abs(SC.lobe_norm(0, cos_i) - 2 * math.pi) < 1e-12
    assert abs(SC.lobe_norm(1, cos_i) - (2 * math.pi + math.pi * cos_i) / 2) < 1e-12
    want2 = (2 * math.pi + 2 * math.pi * cos_i + 2 * math.pi / 3) / 4
    assert abs(SC.lobe_norm(2, cos_i) - want2) < 1e-12


@pytest.mark.parametrize("alpha", [0, 1, 3, 4, 8, 16])
def test_lobe_norm_normal_incidence(alpha):
    """At normal incidence cos psi = cos theta: F = 4 pi (1 - 2^-(alpha+1)) / (alpha + 1)."""
    want = 4 * math.pi * (1 - 2.0 ** (-(alpha + 1))) / (alpha + 1)
    assert abs(SC.lobe_norm(alpha, 1.0) - want) < 1e-12 * want


def test_tiles_partition_each_triangle():
    tris = W.box_triangles((0.0, 0.0, 0.0), (1.0, 2.0, 3.0))
    T = len(tris)
    tri, e, s, r = W._pack(tris, [5.0] * T, [0.01] * T, [0.0] * T)
    w = W.Workload("box", tri, e, s, r, np.zeros((1, 3)), np.ones((1, 3)), np.array([28e9]))
    tt, cc, aa = SC.tiles(w, 0.1)
    for t in range(T):
        sel = tt == t
        v0, v1, v2 = w.tri[t]
        A = 0.5 * np.linalg.norm(np.cross(v1 - v0, v2 - v0))
        m = max(1, math.ceil(math.sqrt(A / 0.1)))
        assert sel.sum() == m * m
        assert abs(aa[sel].sum() - A) < 1e-12 * A
        # equal areas: the area-weighted centroid is the triangle's centroid
        assert np.allclose((cc[sel] * aa[sel, None]).sum(0) / A, (v0 + v1 + v2) / 3, atol=1e-12)
        # every centroid lies in the triangle's plane
        n = np.cross(v1 - v0, v2 - v0)
        assert np.allclose((cc[sel] - v0) @ n, 0.0, atol=1e-12)


def _wall(rough=0.2e-3, tile=0.5):
    tris, eps_r, sigma, rgh = W.vertical_plane(rough=rough)
    T = len(tris)
    tri, e, s, r = W._pack(tris, [eps_r] * T, [sigma] * T, [rgh] * T)
    return tri, e, s, r


def test_specular_direction_is_the_reflection_scaled():
    """Rx placed exactly in the specular direction from a tile's centroid C:
    C is then the specular point of the wall for that Tx and Rx, the
    scattered field has the reflected field's polarisation and phase, and
    a_s / a_r = [sqrt(dS cos theta_i / F) sqrt(1 - rho^2) / (r_i r_s)] /
    [rho / (r_i + r_s)] -- the reflection from the image-method oracle."""
    tri, e, s, r = _wall()
    f = np.array([140e9, 300e9])
    tx = np.array([4.0, 1.0, 2.0])
    w0 = W.Workload("wall", tri, e, s, r, tx[None], np.array([[6.0, 3.0, 1.0]]), f, geodesic_N=8, max_bounces=1)
    tt, cc, aa = SC.tiles(w0, 400.0)
    j = int(np.argmin(np.linalg.norm(cc - np.array([0.0, 2.0, 1.5]), axis=1)))
    C = cc[j]
    n = np.array([1.0, 0.0, 0.0])
    ki = (C - tx) / np.linalg.norm(C - tx)
    kr = ki - 2 * np.dot(ki, n) * n
    rx = C + 7.0 * kr
    w = W.Workload("wall", tri, e, s, r, tx[None], rx[None], f, geodesic_N=8, max_bounces=1)
    ps = [p for p in SC.scattering_paths(w, 400.0, tl=(tt, cc, aa)) if p.tile == j]
    assert len(ps) == 1
    d = ps[0]
    _, _, ng = O.scene_groups(w)
    for pol in (0, 1):
        a_s = SC.scattering_field(w, ps, 4, pol_tx=pol, pol_rx=pol)[0]
        keys = np.array([[0, 0, 1, g] for g in range(ng)], np.int32)
        a_r = O.field(w, keys, pol_tx=pol, pol_rx=pol).sum(axis=0)
        cs = -float(np.dot(ki, -n)) if np.dot(ki, n) > 0 else -float(np.dot(ki, n))
        F = SC.lobe_norm(4, cs)
        for fi, fr in enumerate(f):
            rho = O.roughness(float(np.float32(r[0])), fr, cs)
            want = (math.sqrt(d.dS * cs / F) * math.sqrt(1 - rho * rho) / (d.ri * d.rs)) / (rho / (d.ri + d.rs))
            ratio = a_s[fi] / a_r[fi]
            assert abs(ratio - want) <= 1e-9 * want, (pol, fr, ratio, want)


def test_lobe_peaks_in_the_specular_direction_and_same_side_rule():
    tri, e, s, r = _wall()
    f = np.array([300e9])
    tx = np.array([4.0, 1.0, 2.0])
    C0_ = np.array([0.0, 2.0, 1.5])
    n = np.array([1.0, 0.0, 0.0])
    ki = (C0_ - tx) / np.linalg.norm(C0_ - tx)
    kr = ki - 2 * np.dot(ki, n) * n
    mags = []
    for ang in (0.0, 0.2, 0.5, 0.9):   # rotate the Rx direction away from specular about z
        c, sn = math.cos(ang), math.sin(ang)
        d = np.array([kr[0] * c - kr[1] * sn, kr[0] * sn + kr[1] * c, kr[2]])
        rx = C0_ + 7.0 * d
        w = W.Workload("wall", tri, e, s, r, tx[None], rx[None], f, geodesic_N=8, max_bounces=1)
        tl = (np.array([0]), C0_[None], np.array([0.25]))
        ps = SC.scattering_paths(w, 0.25, tl=tl)
        assert len(ps) == 1
        mags.append(abs(SC.scattering_field(w, ps, 4)[0, 0]) * ps[0].ri * ps[0].rs)
    assert all(a > b for a, b in zip(mags, mags[1:]))
    # Rx behind the wall: no scattering path
    w = W.Workload("wall", tri, e, s, r, tx[None], np.array([[-3.0, 2.0, 1.0]]), f, geodesic_N=8, max_bounces=1)
    assert SC.scattering_paths(w, 0.25, tl=(np.array([0]), C0_[None], np.array([0.25]))) == []


def test_field_scale_is_the_terms_at_unit_fresnel_coefficients():
    """with_scale: with Tx, the tile and Rx at one height on a vertical wall
    the plane of incidence is horizontal, so a theta-polarised wave is pure
    TE and a phi-polarised one pure TM: one term, |a| = scale |R_TE| or
    scale |R_TM| (eq. (6)-(7)).  On a random scene |a| <= scale (triangle
    inequality and |R| <= 1), strictly where both terms are present."""
    tri, e, s, r = _wall()
    f = np.array([28e9, 140e9])
    w0 = W.Workload("wall", tri, e, s, r, np.array([[4.0, 1.0, 2.0]]), np.array([[6.0, 3.0, 1.0]]), f,
                    geodesic_N=8, max_bounces=1)
    tt, cc, aa = SC.tiles(w0, 400.0)
    j = int(np.argmin(np.linalg.norm(cc - np.array([0.0, 2.0, 1.5]), axis=1)))
    C = cc[j]
    tx = np.array([4.0, 1.0, C[2]])
    rx = np.array([5.0, 6.0, C[2]])
    w = W.Workload("wall", tri, e, s, r, tx[None], rx[None], f, geodesic_N=8, max_bounces=1)
    ps = [p for p in SC.scattering_paths(w, 400.0, tl=(tt, cc, aa)) if p.tile == j]
    assert len(ps) == 1
    d = ps[0]
    ki = (d.C - tx) / d.ri
    cs = abs(ki[0])  # the wall's normal is the x axis
    for pol in (0, 1):
        a, m = SC.scattering_field(w, ps, 4, pol_tx=pol, pol_rx=pol, with_scale=True)
        assert np.all(np.abs(a) > 0)
        R = np.array([abs(O.fresnel(float(np.float32(e[0])), float(np.float32(s[0])), fr, cs)[pol]) for fr in f])
        assert np.allclose(np.abs(a), m * R, rtol=1e-12, atol=0), (pol, np.abs(a), m, R)
    wr = W.random_box_scene(5, n_boxes=6, n_rx=3, freq=(28e9,))
    wr.rough = np.full(len(wr.tri), 0.15e-3)
    ps = SC.scattering_paths(wr, 4.0)
    assert len(ps) > 50
    for prx in (0, 1):
        a, m = SC.scattering_field(wr, ps, 3, pol_tx=0, pol_rx=prx, with_scale=True)
        assert np.all(np.abs(a) <= m * (1 + 1e-12))
        assert np.any(np.abs(a) < 0.9 * m)
