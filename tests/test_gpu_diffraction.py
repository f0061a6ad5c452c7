"""GPU first-order edge diffraction against the oracle (reading R24), through
the C-ABI: the transition function, the scene's wedges, the diffraction
paths (indices exact, geometry to FP64 rounding), per-path fields and the
diffracted contribution added to H."""
import sys

import numpy as np
import pytest

from oracle import diffraction as D
from oracle import oracle as O
from paper_2208_10006_amd import workloads as W

pytestmark = pytest.mark.gpu

# the reflection paths' amplitude tolerance: the phase k (s + s') ~ 1e4 rad
# turns the ~1e-15 relative difference of two FP64 geometries into ~1e-11 of
# the field, and near a shadow or reflection boundary the coefficient's
# sensitivity to the angles multiplies that (1e-8 measured 4e-3 rad from one)
AMP_RTOL = 1e-7


@pytest.fixture(scope="module")
def S():
    from paper_2208_10006_amd import sbr
    return sbr


@pytest.fixture(scope="module")
def ctx(S):
    return S.Context(0)


def banner(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _box(tx, rx, freq=(28e9,), sigma=0.0326, rough=0.0):
    tris = W.box_triangles((0.0, 0.0, 0.0), (1.0, 2.0, 3.0))
    T = len(tris)
    tri, e, s, r = W._pack(tris, [5.31] * T, [sigma] * T, [rough] * T)
    return W.Workload("box", tri, e, s, r, np.array(tx, float), np.array(rx, float), np.array(freq, float),
                      geodesic_N=16, max_bounces=1)


def test_transition_function(S, ctx):
    """The GPU's series (X < 5), continued fraction (5 <= X < 80) and asymptotic series (X >= 80) against the
    oracle's Fresnel-integral form (itself good to ~1e-11 at X ~ 1e5)."""
    banner("utd transition")
    X = np.concatenate([[0.0], np.logspace(-9, 5, 281), [4.999999, 5.0, 5.000001, 7.99, 8.0, 19.99, 20.0, 79.999999, 80.0]])
    got = S.sbr_utd_transition(ctx, X)
    want = D.transition(X)
    tol = 1e-12 * np.maximum(np.abs(want), 1e-6) + 5e-11 * (X > 1e3)
    assert np.all(np.abs(got - want) <= tol), np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-30))


def _scene_cases():
    return {"box": lambda: _box([[3.0, 1.0, 1.0]], [[-1.0, 2.5, 2.2]]),
            "random": lambda: W.random_box_scene(5, n_boxes=12),
            "urban": lambda: W.urban_canyon(),
            "office": lambda: W.massive_mimo_office(nf=4)}


@pytest.mark.parametrize("which", ["box", "random", "urban", "office"])
def test_wedges_match_oracle(S, ctx, which):
    banner("wedges", which)
    w = _scene_cases()[which]()
    sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    geo, grp = S.sbr_scene_wedges(ctx, sc)
    wd = D.wedges(w)
    assert len(wd) == len(geo) and len(wd) > 0
    a = np.array([x.a for x in wd])
    b = np.array([x.b for x in wd])
    assert np.array_equal(geo[:, 0:3], a)
    assert np.allclose(geo[:, 3:6], b, rtol=0, atol=1e-12 * max(1.0, np.abs(b).max()))
    assert np.allclose(geo[:, 6], [x.n for x in wd], rtol=0, atol=1e-13)
    assert np.array_equal(grp, np.array([[x.g0, x.gn] for x in wd]))


def _compare(S, ctx, w, pols=((0, 0), (1, 1), (0, 1))):
    """GPU paths, fields and H against the oracle on workload w; returns the
    number of paths compared."""
    sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    d = S.sbr_diffract(ctx, sc, w.tx, w.rx)
    info = S.sbr_diff_info(d)
    ids, rec = S.sbr_diff_paths(d)
    wd = D.wedges(w)
    ops = D.diffraction_paths(w, wd)
    print(info, "oracle paths", len(ops), "ambiguous", sum(p.ambiguous for p in ops), flush=True)
    assert info["wedges"] == len(wd)
    assert info["candidates"] == len(wd) * len(w.tx) * len(w.rx)
    gk = [tuple(x) for x in ids.tolist()]
    ok = {(p.p, p.q, p.wedge): p for p in ops}
    gset, oset = set(gk), set(ok)
    for t in gset ^ oset:  # only paths the oracle calls ambiguous may differ
        assert t in ok and ok[t].ambiguous, ("path", t, t in gset)
    assert gk == sorted(gk, key=lambda t: (t[1], t[0], t[2]))  # (rx, tx, wedge) order
    common = [i for i, t in enumerate(gk) if t in ok]
    for i in common:
        p = ok[gk[i]]
        want = np.array([*p.Q, p.sp, p.s, p.beta0, p.phip, p.phi])
        assert np.allclose(rec[i], want, rtol=1e-12, atol=1e-12 * (1 + np.abs(p.Q).max())), (gk[i], rec[i], want)
    osel = [ok[gk[i]] for i in common]
    for ptx, prx in pols:
        a_g = S.sbr_diff_field(ctx, d, w.freq, w.atm_db_per_m, w.atm_deg_per_m, ptx, prx)
        a_o, m_o = D.diffraction_field(w, osel, wd, atm_db=w.atm_db_per_m, atm_deg=w.atm_deg_per_m, pol_tx=ptx,
                                       pol_rx=prx, with_scale=True)
        if common:
            # relative to the magnitude each value is a sum of (a cross-polar
            # value is a near cancellation of the soft and hard terms)
            den = np.maximum(m_o, 1e-6 * m_o.max())
            err = np.abs(a_g[common] - a_o) / den
            assert err.max() <= AMP_RTOL, (ptx, prx, err.max())
        # the channel: H0 + every path of the pair, in both precisions
        rng = np.random.default_rng(7)
        shape = (len(w.freq), len(w.rx), len(w.tx))
        H0 = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * 1e-9
        H128 = H0.copy()
        H64 = H0.astype(np.complex64)
        S.sbr_diff_channel(ctx, d, w.freq, w.atm_db_per_m, w.atm_deg_per_m, ptx, prx, H_c64=H64, H_c128=H128)
        Hg = H128 - H0
        Ho = np.zeros(shape, np.complex128)  # every GPU path's own field, summed per pair
        for i, t in enumerate(gk):
            Ho[:, t[1], t[0]] += a_g[i]
        assert np.allclose(Hg, Ho, rtol=1e-12, atol=1e-14 * max(np.abs(Ho).max(), 1e-300))
        assert np.allclose(H64, (H0.astype(np.complex64).astype(np.complex128) + Ho).astype(np.complex64),
                           rtol=2e-6, atol=1e-6 * np.abs(H0).max())
    return len(common)


def test_single_box(S, ctx):
    """One box, Tx and Rx around it (shadowed and lit links), two frequencies
    and rough faces: every vertical and horizontal edge in view."""
    banner("diffraction single box")
    tx = [[3.0, 1.0, 1.0], [-2.0, -1.0, 4.0], [0.5, 5.0, 0.5]]
    rx = [[-1.0, 2.5, 2.2], [2.0, -2.0, 1.5], [0.3, 1.0, 5.0], [4.0, 4.0, 3.5]]
    w = _box(tx, rx, freq=(28e9, 140e9), rough=0.1e-3)
    n = _compare(S, ctx, w)
    assert n >= 10, n


def test_random_scene_with_atmosphere(S, ctx):
    """Random boxes on ground (per-box materials and roughness), 8 Rx, two
    frequencies with attenuation and dispersion tables."""
    banner("diffraction random scene 5")
    w = W.random_box_scene(5, n_boxes=12, n_rx=8, freq=(28e9, 60e9))
    w.atm_db_per_m = np.array([0.01, 0.02], np.float32)
    w.atm_deg_per_m = np.array([3.0, -2.0], np.float32)
    n = _compare(S, ctx, w, pols=((0, 0), (1, 0)))
    assert n >= 5, n


def test_office_two_elements(S, ctx):
    """The office hall (5,004 triangles, 4,992 convex desk and partition
    edges, 12 concave hall edges) with two Tx elements of the 16 x 16 MIMO
    arrays and its 16 Rx."""
    banner("diffraction office 16x16 tx 0, 15")
    w = W.mimo_office(16, nf=3).subset_tx([0, 15])
    n = _compare(S, ctx, w, pols=((0, 0),))
    assert n >= 1, n


def test_no_wedges_no_paths(S, ctx):
    banner("diffraction free space")
    w = W.free_space()
    sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    d = S.sbr_diffract(ctx, sc, w.tx, w.rx)
    assert S.sbr_diff_info(d) == {"wedges": 0, "candidates": 0, "geometric": 0, "paths": 0}
    H = np.full((1, 1, 1), 1 + 2j)
    S.sbr_diff_channel(ctx, d, w.freq, H_c128=H)
    assert H[0, 0, 0] == 1 + 2j
    with pytest.raises(S.SbrError):
        S.sbr_diffract(ctx, sc, np.full((1, 3), np.nan), w.rx)
