"""GPU first-order directive scattering against the oracle (reading R25),
through the C-ABI: the lobe normalisation, the tiles, the scattering paths
(indices exact, lengths to FP64 rounding), per-path fields and the
scattered contribution added to H."""
import sys

import numpy as np
import pytest

from oracle import diffraction as D
from oracle import oracle as O
from oracle import scattering as SC
from paper_2208_10006_amd import workloads as W

pytestmark = pytest.mark.gpu

# relative to the path's whole scattered field |E_s| (both receive
# polarisations), or to its two terms with the Fresnel coefficients at their
# bound 1 where that is larger (the TE and TM terms nearly cancel, or R_TM is
# a near-cancelling quotient near the Brewster angle): the phase
# k (r_i + r_s) ~ 1e5 rad at 300 GHz turns the ~1e-16 relative difference of
# two FP64 lengths into ~1e-11 of the field
AMP_RTOL = 1e-8


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


@pytest.mark.parametrize("alpha", [0, 1, 2, 4, 7, 12, 20, 32])
def test_lobe_norm(S, ctx, alpha):
    """The GPU's closed form (a table of non-negative terms) against the
    oracle's quadrature over the half-space."""
    banner("lobe norm", alpha)
    ci = np.array([1.0, 0.999, 0.9, 0.7, 0.5, 0.3, 0.1, 0.01, 0.0])
    got = S.sbr_scatter_lobe_norm(ctx, alpha, ci)
    want = np.array([SC.lobe_norm(alpha, c, n_theta=200) for c in ci])
    assert np.all(np.abs(got - want) <= 5e-14 * want), np.max(np.abs(got - want) / want)


def _clear_legs(w, tl):
    """(tile, Tx) and (tile, Rx) legs with the point off the tile's plane and
    nothing in the way, counted with the oracle's blocking test."""
    tri = np.asarray(w.tri, np.float64)
    groups = O.scene_groups(w)[0]
    tt, cc, _ = tl
    cnt = 0
    for pts, from_point in ((w.tx, True), (w.rx, False)):
        for P in np.asarray(pts, np.float64):
            for j in range(len(tt)):
                v0, v1, v2 = tri[tt[j]]
                n = np.cross(v1 - v0, v2 - v0)
                n /= np.linalg.norm(n)
                if float(np.dot(P - cc[j], n)) == 0.0:
                    continue
                a, b = (P, cc[j]) if from_point else (cc[j], P)
                cnt += not D._blocked(tri, groups, a, b, (int(groups[tt[j]]),))[0]
    return cnt


def _compare(S, ctx, w, tile_area, alpha, pols=((0, 0), (1, 1), (0, 1)), check_legs=False):
    """GPU tiles, paths, fields and H against the oracle on workload w;
    returns the number of paths compared."""
    sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    d = S.sbr_scatter(ctx, sc, w.tx, w.rx, tile_area, alpha)
    info = S.sbr_scat_info(d)
    tt, cc, aa = SC.tiles(w, tile_area)
    geo, gtri = S.sbr_scat_tiles(d)
    assert info["tiles"] == len(tt) and np.array_equal(gtri, tt)
    scale = max(1.0, float(np.abs(w.tri).max()))
    assert np.allclose(geo[:, :3], cc, rtol=0, atol=1e-13 * scale)
    assert np.allclose(geo[:, 3], aa, rtol=1e-13, atol=0)
    assert info["candidates"] == len(tt) * len(w.tx) * len(w.rx)
    if check_legs:
        assert info["clear_legs"] == _clear_legs(w, (tt, cc, aa))
    ids, rec = S.sbr_scat_paths(d)
    ops = SC.scattering_paths(w, tile_area, tl=(tt, cc, aa))
    print(info, "oracle paths", len(ops), "ambiguous", sum(p.ambiguous for p in ops), flush=True)
    gk = [tuple(x) for x in ids.tolist()]
    ok = {(p.p, p.q, p.tile): p for p in ops}
    gset, oset = set(gk), set(ok)
    for t in gset ^ oset:  # only paths the oracle calls ambiguous may differ
        assert t in ok and ok[t].ambiguous, ("path", t, t in gset)
    assert gk == sorted(gk, key=lambda t: (t[1], t[0], t[2]))  # (rx, tx, tile) order
    common = [i for i, t in enumerate(gk) if t in ok]
    for i in common:
        p = ok[gk[i]]
        assert np.allclose(rec[i], [p.ri, p.rs], rtol=1e-13, atol=0), (gk[i], rec[i], p.ri, p.rs)
    osel = [ok[gk[i]] for i in common]
    for ptx, prx in pols:
        a_g = S.sbr_scat_field(ctx, d, w.freq, w.atm_db_per_m, w.atm_deg_per_m, ptx, prx)
        if common:
            a_o, m_o = SC.scattering_field(w, osel, alpha, atm_db=w.atm_db_per_m, atm_deg=w.atm_deg_per_m,
                                           pol_tx=ptx, pol_rx=prx, with_scale=True)
            a_x = SC.scattering_field(w, osel, alpha, atm_db=w.atm_db_per_m, atm_deg=w.atm_deg_per_m, pol_tx=ptx,
                                      pol_rx=1 - prx)
            den = np.sqrt(np.abs(a_o) ** 2 + np.abs(a_x) ** 2)  # |E_s| . the receive basis of k_s
            assert den.max() > 0, "no scattered power: give the faces roughness"
            den = np.maximum(den, m_o)  # the terms at |R| = 1
            den = np.maximum(den, 1e-6 * den.max())
            err = np.abs(a_g[common] - a_o) / den
            print("pol", ptx, prx, "max rel err", float(err.max()), flush=True)
            assert err.max() <= AMP_RTOL, (ptx, prx, err.max())
        # the channel: H0 + every path of the pair, in both precisions
        rng = np.random.default_rng(7)
        shape = (len(w.freq), len(w.rx), len(w.tx))
        H0 = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * 1e-9
        H128 = H0.copy()
        H64 = H0.astype(np.complex64)
        S.sbr_scat_channel(ctx, d, w.freq, w.atm_db_per_m, w.atm_deg_per_m, ptx, prx, H_c64=H64, H_c128=H128)
        Ho = np.zeros(shape, np.complex128)  # every GPU path's own field, summed per pair
        for i, t in enumerate(gk):
            Ho[:, t[1], t[0]] += a_g[i]
        assert np.allclose(H128 - H0, Ho, rtol=1e-12, atol=1e-14 * max(np.abs(Ho).max(), 1e-300))
        assert np.allclose(H64, (H0.astype(np.complex64).astype(np.complex128) + Ho).astype(np.complex64),
                           rtol=2e-6, atol=1e-6 * np.abs(H0).max())
    return len(common)


def test_single_box(S, ctx):
    """One box, Tx and Rx around it, two frequencies and rough faces (the
    scattered share 1 - rho^2 is non-zero): tiles of 0.1 m^2 on its faces."""
    banner("scattering single box")
    tx = [[3.0, 1.0, 1.0], [-2.0, -1.0, 4.0], [0.5, 5.0, 0.5]]
    rx = [[-1.0, 2.5, 2.2], [2.0, -2.0, 1.5], [0.3, 1.0, 5.0], [4.0, 4.0, 3.5]]
    w = _box(tx, rx, freq=(28e9, 300e9), rough=0.1e-3)
    n = _compare(S, ctx, w, 0.1, 4, check_legs=True)
    assert n >= 100, n


@pytest.mark.parametrize("alpha", [0, 32])
def test_lobe_exponent_limits(S, ctx, alpha):
    """The uniform lobe (alpha = 0) and the narrowest one accepted."""
    banner("scattering box alpha", alpha)
    w = _box([[3.0, 1.0, 1.0]], [[2.0, -2.0, 1.5], [-1.0, 2.5, 2.2]], freq=(140e9,), rough=0.2e-3)
    n = _compare(S, ctx, w, 0.5, alpha, pols=((0, 0), (1, 0)))
    assert n >= 10, n


def test_random_scene_with_atmosphere(S, ctx):
    """Random boxes on ground (per-box materials and roughness), 8 Rx, two
    frequencies with attenuation and dispersion tables, 4 m^2 tiles."""
    banner("scattering random scene 5")
    w = W.random_box_scene(5, n_boxes=12, n_rx=8, freq=(28e9, 140e9))
    w.rough = np.full(len(w.tri), 0.15e-3)
    w.atm_db_per_m = np.array([0.01, 0.02], np.float32)
    w.atm_deg_per_m = np.array([3.0, -2.0], np.float32)
    n = _compare(S, ctx, w, 4.0, 3, pols=((0, 0), (1, 0)))
    assert n >= 100, n


def test_office_one_element(S, ctx):
    """The office hall (5,004 triangles) with one Tx element of the 16 x 16
    MIMO arrays and two of its Rx, 1 m^2 tiles, every face 0.1 mm rough."""
    banner("scattering office 16x16 tx 0, rx 0-1")
    w = W.mimo_office(16, nf=3).subset_tx([0])
    w.rx = w.rx[:2]
    w.rough = np.full(len(w.tri), 0.1e-3)
    n = _compare(S, ctx, w, 1.0, 4, pols=((0, 0),))
    assert n >= 100, n


def test_smooth_faces_scatter_nothing(S, ctx):
    """rho = 1 on smooth faces: paths exist, their fields are zero."""
    banner("scattering smooth box")
    w = _box([[3.0, 1.0, 1.0]], [[2.0, -2.0, 1.5]], rough=0.0)
    sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    d = S.sbr_scatter(ctx, sc, w.tx, w.rx, 0.5, 4)
    assert S.sbr_scat_info(d)["paths"] > 0
    assert np.all(S.sbr_scat_field(ctx, d, w.freq) == 0)


def test_free_space_and_rejects(S, ctx):
    banner("scattering free space, rejects")
    w = W.free_space()
    sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    d = S.sbr_scatter(ctx, sc, w.tx, w.rx, 1.0, 4)
    assert S.sbr_scat_info(d) == {"tiles": 0, "candidates": 0, "clear_legs": 0, "paths": 0}
    H = np.full((1, 1, 1), 1 + 2j)
    S.sbr_scat_channel(ctx, d, w.freq, H_c128=H)
    assert H[0, 0, 0] == 1 + 2j
    wb = _box([[3.0, 1.0, 1.0]], [[2.0, -2.0, 1.5]])
    sb = S.sbr_scene_build(ctx, wb.tri, wb.eps_r, wb.sigma, wb.rough)
    for ta, al in ((0.0, 4), (-1.0, 4), (float("nan"), 4), (1.0, -1), (1.0, 33)):
        with pytest.raises(S.SbrError):
            S.sbr_scatter(ctx, sb, wb.tx, wb.rx, ta, al)
    with pytest.raises(S.SbrError):
        S.sbr_scatter(ctx, sb, np.full((1, 3), np.nan), wb.rx, 1.0, 4)
    # limits, checked before the tile table is built: a triangle of about
    # 1.5 m^2 at 1e-12 m^2 tiles (m ~ 1.2e6), and 12 triangles at 1e-5 m^2
    # (about 1.8 M tiles) x 64 Tx x 64 Rx >= 2^32 candidates
    with pytest.raises(S.SbrError):
        S.sbr_scatter(ctx, sb, wb.tx, wb.rx, 1e-12, 4)
    many = np.concatenate([wb.tx + [0.0, 0.0, 0.01 * i] for i in range(64)])
    with pytest.raises(S.SbrError):
        S.sbr_scatter(ctx, sb, many, many + [0.0, -4.0, 0.0], 1e-5, 4)
    with pytest.raises(S.SbrError):
        S.sbr_scatter_lobe_norm(ctx, 33, np.array([0.5]))
