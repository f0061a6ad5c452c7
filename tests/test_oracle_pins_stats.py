"""Pins of the oracle's per-link statistics over paths of every mechanism
(Table I's quantities from reflection, diffraction and scattering paths
together): the departure and arrival angles and delays of diffraction and
scattering paths at hand-computed geometries (reading R17's senses), and
the per-link statistics on closed forms."""
import math

import numpy as np

from oracle import diffraction as D
from oracle import oracle as O
from oracle import scattering as SC
from paper_2208_10006_amd import workloads as W

C0 = 299792458.0


def _box_workload(tx, rx):
    tris = W.box_triangles((0.0, 0.0, 0.0), (1.0, 2.0, 3.0))
    T = len(tris)
    tri, e, s, r = W._pack(tris, [5.31] * T, [0.0326] * T, [0.0] * T)
    return W.Workload("box", tri, e, s, r, np.array([tx], float), np.array([rx], float), np.array([28e9]),
                      geodesic_N=16, max_bounces=1)


def test_diffraction_records_on_a_vertical_edge():
    """Tx and Rx at distance sqrt(5) from the box's vertical edge x = 1, y = 2,
    at heights 0.5 and 2.5: Keller's cone puts Q at the height midway,
    Q = (1, 2, 1.5); departure along (-2, 1, 1) / sqrt(6), arrival (Rx -> Q)
    along (-1, -2, -1) / sqrt(6), delay 2 sqrt(6) / c."""
    w = _box_workload((3.0, 1.0, 0.5), (2.0, 4.0, 2.5))
    wd = D.wedges(w)
    ps = [p for p in D.diffraction_paths(w, wd)
          if np.allclose(sorted([tuple(wd[p.wedge].a), tuple(wd[p.wedge].b)]), [(1.0, 2.0, 0.0), (1.0, 2.0, 3.0)])]
    assert len(ps) == 1
    assert np.allclose(ps[0].Q, [1.0, 2.0, 1.5], atol=1e-12)
    rec = D.path_records(w, ps)[0]
    el = math.degrees(math.asin(1.0 / math.sqrt(6.0)))  # 24.0948 degrees
    want = [2.0 * math.sqrt(6.0) / C0, 153.43494882292202, el, -116.56505117707799, -el]
    assert np.allclose(rec, want, rtol=1e-12, atol=1e-10), (rec, want)


def test_scattering_records_on_a_wall_tile():
    """Tile centroid C = (0, 2, 1.5) on the wall x = 0, Tx (4, 1, 2), Rx
    (6, 3, 1): departure along (-4, 1, -0.5), arrival (Rx -> C) along
    (-6, -1, 0.5), delay (|(-4, 1, -0.5)| + |(-6, -1, 0.5)|) / c."""
    tris, eps_r, sigma, rgh = W.vertical_plane(rough=0.1e-3)
    T = len(tris)
    tri, e, s, r = W._pack(tris, [eps_r] * T, [sigma] * T, [rgh] * T)
    w = W.Workload("wall", tri, e, s, r, np.array([[4.0, 1.0, 2.0]]), np.array([[6.0, 3.0, 1.0]]),
                   np.array([28e9]), geodesic_N=8, max_bounces=1)
    C = np.array([0.0, 2.0, 1.5])
    ps = SC.scattering_paths(w, 0.25, tl=(np.array([0]), C[None], np.array([0.25])))
    assert len(ps) == 1
    rec = SC.path_records(w, ps)[0]
    ri, rs = math.sqrt(16 + 1 + 0.25), math.sqrt(36 + 1 + 0.25)
    want = [(ri + rs) / C0, 165.96375653207352, math.degrees(math.asin(-0.5 / ri)),
            -170.53767779197437, math.degrees(math.asin(0.5 / rs))]
    assert np.allclose(rec, want, rtol=1e-12, atol=1e-10), (rec, want)


def test_link_stats_closed_forms():
    """Two paths of equal power P at delays t1, t2: PG = 10 log10(2 P),
    tau_rms = |t1 - t2| / 2; azimuths 170 and -170 degrees average to 180
    (the circular mean across the +-180 cut), elevations 10 and 30 to 20.
    One path: its own angles, tau_rms 0."""
    pg, tau, ang = O.link_stats([1e-9, 1e-9], [10e-9, 16e-9],
                                [[170.0, 10.0, 0.0, -5.0], [-170.0, 30.0, 90.0, 5.0]])
    assert abs(pg - 10 * math.log10(2e-9)) < 1e-12
    assert abs(tau - 3e-9) < 1e-20
    assert abs(abs(ang[0]) - 180.0) < 1e-9 and abs(ang[1] - 20.0) < 1e-12
    assert abs(ang[2] - 45.0) < 1e-9 and abs(ang[3]) < 1e-12
    pg, tau, ang = O.link_stats([2e-6], [5e-9], [[12.0, -3.0, 45.0, 7.0]])
    assert abs(pg - 10 * math.log10(2e-6)) < 1e-12 and tau == 0.0
    assert np.allclose(ang, [12.0, -3.0, 45.0, 7.0], atol=1e-12)
