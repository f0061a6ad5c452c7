"""Pins of the oracle's per-path angles, reception-sphere radius and
ambiguity flags (CPU only).

* Angles (Sec. II-A-3, Table I quantities; reading R17: the departure angle
  is the direction of travel leaving the Tx, the arrival angle the direction
  from the Rx toward the last interaction; azimuth atan2(y, x), elevation
  asin(z)).  For reflectors that are coordinate planes the reflection points
  have closed forms (mirror the source, cut the line to the receiver), so
  the expected angles are computed here from that geometry alone.  A swapped
  arrival sense, an azimuth / elevation swap or a mirrored elevation fails.
* Reception radius (Sec. II-A-3: the sphere grows with the distance the ray
  has travelled; readings R2, R3: r = coeff * alpha * (L + t*) / sqrt(3),
  L the unfolded length before the segment, t* the closest approach).  A
  receiver placed at a known perpendicular offset from a known ray is
  captured at (1 - 1e-3) of that radius and missed at (1 + 1e-3), on a
  direct ray and on a reflected one (where dropping L would miss), and the
  1e-5 band of R21 marks captures at the boundary.
* Ambiguity flags (reading R21): a hit within 1e-5 (barycentric) of an edge
  or a vertex, a crossing of another triangle's edge band no farther than
  the hit, a tie within 1e-5 relative in t, and grazing incidence with
  |d.n| < 1e-5 each raise their own flag; an interior hit raises none, and
  values just outside each band raise none either.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_10006_amd import workloads as W

PHI = (1 + 5 ** 0.5) / 2


def _room_groups(w):
    """Face group of each wall of the axis-aligned room, by the coordinate
    its triangles share: {('x', 0.0): g, ('x', 10.0): g, ...}."""
    g, _, _ = O.scene_groups(w)
    out = {}
    for t in range(w.T):
        v = w.tri[t]
        for ax, name in enumerate("xyz"):
            if np.all(v[:, ax] == v[0, ax]):
                out[(name, float(v[0, ax]))] = int(g[t])
    return out


def _az_el(u):
    u = np.asarray(u, float) / np.linalg.norm(u)
    return math.degrees(math.atan2(u[1], u[0])), math.degrees(math.asin(u[2]))


def _mirror(p, axis, value):
    q = np.array(p, float)
    q[axis] = 2 * value - q[axis]
    return q


def _cut(a, b, axis, value):
    """Point of segment a -> b on the plane coordinate[axis] = value."""
    s = (value - a[axis]) / (b[axis] - a[axis])
    return a + s * (b - a)


def _image_points(tx, rx, walls):
    """Reflection points of the path tx -> walls[0] -> ... -> rx over
    coordinate planes (axis, value): mirror the source through the walls,
    then cut back from the receiver."""
    imgs = [np.asarray(tx, float)]
    for ax, val in walls:
        imgs.append(_mirror(imgs[-1], ax, val))
    X = [None] * (len(walls) + 2)
    X[0], X[-1] = np.asarray(tx, float), np.asarray(rx, float)
    for i in range(len(walls), 0, -1):
        ax, val = walls[i - 1]
        X[i] = _cut(imgs[i], X[i + 1], ax, val)
    return X


ROOM_CASES = {
    "los": [],
    "floor": [("z", 0.0)],
    "ceiling": [("z", 3.0)],
    "wall_x10": [("x", 10.0)],
    "wall_y0": [("y", 0.0)],
    "y8_then_x10": [("y", 8.0), ("x", 10.0)],
    "floor_x10_ceiling": [("z", 0.0), ("x", 10.0), ("z", 3.0)],
}


@pytest.mark.parametrize("case", sorted(ROOM_CASES))
def test_path_angles_room_closed_form(case):
    w = W.tiny_room()
    groups = _room_groups(w)
    walls = ROOM_CASES[case]
    k = len(walls)
    key = np.full((1, 3 + w.max_bounces), -1, np.int32)
    key[0, :3] = (0, 0, k)
    for i, (ax, val) in enumerate(walls):
        key[0, 3 + i] = groups[(ax, val)]
    rec = O.paths(w, key)[0]
    assert rec[0] == 1.0, f"{case}: the image path must be valid"
    X = _image_points(w.tx[0], w.rx[0], [("xyz".index(a), v) for a, v in walls])
    aod = _az_el(X[1] - X[0])
    aoa = _az_el(X[k] - X[k + 1])
    assert abs(rec[3] - aod[0]) < 1e-9 and abs(rec[4] - aod[1]) < 1e-9, (case, rec[3:5], aod)
    assert abs(rec[5] - aoa[0]) < 1e-9 and abs(rec[6] - aoa[1]) < 1e-9, (case, rec[5:7], aoa)
    # lengths along the legs equal the image distance
    assert abs(rec[1] - sum(np.linalg.norm(X[i + 1] - X[i]) for i in range(k + 1))) < 1e-12 * rec[1]


def test_path_angles_room_hand_values():
    """The same angles written out from the room's numbers: Tx (2, 2, 1.5),
    Rx (7, 5, 1.5), room 10 x 8 x 3 m."""
    w = W.tiny_room()
    groups = _room_groups(w)

    def rec_of(walls):
        key = np.full((1, 3 + w.max_bounces), -1, np.int32)
        key[0, :3] = (0, 0, len(walls))
        for i, wl in enumerate(walls):
            key[0, 3 + i] = groups[wl]
        return O.paths(w, key)[0]

    d = math.degrees
    los = rec_of([])
    # departure toward (5, 3, 0); arrival back toward the Tx, (-5, -3, 0)
    assert np.allclose(los[3:7], [d(math.atan2(3, 5)), 0.0, d(math.atan2(-3, -5)), 0.0], atol=1e-12)
    floor = rec_of([("z", 0.0)])
    # specular point (4.5, 3.5, 0): Tx -> (2.5, 1.5, -1.5), Rx -> (-2.5, -1.5, -1.5)
    el = -d(math.asin(1.5 / math.sqrt(2.5 ** 2 + 1.5 ** 2 + 1.5 ** 2)))
    assert np.allclose(floor[3:7], [d(math.atan2(1.5, 2.5)), el, d(math.atan2(-1.5, -2.5)), el], atol=1e-12)
    ceil = rec_of([("z", 3.0)])
    assert np.allclose(ceil[3:7], [d(math.atan2(1.5, 2.5)), -el, d(math.atan2(-1.5, -2.5)), -el], atol=1e-12)
    wall = rec_of([("x", 10.0)])
    # image of the Tx at (18, 2, 1.5): specular point (10, 2 + 24/11, 1.5)
    assert np.allclose(wall[3:7], [d(math.atan2(24 / 11, 8)), 0.0, d(math.atan2(24 / 11 - 3, 3)), 0.0], atol=1e-12)


def test_path_angles_oblique_plane():
    """One oblique reflection off the plane x = 0 (Sec. I image method)."""
    tx, rx = np.array([2.0, -1.3, 1.7]), np.array([3.5, 2.2, -0.9])
    w = W.one_plane(tx=tuple(tx), rx=tuple(rx), K=1, N=8)
    rec = O.paths(w, np.array([[0, 0, 1, 0]], np.int32))[0]
    assert rec[0] == 1.0
    img = tx * np.array([-1.0, 1.0, 1.0])
    X1 = img + (0 - img[0]) / (rx[0] - img[0]) * (rx - img)
    assert abs(X1[0]) < 1e-15
    aod, aoa = _az_el(X1 - tx), _az_el(X1 - rx)
    assert np.allclose(rec[3:7], [*aod, *aoa], atol=1e-9)
    # the departure points into the plane (negative x), the arrival looks back at it
    assert abs(rec[3]) > 90.0 and abs(rec[5]) > 90.0


# ------------------------------------------------------------------ reception radius
def _corner(i):
    """Icosahedron vertex i of the launch ordering (corners are rays 0..11 at
    any N): (0, +-1, +-phi), (+-1, +-phi, 0), (+-phi, 0, +-1), sign pairs in
    the order (-,-), (-,+), (+,-), (+,+), normalised."""
    sg = [(-1, -1), (-1, 1), (1, -1), (1, 1)]
    a, b = sg[i % 4]
    v = [(0.0, a, b * PHI), (a, b * PHI, 0.0), (a * PHI, 0.0, b)][i // 4]
    return np.array(v) / math.sqrt(1 + PHI * PHI)


def _free_space_at(tx, rx):
    return W.Workload("free", np.zeros((0, 3, 3)), np.zeros(0, np.float32), np.zeros(0, np.float32),
                      np.zeros(0, np.float32), np.array([tx], float), np.array([rx], float), np.array([28e9]),
                      geodesic_N=1, max_bounces=0)


@pytest.mark.parametrize("ray", [0, 5, 11])
def test_capture_radius_direct_ray(ray):
    """Ray `ray` of an N = 1 launch from the Tx, receiver at distance D along
    it and perpendicular offset delta: captured iff delta <= coeff alpha D /
    sqrt(3)."""
    tx = np.array([1.0, -2.0, 0.5])
    u = _corner(ray)
    e = np.cross(u, [0.3, 0.5, 0.8])
    e /= np.linalg.norm(e)
    alpha, coeff, D = 0.05, 1.7, 6.0
    r = coeff * alpha * D / math.sqrt(3.0)
    for f, captured, near in [(1 - 1e-3, True, False), (1 + 1e-3, False, False),
                              (1 - 1e-6, True, True), (1 + 1e-6, False, True)]:
        w = _free_space_at(tx, tx + D * u + f * r * e)
        tr = O.sbr(w, alpha=alpha, coeff=coeff)
        got = [(int(ry), int(k[2])) for ry, k in zip(tr.ev_ray, tr.ev_key)]
        assert got == ([(ray, 0)] if captured else []), (f, got)
        near_rays = [int(x) for x in tr.near_ray]
        if captured:
            # R21: a capture within 1e-5 of the sphere is marked ambiguous
            assert bool(tr.ev_amb[0] & 1) == near, (f, tr.ev_amb)
        else:
            # a miss inside the band is recorded as a near miss, farther out not at all
            assert near_rays == ([ray] if near else []), (f, near_rays)


def test_capture_radius_after_reflection():
    """Ray 9 (direction (-phi, 0, 1)) reflects off the plane x = 0; the
    receiver sits at distance D1 along the reflected ray with a perpendicular
    offset.  The radius uses the unfolded length t0 + D1 (t0 to the
    reflection point), which is about 1.7 times t* = D1 alone: a radius
    without the length before the segment would miss every case below."""
    tx = np.array([3.0, 10.0, 10.0])
    u = _corner(9)
    assert u[0] < 0 and abs(u[1]) < 1e-15 and u[2] > 0
    t0 = tx[0] / -u[0]
    X = tx + t0 * u
    d1 = u * np.array([-1.0, 1.0, 1.0])
    alpha, D1 = 0.05, 5.0
    r = alpha * (t0 + D1) / math.sqrt(3.0)
    assert alpha * D1 / math.sqrt(3.0) < 0.7 * r
    for f, captured in [(1 - 1e-3, True), (1 + 1e-3, False), (0.7, True)]:
        rx = X + D1 * d1 + f * r * np.array([0.0, 1.0, 0.0])
        w = W.one_plane(tx=tuple(tx), rx=tuple(rx), K=1, N=1)
        tr = O.sbr(w, alpha=alpha, coeff=1.0)
        got = sorted((int(ry), int(k[2]), int(k[3])) for ry, k in zip(tr.ev_ray, tr.ev_key))
        g, _, _ = O.scene_groups(w)
        assert got == ([(9, 1, int(g[0]))] if captured else []), (f, got)


# ------------------------------------------------------------------ ambiguity flags
def _frame(u):
    e1 = np.cross(u, [0.0, 1.0, 0.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(u, e1)
    return e1, e2


def _tri_around(P, bary, E1, E2):
    """Triangle (A, A + E1, A + E2) in which P has barycentric coordinates
    (1 - b1 - b2, b1, b2)."""
    b1, b2 = bary
    A = P - b1 * E1 - b2 * E2
    return np.array([A, A + E1, A + E2])


def _scene(tris, tx):
    tris = np.array(tris, float)
    T = len(tris)
    return W.Workload("flags", tris, np.full(T, 5.0, np.float32), np.full(T, 0.01, np.float32),
                      np.zeros(T, np.float32), np.array([tx], float), np.array([[50.0, 50.0, 50.0]]),
                      np.array([28e9]), geodesic_N=1, max_bounces=0)


RAY = 11  # direction (phi, 0, 1) / |.|


def _trace_one(tris):
    tx = np.zeros(3)
    w = _scene(tris, tx)
    tr = O.sbr(w, ray_ids=np.array([RAY]), alpha=1e-3, coeff=1.0)
    return int(tr.seq[0, 0]), float(tr.t[0, 0]), int(tr.amb[0, 0])


def _setup(dist=5.0):
    u = _corner(RAY)
    e1, e2 = _frame(u)
    return u, dist * u, 2.0 * e1, 2.0 * e2


def test_interior_hit_is_unambiguous():
    u, P, E1, E2 = _setup()
    hit, t, amb = _trace_one([_tri_around(P, (1 / 3, 1 / 3), E1, E2)])
    assert hit == 0 and abs(t - 5.0) < 1e-12 and amb == 0


@pytest.mark.parametrize("bary,flag", [((0.5 - 2.5e-7, 0.5 - 2.5e-7), 1),   # inside, 5e-7 from edge BC
                                       ((1e-7, 0.4), 1),                    # inside, 1e-7 from edge AC
                                       ((5e-8, 5e-8), 1),                   # next to vertex A
                                       ((0.5 - 5e-5, 0.5 - 5e-5), 0)])      # 1e-4 from the edge: clear
def test_edge_and_vertex_hits(bary, flag):
    u, P, E1, E2 = _setup()
    hit, t, amb = _trace_one([_tri_around(P, bary, E1, E2)])
    assert hit == 0 and abs(t - 5.0) < 1e-12
    assert amb == flag, amb


def test_near_edge_crossing_of_another_triangle():
    """The ray passes 5e-7 (barycentric) outside a nearer triangle and hits a
    farther one in its interior: the hit is flagged 2 (another triangle's edge
    band is crossed no farther than the hit).  Alone, the near miss leaves the
    ray without a hit, still flagged 2."""
    u, P, E1, E2 = _setup(3.0)
    near = _tri_around(P, (0.5 + 2.5e-7, 0.5 + 2.5e-7), E1, E2)  # barycentric 1 - b1 - b2 = -5e-7
    _, P8, _, _ = _setup(8.0)
    far = _tri_around(P8, (1 / 3, 1 / 3), E1, E2)
    hit, t, amb = _trace_one([near, far])
    assert hit == 1 and abs(t - 8.0) < 1e-12 and amb == 2, (hit, t, amb)
    hit, t, amb = _trace_one([near])
    assert hit == -1 and amb == 2
    clear = _tri_around(P, (0.5 + 5e-5, 0.5 + 5e-5), E1, E2)     # 1e-4 outside: no flag
    hit, t, amb = _trace_one([clear, far])
    assert hit == 1 and amb == 0


@pytest.mark.parametrize("rel,flag", [(0.0, 4), (4e-6, 4), (3e-5, 0)])
def test_tie_in_t(rel, flag):
    """Two triangles in different planes crossing the ray at t = 5 and
    t = 5 (1 + rel): a tie within 1e-5 relative is flagged 4 and the nearer
    (then the lower index) wins."""
    u, P, E1, E2 = _setup()
    a = _tri_around(P, (1 / 3, 1 / 3), E1, E2)
    # second triangle tilted 30 degrees about E2 through the point at 5 (1 + rel)
    Q = (5.0 * (1 + rel)) * u
    E1t = math.cos(math.radians(30)) * E1 + math.sin(math.radians(30)) * 2.0 * u
    b = _tri_around(Q, (1 / 3, 1 / 3), E1t, E2)
    hit, t, amb = _trace_one([a, b])
    assert hit == 0 and abs(t - 5.0) < 1e-12
    assert amb == flag, amb


@pytest.mark.parametrize("dn,flag", [(5e-6, 8), (2e-5, 0)])
def test_grazing_incidence(dn, flag):
    """A plane through the point at t = 5 whose normal makes |d.n| = dn with
    the ray: grazing (flag 8) below 1e-5."""
    u, P, E1, E2 = _setup()
    e1 = E1 / 2.0
    n = math.sqrt(1 - dn * dn) * e1 + dn * u
    along = u - (u @ n) * n
    along /= np.linalg.norm(along)
    tri = _tri_around(P, (1 / 3, 1 / 3), 4.0 * along, E2)
    assert abs(abs(np.cross(tri[1] - tri[0], tri[2] - tri[0]) @ u) /
               np.linalg.norm(np.cross(tri[1] - tri[0], tri[2] - tri[0])) - dn) < 1e-12
    hit, t, amb = _trace_one([tri])
    assert hit == 0 and abs(t - 5.0) < 1e-6
    assert amb == flag, amb


@pytest.mark.parametrize("gap,flag", [(1e-5, 1), (1e-4, 0)])
def test_sliver_edge_band_is_absolute(gap, flag):
    """On a sliver 1 cm wide the 1e-5 barycentric band is 1e-7 m, below what
    FP32 positions resolve; the edge band also holds points within 4e-6 of
    (distance from the scene centre + distance travelled) of the boundary,
    here about 2e-5 m: a hit 1e-5 m inside the long edge is flagged, one
    1e-4 m inside is not (barycentric 1e-3 and 1e-2, outside that band)."""
    u, P, E1, E2 = _setup()
    e1, e2 = E1 / 2.0, E2 / 2.0
    # long edge along e2 through P - gap e1; the sliver spans 1 cm across
    A = P - gap * e1 - 1.0 * e2
    tri = np.array([A, A + 2.0 * e2, A + 0.01 * e1 + 1.0 * e2])
    hit, t, amb = _trace_one([tri])
    assert hit == 0 and abs(t - 5.0) < 1e-12
    assert amb == flag, amb
