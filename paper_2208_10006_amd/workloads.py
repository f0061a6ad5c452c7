"""Seeded synthetic workloads for the SBR channel simulator.

This module only *generates inputs*: triangle scenes with per-triangle
materials, transmit/receive point sets, frequency grids and synthetic
atmospheric tables.  It contains none of the method's arithmetic (no ray
launching, intersection, reception or field computation), so both the GPU
path and the CPU oracle may consume its output.

The paper's own office model, its material data and the ITU-R line tables
are not available; these generators stand in for them with the shapes and
sizes of the workloads the method is meant for (indoor room, THz urban
canyon, massive-MIMO near-field office, batched uneven scenes).  The scene
inputs follow the problem statement of Section II (triangle scenes with
relative permittivity, conductivity and roughness, eq. (6)-(8); point arrays
eq. (11)-(12); a frequency grid for eq. (3), (9), (10)).

Everything is FP64 for geometry and frequency, FP32 for material constants
and attenuation tables, matching the C-ABI in ``include/sbr.h``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

C0 = 299_792_458.0  # speed of light, m/s (used only to size UPA spacing)


@dataclass
class Workload:
    """One SBR problem instance (scene + arrays + launch + band)."""

    name: str
    tri: np.ndarray            # f64 [T,3,3] triangle vertices, metres
    eps_r: np.ndarray          # f32 [T] relative permittivity
    sigma: np.ndarray          # f32 [T] conductivity, S/m
    rough: np.ndarray          # f32 [T] surface-height std, m
    tx: np.ndarray             # f64 [Nt,3]
    rx: np.ndarray             # f64 [Nr,3]
    freq: np.ndarray           # f64 [Nf] Hz
    atm_db_per_m: Optional[np.ndarray] = None   # f32 [Nf] or None
    atm_deg_per_m: Optional[np.ndarray] = None  # f32 [Nf] or None
    geodesic_N: int = 64       # rays per element = 10 N^2 + 2
    max_bounces: int = 3
    radius_coeff: float = 1.0
    alpha: float = 0.0         # <= 0: mean geodesic edge angle
    meta: dict = field(default_factory=dict)

    @property
    def T(self) -> int:
        return int(self.tri.shape[0])

    @property
    def rays_per_element(self) -> int:
        return 10 * self.geodesic_N * self.geodesic_N + 2

    def subset_tx(self, idx) -> "Workload":
        w = Workload(**{k: getattr(self, k) for k in self.__dataclass_fields__})
        w.tx = np.ascontiguousarray(self.tx[idx])
        return w


# ----------------------------------------------------------------------------
# primitive geometry builders (triangle soup only)
# ----------------------------------------------------------------------------

def _quad(a, b, c, d):
    """Two triangles covering the planar quad a-b-c-d (in order)."""
    return [np.array([a, b, c]), np.array([a, c, d])]


def box_triangles(lo, hi, yaw_rad: float = 0.0, bottom: bool = True):
    """Closed axis-aligned (then yawed about its vertical axis) box: 12 triangles
    (10 without the bottom).  Order: bottom, top, -x', +x', -y', +y' faces."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    cx, cy = 0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1])
    hx, hy = 0.5 * (hi[0] - lo[0]), 0.5 * (hi[1] - lo[1])
    z0, z1 = lo[2], hi[2]
    c, s = np.cos(yaw_rad), np.sin(yaw_rad)

    def P(sx, sy, z):
        x = sx * hx
        y = sy * hy
        return np.array([cx + c * x - s * y, cy + s * x + c * y, z])

    v = {}
    for sx in (-1, 1):
        for sy in (-1, 1):
            for iz, z in enumerate((z0, z1)):
                v[(sx, sy, iz)] = P(sx, sy, z)
    tris = []
    if bottom:
        tris += _quad(v[(-1, -1, 0)], v[(1, -1, 0)], v[(1, 1, 0)], v[(-1, 1, 0)])
    tris += _quad(v[(-1, -1, 1)], v[(1, -1, 1)], v[(1, 1, 1)], v[(-1, 1, 1)])
    tris += _quad(v[(-1, -1, 0)], v[(-1, 1, 0)], v[(-1, 1, 1)], v[(-1, -1, 1)])
    tris += _quad(v[(1, -1, 0)], v[(1, 1, 0)], v[(1, 1, 1)], v[(1, -1, 1)])
    tris += _quad(v[(-1, -1, 0)], v[(1, -1, 0)], v[(1, -1, 1)], v[(-1, -1, 1)])
    tris += _quad(v[(-1, 1, 0)], v[(1, 1, 0)], v[(1, 1, 1)], v[(-1, 1, 1)])
    return tris


def _footprint_dist(px, py, cx, cy, hx, hy, yaw):
    """Distance from point (px,py) to a yawed rectangle footprint (0 inside)."""
    c, s = np.cos(yaw), np.sin(yaw)
    dx, dy = px - cx, py - cy
    lx = c * dx + s * dy
    ly = -s * dx + c * dy
    ex = np.maximum(np.abs(lx) - hx, 0.0)
    ey = np.maximum(np.abs(ly) - hy, 0.0)
    return np.hypot(ex, ey)


def upa(center, n: int, spacing: float, plane: str = "yz", cols: Optional[int] = None) -> np.ndarray:
    """Uniform planar array of n x cols points (cols = n by default); element
    (i, j) has index i*cols + j and sits at centre + (i-(n-1)/2) d u +
    (j-(cols-1)/2) d v (eq. (11)-(12) point sets)."""
    center = np.asarray(center, float)
    cols = n if cols is None else cols
    axes = {"yz": (np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0])),
            "xz": (np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.0, 1.0])),
            "xy": (np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]))}[plane]
    out = np.empty((n * cols, 3))
    for i in range(n):
        for j in range(cols):
            out[i * cols + j] = (center + (i - (n - 1) / 2) * spacing * axes[0]
                                 + (j - (cols - 1) / 2) * spacing * axes[1])
    return out


def upa_shape(n: int):
    """rows x cols of an n-element UPA: the most nearly square factorisation
    with rows <= cols (16 -> 4 x 4, 32 -> 4 x 8, 64 -> 8 x 8, 128 -> 8 x 16)."""
    rows = int(np.floor(np.sqrt(n)))
    while n % rows:
        rows -= 1
    return rows, n // rows


def _pack(tris, eps, sig, rough):
    T = len(tris)
    tri = np.zeros((T, 3, 3)) if T == 0 else np.ascontiguousarray(np.stack(tris), dtype=np.float64)
    return (tri, np.asarray(eps, np.float32).reshape(T), np.asarray(sig, np.float32).reshape(T),
            np.asarray(rough, np.float32).reshape(T))


# ----------------------------------------------------------------------------
# small analytic scenes (pins and unit cases)
# ----------------------------------------------------------------------------

def free_space(tx=(0.0, 0.0, 1.5), rx=(5.0, 3.0, 1.5), freq=28e9, N=16) -> Workload:
    """Empty scene (T = 0): a single line-of-sight path."""
    tri, e, s, r = _pack([], [], [], [])
    return Workload("free_space", tri, e, s, r, np.array([tx], float), np.array([rx], float),
                    np.atleast_1d(np.asarray(freq, float)), geodesic_N=N, max_bounces=2)


def vertical_plane(x0=0.0, y=(-50.0, 70.0), z=(-40.0, 60.0), eps_r=5.31, sigma=0.0326, rough=0.0):
    """Large plane x = x0, split along a diagonal that avoids the origin's normal."""
    a = (x0, y[0], z[0]); b = (x0, y[1], z[0]); c = (x0, y[1], z[1]); d = (x0, y[0], z[1])
    return _quad(a, b, c, d), eps_r, sigma, rough


def one_plane(tx=(2.0, 0.3, 0.2), rx=(5.0, 0.3, 0.2), freq=28e9, N=32, K=2,
              eps_r=5.31, sigma=0.0326, rough=0.0) -> Workload:
    tris, e, s, r = vertical_plane(eps_r=eps_r, sigma=sigma, rough=rough)
    T = len(tris)
    tri, e, s, r = _pack(tris, [e] * T, [s] * T, [r] * T)
    return Workload("one_plane", tri, e, s, r, np.array([tx], float), np.array([rx], float),
                    np.atleast_1d(np.asarray(freq, float)), geodesic_N=N, max_bounces=K)


def two_parallel_planes(width=6.0, tx=(1.5, 0.4, 0.3), rx=(4.0, 3.1, -0.2), freq=28e9,
                        N=32, K=3, eps_r=5.31, sigma=0.0326) -> Workload:
    """Planes x = 0 and x = width."""
    t1, _, _, _ = vertical_plane(0.0)
    t2, _, _, _ = vertical_plane(width, y=(-60.0, 55.0), z=(-45.0, 52.0))
    tris = t1 + t2
    T = len(tris)
    tri, e, s, r = _pack(tris, [eps_r] * T, [sigma] * T, [0.0] * T)
    return Workload("two_parallel_planes", tri, e, s, r, np.array([tx], float),
                    np.array([rx], float), np.atleast_1d(np.asarray(freq, float)),
                    geodesic_N=N, max_bounces=K)


def two_perpendicular_planes(tx=(2.0, 1.2, 0.3), rx=(1.1, 3.3, -0.4), freq=28e9, N=32, K=2,
                             eps_r=5.31, sigma=0.0326) -> Workload:
    """Half-planes x = 0 (y >= 0) and y = 0 (x >= 0) meeting along the z axis."""
    z = (-40.0, 50.0)
    a1 = _quad((0.0, 0.0, z[0]), (0.0, 80.0, z[0]), (0.0, 80.0, z[1]), (0.0, 0.0, z[1]))
    a2 = _quad((0.0, 0.0, z[0]), (90.0, 0.0, z[0]), (90.0, 0.0, z[1]), (0.0, 0.0, z[1]))
    tris = a1 + a2
    T = len(tris)
    tri, e, s, r = _pack(tris, [eps_r] * T, [sigma] * T, [0.0] * T)
    return Workload("two_perpendicular_planes", tri, e, s, r, np.array([tx], float),
                    np.array([rx], float), np.atleast_1d(np.asarray(freq, float)),
                    geodesic_N=N, max_bounces=K)


# ----------------------------------------------------------------------------
# the five configured workloads
# ----------------------------------------------------------------------------

def tiny_room(N: int = 64, K: int = 3, freq=28e9, tx=(2.0, 2.0, 1.5), rx=(7.0, 5.0, 1.5)) -> Workload:
    """Axis-aligned 10 x 8 x 3 m box, 12 triangles, eps_r 5.31, sigma 0.0326 S/m,
    smooth; Tx (2,2,1.5), Rx (7,5,1.5), 28 GHz, level-6 launch (N = 64), K = 3."""
    tris = box_triangles((0.0, 0.0, 0.0), (10.0, 8.0, 3.0))
    T = len(tris)
    tri, e, s, r = _pack(tris, [5.31] * T, [0.0326] * T, [0.0] * T)
    return Workload("tiny_room", tri, e, s, r, np.array([tx], float), np.array([rx], float),
                    np.atleast_1d(np.asarray(freq, float)), geodesic_N=N, max_bounces=K)


def _urban_geometry(rng, n_boxes=200, tx_xy=(0.0, 0.0), half=250.0):
    tris = [*_quad((-half, -half, 0.0), (half, -half, 0.0), (half, half, 0.0), (-half, half, 0.0))]
    g_eps = rng.uniform(3.0, 7.0)
    g_rough = rng.uniform(0.05e-3, 0.2e-3)
    eps = [g_eps] * 2
    rough = [g_rough] * 2
    boxes = []
    while len(boxes) < n_boxes:
        sx, sy = rng.uniform(10.0, 40.0, size=2)
        h = rng.uniform(10.0, 60.0)
        cx, cy = rng.uniform(-235.0, 235.0, size=2)
        yaw = rng.uniform(0.0, np.pi / 2)
        if _footprint_dist(tx_xy[0], tx_xy[1], cx, cy, sx / 2, sy / 2, yaw) < 15.0:
            continue
        e = rng.uniform(3.0, 7.0)
        ro = rng.uniform(0.05e-3, 0.2e-3)
        boxes.append((cx, cy, sx / 2, sy / 2, yaw, h))
        bt = box_triangles((cx - sx / 2, cy - sy / 2, 0.0), (cx + sx / 2, cy + sy / 2, h), yaw)
        tris += bt
        eps += [e] * len(bt)
        rough += [ro] * len(bt)
    return tris, eps, rough, boxes


def _outside_footprints(px, py, boxes, margin):
    """Boolean mask of points farther than `margin` from every yawed footprint."""
    px = np.asarray(px, float)[:, None]
    py = np.asarray(py, float)[:, None]
    b = np.asarray(boxes, float)
    if len(b) == 0:
        return np.ones(px.shape[0], bool)
    cx, cy, hx, hy, yaw = b[:, 0], b[:, 1], b[:, 2], b[:, 3], b[:, 4]
    d = _footprint_dist(px, py, cx[None, :], cy[None, :], hx[None, :], hy[None, :], yaw[None, :])
    return np.all(d > margin, axis=1)


def height_map(boxes, heights, n: int = 128, half: float = 250.0) -> np.ndarray:
    """Max building height per pixel on an n x n grid over [-half, half]^2
    (pixel centres), divided by 60 m.  [n][n] float32, row = y, column = x."""
    c = (np.arange(n) + 0.5) * (2 * half / n) - half
    gx, gy = np.meshgrid(c, c, indexing="xy")
    hm = np.zeros(n * n)
    px, py = gx.ravel(), gy.ravel()
    for (cx, cy, hx, hy, yaw), h in zip(boxes, heights):
        inside = _footprint_dist(px, py, cx, cy, hx, hy, yaw) <= 0.0
        hm[inside] = np.maximum(hm[inside], h)
    return (hm / 60.0).reshape(n, n).astype(np.float32)


def urban_surrogate_scene(seed: int, n_rx: int = 1000, random_rx: bool = False, N: int = 1024, K: int = 6):
    """Urban-canyon generator for the surrogate: carrier f_c ~ logU(28, 300) GHz,
    Tx at a random outdoor xy at 25 m, Rx either the grid points of the
    configured canyon (first n_rx outside footprints) or n_rx uniform random
    outdoor points at 1.5 m.  Returns (workload, height map, building heights)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fc = float(np.exp(rng.uniform(np.log(28e9), np.log(300e9))))
    while True:
        tx_xy = rng.uniform(-200.0, 200.0, size=2)
        tris, eps, rough, boxes = _urban_geometry(rng, tx_xy=tuple(tx_xy))
        if _outside_footprints([tx_xy[0]], [tx_xy[1]], [b[:5] for b in boxes], 15.0)[0]:
            break
    T = len(tris)
    tri, e, s, r = _pack(tris, eps, [0.0326] * T, rough)
    fb = [b[:5] for b in boxes]
    if random_rx:
        pts = np.zeros((0, 2))
        while len(pts) < n_rx:
            cand = rng.uniform(-236.25, 236.25, size=(4 * n_rx, 2))
            ok = _outside_footprints(cand[:, 0], cand[:, 1], fb, 1.0)
            far = np.hypot(cand[:, 0] - tx_xy[0], cand[:, 1] - tx_xy[1]) > 1.0
            pts = np.concatenate([pts, cand[ok & far]])
        pts = pts[:n_rx]
    else:
        g = (np.arange(64) - 31.5) * 7.5
        gx, gy = np.meshgrid(g, g, indexing="ij")
        allp = np.stack([gx.ravel(), gy.ravel()], axis=1)[rng.permutation(64 * 64)]
        ok = _outside_footprints(allp[:, 0], allp[:, 1], fb, 1.0)
        pts = allp[ok][:n_rx]
    rx = np.concatenate([pts, np.full((len(pts), 1), 1.5)], axis=1)
    atm = np.array([0.001 + 0.029 * np.exp(-((fc - 300e9) / 2.5e9) ** 2)], np.float32)
    w = Workload(f"urban_surrogate_{seed}", tri, e, s, r, np.array([[tx_xy[0], tx_xy[1], 25.0]]), rx,
                 np.array([fc]), atm_db_per_m=atm, geodesic_N=N, max_bounces=K)
    heights = [b[5] for b in boxes]
    return w, height_map(fb, heights), heights


def urban_canyon(seed: int = 2, N: int = 1024, K: int = 6, n_rx: int = 1000,
                 fc: float = 300e9, bw: float = 10e9, nf: int = 256,
                 tx=(0.0, 0.0, 25.0)) -> Workload:
    """500 x 500 m ground + 200 random yawed box buildings (2,402 triangles),
    roughness U(0.05, 0.2) mm, eps_r U(3, 7), sigma 0.0326 S/m; 300 GHz carrier,
    10 GHz on 256 subcarriers, synthetic atmosphere 0.001-0.03 dB/m; 1 Tx at 25 m,
    1,000 Rx at 1.5 m on a 7.5 m grid outside all footprints; N = 1024, K = 6."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tris, eps, rough, boxes = _urban_geometry(rng, tx_xy=tx[:2])
    T = len(tris)
    tri, e, s, r = _pack(tris, eps, [0.0326] * T, rough)
    # Rx: seeded permutation of a 64 x 64 grid, keep points outside footprints dilated by 1 m.
    g = (np.arange(64) - 31.5) * 7.5
    gx, gy = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([gx.ravel(), gy.ravel()], axis=1)
    perm = rng.permutation(len(pts))
    cand = pts[perm]
    ok = _outside_footprints(cand[:, 0], cand[:, 1], [b[:5] for b in boxes], 1.0)
    sel = cand[ok][:n_rx]
    rx = np.concatenate([sel, np.full((len(sel), 1), 1.5)], axis=1)
    k = np.arange(nf)
    df = bw / nf
    freq = fc + (k - nf // 2) * df
    atm = (0.001 + 0.029 * np.exp(-((freq - fc) / 2.5e9) ** 2)).astype(np.float32)
    w = Workload("urban_canyon", tri, e, s, r, np.array([tx], float), rx, freq,
                 atm_db_per_m=atm, atm_deg_per_m=None, geodesic_N=N, max_bounces=K)
    w.meta["boxes"] = boxes
    return w


OFFICE_TX = (1.0, 10.0, 2.5)
OFFICE_RX = (26.0, 7.0, 1.2)


def massive_mimo_office(seed: int = 3, N: int = 316, K: int = 4, nf: int = 1024,
                        fc: float = 100e9, bw: float = 2e9, n_tx_side: int = 16,
                        n_rx_side: int = 8) -> Workload:
    """30 x 20 x 3 m hall + 208 desks + 208 partitions (5,004 triangles), all
    eps_r 5.31, sigma 0.0326, smooth; 100 GHz, 1,024 subcarriers over 2 GHz;
    16 x 16 Tx UPA and 8 x 8 Rx UPA at lambda/2 in the y-z plane; per-element
    launch of N = 316 (998,562 rays), K = 4."""
    tri, e, s, r = office_scene(seed)
    k = np.arange(nf)
    freq = fc + (k - nf // 2) * (bw / nf)
    delta = C0 / fc / 2
    tx = upa(OFFICE_TX, n_tx_side, delta)
    rx = upa(OFFICE_RX, n_rx_side, delta)
    return Workload("massive_mimo_office", tri, e, s, r, tx, rx, freq, geodesic_N=N, max_bounces=K)


def mimo_office(n: int, seed: int = 3, N: int = 316, K: int = 4, nf: int = 1024, fc: float = 100e9,
                bw: float = 2e9) -> Workload:
    """n x n MIMO in the massive-MIMO office (Sec. IV-C, Fig. 6 and 7): an
    n-element Tx UPA and an n-element Rx UPA (upa_shape(n), lambda/2 spacing,
    y-z plane) at the office's Tx and Rx positions; same scene, band and launch
    as massive_mimo_office."""
    tri, e, s, r = office_scene(seed)
    k = np.arange(nf)
    freq = fc + (k - nf // 2) * (bw / nf)
    delta = C0 / fc / 2
    rows, cols = upa_shape(n)
    tx = upa(OFFICE_TX, rows, delta, cols=cols)
    rx = upa(OFFICE_RX, rows, delta, cols=cols)
    return Workload(f"mimo_office_{n}x{n}", tri, e, s, r, tx, rx, freq, geodesic_N=N, max_bounces=K,
                    meta={"n": n, "upa": (rows, cols)})


def office_scene(seed: int = 3):
    """The office hall: 30 x 20 x 3 m box + 208 desks + 208 partitions (yawed
    boxes kept 0.5 m clear of the Tx and Rx array centres), all eps_r 5.31,
    sigma 0.0326, smooth.  Returns packed (tri, eps_r, sigma, rough)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tris = box_triangles((0.0, 0.0, 0.0), (30.0, 20.0, 3.0))
    tx_c = np.array(OFFICE_TX)
    rx_c = np.array(OFFICE_RX)
    lift = 1e-3
    objs = 0
    while objs < 416:
        desk = objs % 2 == 0
        if desk:
            lx, ly, h = 1.6, 0.8, 0.75
        else:
            lx, ly, h = rng.uniform(1.2, 3.0), 0.05, 1.8
        yaw = rng.uniform(0.0, np.pi)
        rad = 0.5 * np.hypot(lx, ly)
        cx = rng.uniform(rad, 30.0 - rad)
        cy = rng.uniform(rad, 20.0 - rad)
        if min(_footprint_dist(a[0], a[1], cx, cy, lx / 2, ly / 2, yaw) for a in (tx_c, rx_c)) < 0.5:
            continue
        tris += box_triangles((cx - lx / 2, cy - ly / 2, lift), (cx + lx / 2, cy + ly / 2, lift + h), yaw)
        objs += 1
    T = len(tris)
    return _pack(tris, [5.31] * T, [0.0326] * T, [0.0] * T)


def random_box_scene(seed: int, n_boxes: int = 20, extent: float = 40.0, n_rx: int = 8,
                     N: int = 24, K: int = 3, freq=(28e9,)) -> Workload:
    """Small random urban-like scene for parity tests: ground + yawed boxes with
    per-box materials and roughness; Tx and Rx at random free positions."""
    rng = np.random.Generator(np.random.PCG64(seed))
    half = extent / 2
    tris = [*_quad((-half, -half, 0.0), (half, -half, 0.0), (half, half, 0.0), (-half, half, 0.0))]
    eps = [rng.uniform(3.0, 7.0)] * 2
    sig = [0.0326] * 2
    rough = [rng.uniform(0.0, 0.2e-3)] * 2
    boxes = []
    while len(boxes) < n_boxes:
        sx, sy = rng.uniform(2.0, 8.0, size=2)
        h = rng.uniform(2.0, 12.0)
        cx, cy = rng.uniform(-half + 5, half - 5, size=2)
        yaw = rng.uniform(0.0, np.pi / 2)
        if _footprint_dist(0.0, 0.0, cx, cy, sx / 2, sy / 2, yaw) < 3.0:
            continue
        boxes.append((cx, cy, sx / 2, sy / 2, yaw))
        bt = box_triangles((cx - sx / 2, cy - sy / 2, 0.0), (cx + sx / 2, cy + sy / 2, h), yaw)
        tris += bt
        eps += [rng.uniform(3.0, 7.0)] * len(bt)
        sig += [rng.uniform(0.01, 0.1)] * len(bt)
        rough += [rng.uniform(0.0, 0.2e-3)] * len(bt)
    rx = []
    while len(rx) < n_rx:
        px, py = rng.uniform(-half + 2, half - 2, size=2)
        if all(_footprint_dist(px, py, *b) > 1.0 for b in boxes) and np.hypot(px, py) > 2.0:
            rx.append((px, py, rng.uniform(1.0, 2.0)))
    T = len(tris)
    tri, e, s, r = _pack(tris, eps, sig, rough)
    return Workload(f"random_box_{seed}", tri, e, s, r, np.array([[0.0, 0.0, 6.0]]), np.array(rx),
                    np.asarray(freq, float), geodesic_N=N, max_bounces=K)


def batched_uneven(seed: int) -> Workload:
    """One scene of the batched uneven workload: family in {room, office, urban},
    triangle count lognormal (median 3,000, sigma_ln 1) clipped to [100, 50,000],
    rays 2^U(14,22), K ~ U{2..8}, carrier U(28, 300) GHz, 1-64 Rx."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fam = int(rng.integers(0, 3))
    T_target = int(np.clip(np.exp(np.log(3000.0) + rng.normal()), 100, 50_000))
    R = 2.0 ** rng.uniform(14, 22)
    N = max(1, int(round(np.sqrt((R - 2) / 10))))
    K = int(rng.integers(2, 9))
    f = float(rng.uniform(28e9, 300e9))
    nrx = int(rng.integers(1, 65))
    n_obj = max(1, (T_target - 12) // 12)
    if fam == 0:      # room with furniture boxes
        L = np.array([rng.uniform(6, 20), rng.uniform(5, 15), 3.0])
        tris = box_triangles((0, 0, 0), L)
    elif fam == 1:    # office hall
        L = np.array([rng.uniform(20, 60), rng.uniform(15, 40), 3.0])
        tris = box_triangles((0, 0, 0), L)
    else:             # urban block
        L = np.array([rng.uniform(150, 500), rng.uniform(150, 500), 60.0])
        tris = [*_quad((0, 0, 0), (L[0], 0, 0), (L[0], L[1], 0), (0, L[1], 0))]
    tx = np.array([L[0] * 0.5, L[1] * 0.5, min(L[2] * 0.8, 25.0)])
    hmax = L[2] * (0.9 if fam < 2 else 1.0)
    for _ in range(n_obj):
        sx = rng.uniform(0.02, 0.1) * L[0]
        sy = rng.uniform(0.02, 0.1) * L[1]
        h = rng.uniform(0.1, 0.6) * hmax
        cx = rng.uniform(sx, L[0] - sx)
        cy = rng.uniform(sy, L[1] - sy)
        yaw = rng.uniform(0, np.pi / 2)
        if _footprint_dist(tx[0], tx[1], cx, cy, sx / 2, sy / 2, yaw) < 1.0:
            continue
        tris += box_triangles((cx - sx / 2, cy - sy / 2, 1e-3), (cx + sx / 2, cy + sy / 2, 1e-3 + h), yaw)
    T = len(tris)
    rx = np.stack([rng.uniform(0.05, 0.95, nrx) * L[0], rng.uniform(0.05, 0.95, nrx) * L[1],
                   np.full(nrx, 1.5 if fam == 2 else 1.2) + 1e-3 * np.arange(nrx) / max(nrx, 1)], axis=1)
    tri, e, s, r = _pack(tris, rng.uniform(3, 7, T), [0.0326] * T, rng.uniform(0, 0.2e-3, T))
    return Workload(f"batched_{seed}", tri, e, s, r, tx[None, :], rx, np.array([f]),
                    geodesic_N=N, max_bounces=K, meta={"family": fam})


def _ensure_rx_free(w: Workload) -> Workload:
    return w
