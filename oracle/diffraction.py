"""First-order edge diffraction: the oracle's plain FP64 form.

Test infrastructure only (the product path never imports it).  The paper
lists first-order diffraction among its mechanisms (Sec. II-A-2, Fig. B(b),
Table I) but gives no coefficient; the reading taken here (R24) is the
uniform theory of diffraction of Kouyoumjian and Pathak (Proc. IEEE 1974)
for a straight wedge, with the two reflection-type terms weighted by the
faces' reflection coefficients as proposed by Luebbers (IEEE Trans. AP 1984)
for lossy wedges:

* a wedge is a triangle edge shared by exactly two triangles of different
  face groups whose planes are not parallel; the solid occupies the smaller
  angular sector alpha < pi between the two faces, the field the exterior
  sector n pi = 2 pi - alpha (1 < n < 2); an edge that lies on a triangle of
  a third face group (both ends within 1e-9 (1 + max |coordinate|) of its
  plane, the edge's midpoint inside it with the 1e-9 barycentric margin) is
  not a wedge: it is where a solid rests on another surface;
* face 0 is the triangle of lower index, angles are measured from face 0
  towards face n through the exterior: phi' at the Tx, phi at the Rx, both
  strictly inside (0, n pi);
* the diffraction point Q on the edge makes equal angles beta0 with the edge
  for the incident and the diffracted ray (Keller's cone): unfolding the
  edge, Q divides the edge coordinates of Tx and Rx in the ratio of their
  distances from the edge line; Q must lie strictly inside the edge, and
  neither leg (Tx -> Q, Q -> Rx) may cross a triangle outside the two face
  groups of the wedge (same margins as the image-method paths);
* field: E^d = E^i(Q) D A(s) e^{-jks} with E^i(Q) = (lambda / 4 pi)
  e^{-jks'} / s' times the Tx polarisation, the dyadic
  D = -beta0' beta0 D_s - phi' phi D_h in edge-fixed unit vectors,
  A = sqrt(s' / (s (s + s'))), and
  D_{s,h} = -e^{-j pi/4} / (2 n sqrt(2 pi k) sin beta0)
            [T1 + T2 + R0 T3 + Rn T4],
  the T terms the four cot(.) F(k L a(.)) products of the transition
  function, L = s s' sin^2 beta0 / (s + s'); R0, Rn the Fresnel coefficient
  (TE for D_s, TM for D_h) times the Kirchhoff roughness factor of each
  face at the true incidence angle of the ray reflecting there
  (cos = sin beta0 |sin phi'| on face 0, sin beta0 |sin(n pi - phi)| on
  face n); a perfect conductor (R = -1 for TE, +1 for TM) gives the
  textbook D_s (minus) and D_h (plus).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.special import fresnel as _scipy_fresnel

from . import oracle as O

C0 = 299792458.0


# ---------------------------------------------------------------- transition function and coefficients
def transition(X):
    """Kouyoumjian-Pathak transition function
    F(X) = 2j sqrt(X) e^{jX} int_{sqrt X}^inf e^{-j t^2} dt  (X >= 0),
    the tail integral written with the Fresnel integrals C, S:
    int_u^inf e^{-j t^2} dt = sqrt(pi/2) [(1/2 - C(v)) - j (1/2 - S(v))], v = u sqrt(2/pi)."""
    X = np.asarray(X, np.float64)
    u = np.sqrt(X)
    v = u * math.sqrt(2.0 / math.pi)
    S, Cc = _scipy_fresnel(v)
    tail = math.sqrt(math.pi / 2.0) * ((0.5 - Cc) - 1j * (0.5 - S))
    return 2j * u * np.exp(1j * X) * tail


def _a(beta, n, sign):
    """a^{+-}(beta) = 2 cos^2((2 n pi N - beta) / 2), N the integer nearest to
    (beta +- pi) / (2 n pi), so that 2 pi n N - beta is nearest to +-pi."""
    N = np.round((beta + sign * math.pi) / (2.0 * math.pi * n))
    return 2.0 * np.cos((2.0 * n * math.pi * N - beta) / 2.0) ** 2


def _term(beta, n, kL, sign):
    """cot((pi + sign beta) / (2n)) F(k L a^{sign}(beta))."""
    return 1.0 / np.tan((math.pi + sign * beta) / (2.0 * n)) * transition(kL * _a(beta, n, sign))


def utd_coefficient(n, phi, phip, beta0, k, L, R0, Rn):
    """D = -e^{-j pi/4} / (2 n sqrt(2 pi k) sin beta0) [T1 + T2 + R0 T3 + Rn T4],
    T1 = cot((pi + (phi - phi')) / 2n) F(kL a+(phi - phi')),
    T2 = cot((pi - (phi - phi')) / 2n) F(kL a-(phi - phi')),
    T3 = cot((pi - (phi + phi')) / 2n) F(kL a-(phi + phi'))  (face 0),
    T4 = cot((pi + (phi + phi')) / 2n) F(kL a+(phi + phi'))  (face n)."""
    kL = k * L
    bm, bp = phi - phip, phi + phip
    T1 = _term(bm, n, kL, +1)
    T2 = _term(bm, n, kL, -1)
    T3 = _term(bp, n, kL, -1)
    T4 = _term(bp, n, kL, +1)
    pre = -np.exp(-1j * math.pi / 4.0) / (2.0 * n * math.sqrt(2.0 * math.pi * k) * math.sin(beta0))
    return pre * (T1 + T2 + R0 * T3 + Rn * T4)


def boundary_distance(n, phi, phip):
    """Smallest |pi +- beta - 2 pi n N| over the four terms: the angular
    distance of the Rx from a shadow or reflection boundary."""
    out = math.inf
    for beta in (phi - phip, phi + phip):
        for sign in (+1, -1):
            N = round((beta + sign * math.pi) / (2.0 * math.pi * n))
            out = min(out, abs(sign * math.pi + beta - 2.0 * math.pi * n * N))
    return out


# ---------------------------------------------------------------- wedges
@dataclass
class Wedge:
    a: np.ndarray        # edge start (lexicographically smaller endpoint)
    b: np.ndarray        # edge end
    e: np.ndarray        # unit edge direction a -> b
    t0: np.ndarray       # unit vector in face 0, perpendicular to the edge, into the face
    n0: np.ndarray       # unit normal of face 0 on the exterior side
    n: float             # exterior angle / pi
    tri0: int            # triangle of face 0 (lower index) and of face n
    trin: int
    g0: int              # face groups
    gn: int


def _unit(v):
    return v / np.linalg.norm(v)


def wedges(w, groups=None):
    """The scene's wedge edges in canonical order (by the lower sharing
    triangle, then its local edge index i = vertex i -> vertex (i+1) mod 3)."""
    tri = np.asarray(w.tri, np.float64)
    if groups is None:
        groups = O.scene_groups(w)[0] if len(tri) else np.zeros(0, np.int32)
    owners = {}
    for t in range(len(tri)):
        for i in range(3):
            p, q = tuple(tri[t, i]), tuple(tri[t, (i + 1) % 3])
            key = (p, q) if p < q else (q, p)
            owners.setdefault(key, []).append((t, i))
    out = []
    for key, own in owners.items():
        if len(own) != 2:
            continue
        (ta, ia), (tb, ib) = sorted(own)
        if groups[ta] == groups[tb]:
            continue
        a, b = np.array(key[0]), np.array(key[1])
        e = _unit(b - a)
        na = np.cross(tri[ta, 1] - tri[ta, 0], tri[ta, 2] - tri[ta, 0])
        nb = np.cross(tri[tb, 1] - tri[tb, 0], tri[tb, 2] - tri[tb, 0])
        if np.linalg.norm(np.cross(_unit(na), _unit(nb))) < 1e-9:
            continue
        ca = tri[ta, (ia + 2) % 3]
        cb = tri[tb, (ib + 2) % 3]
        t0 = _unit((ca - a) - np.dot(ca - a, e) * e)
        t1 = _unit((cb - a) - np.dot(cb - a, e) * e)
        n0 = np.cross(e, t0)
        if np.dot(n0, t1) > 0:
            n0 = -n0
        alpha = math.acos(max(-1.0, min(1.0, float(np.dot(t0, t1)))))
        if _covered(tri, groups, a, b, (groups[ta], groups[tb])):
            continue
        out.append(((ta, ia), Wedge(a, b, e, t0, n0, 2.0 - alpha / math.pi, ta, tb, int(groups[ta]),
                                    int(groups[tb]))))
    out.sort(key=lambda x: x[0])
    return [wd for _, wd in out]


def _covered(tri, groups, a, b, skip):
    """Whether the edge a-b lies on a triangle outside face groups `skip`."""
    keep = ~np.isin(groups, list(skip))
    T = tri[keep]
    if len(T) == 0:
        return False
    nrm = np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0])
    nrm = nrm / np.linalg.norm(nrm, axis=1)[:, None]
    c = np.einsum("ij,ij->i", nrm, T[:, 0])
    eps = 1e-9 * (1.0 + max(np.abs(a).max(), np.abs(b).max()))
    onp = (np.abs(nrm @ a - c) <= eps) & (np.abs(nrm @ b - c) <= eps)
    if not onp.any():
        return False
    m = 0.5 * (a + b)
    for t, n in zip(T[onp], nrm[onp]):
        # barycentric coordinates of m from the three edge functions
        w = [np.dot(n, np.cross(t[(i + 1) % 3] - t[i], m - t[i])) for i in range(3)]
        area = np.dot(n, np.cross(t[1] - t[0], t[2] - t[0]))
        if min(w) / area >= -1e-9:
            return True
    return False


def _angle(wd: Wedge, P):
    """(edge coordinate, distance from the edge line, angle from face 0 through
    the exterior in [0, 2 pi)) of point P."""
    r = P - wd.a
    z = float(np.dot(r, wd.e))
    v = r - z * wd.e
    rho = float(np.linalg.norm(v))
    phi = math.atan2(float(np.dot(v, wd.n0)), float(np.dot(v, wd.t0)))
    if phi < 0:
        phi += 2.0 * math.pi
    return z, rho, phi


# ---------------------------------------------------------------- occlusion
def _blocked(tri, groups, P, R, skip):
    """Any triangle outside the face groups `skip` crossing the open segment
    P -> R at s in (1e-9, 1 - 1e-9), inclusive barycentrics with a 1e-9
    margin (Moller-Trumbore in FP64), and the smallest distance in
    barycentric terms of a crossing to its triangle's boundary (for the
    ambiguity flag)."""
    keep = ~np.isin(groups, list(skip))
    T = tri[keep]
    if len(T) == 0:
        return False, math.inf
    D = R - P
    v0 = T[:, 0]
    e1 = T[:, 1] - v0
    e2 = T[:, 2] - v0
    pv = np.cross(D, e2)
    det = np.einsum("ij,ij->i", e1, pv)
    ok = det != 0.0
    inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
    tv = P - v0
    u = np.einsum("ij,ij->i", tv, pv) * inv
    qv = np.cross(tv, e1)
    v = (qv @ D) * inv
    s = np.einsum("ij,ij->i", e2, qv) * inv
    inside_seg = ok & (s > 1e-9) & (s < 1.0 - 1e-9)
    hit = inside_seg & (u >= -1e-9) & (u <= 1.0 + 1e-9) & (v >= -1e-9) & (u + v <= 1.0 + 1e-9)
    bary = np.minimum(np.minimum(u, v), 1.0 - u - v)
    near = inside_seg & (np.abs(bary) < 1e-5)
    dmin = float(np.min(np.abs(bary[near]))) if near.any() else math.inf
    return bool(hit.any()), dmin


# ---------------------------------------------------------------- paths and fields
@dataclass
class DiffPath:
    p: int
    q: int
    wedge: int
    Q: np.ndarray
    sp: float           # s', Tx -> Q
    s: float            # Q -> Rx
    beta0: float
    phip: float
    phi: float
    n: float
    ambiguous: bool     # within 1e-9 of a validity limit or 1e-5 (barycentric) of a blocker's boundary


def diffraction_paths(w, wds=None, groups=None):
    """Every valid first-order diffraction path, ordered by (Rx, Tx, wedge)."""
    tri = np.asarray(w.tri, np.float64)
    if groups is None:
        groups = O.scene_groups(w)[0] if len(tri) else np.zeros(0, np.int32)
    if wds is None:
        wds = wedges(w, groups)
    out = []
    for q, R in enumerate(np.asarray(w.rx, np.float64)):
        for p, Tx in enumerate(np.asarray(w.tx, np.float64)):
            for j, wd in enumerate(wds):
                lim = wd.n * math.pi
                zt, rt, ft = _angle(wd, Tx)
                zr, rr, fr = _angle(wd, R)
                if rt <= 0.0 or rr <= 0.0:
                    continue
                if not (0.0 < ft < lim and 0.0 < fr < lim):
                    continue
                length = float(np.linalg.norm(wd.b - wd.a))
                zq = zt + (zr - zt) * rt / (rt + rr)
                if not (0.0 < zq < length):
                    continue
                Q = wd.a + zq * wd.e
                b1, d1 = _blocked(tri, groups, Tx, Q, (wd.g0, wd.gn))
                if b1:
                    continue
                b2, d2 = _blocked(tri, groups, Q, R, (wd.g0, wd.gn))
                if b2:
                    continue
                sp = float(np.linalg.norm(Q - Tx))
                s = float(np.linalg.norm(R - Q))
                cb = float(np.dot((Q - Tx) / sp, wd.e))
                beta0 = math.acos(max(-1.0, min(1.0, cb)))
                amb = (min(ft, lim - ft, fr, lim - fr) < 1e-9 or min(zq, length - zq) < 1e-9 * length
                       or min(d1, d2) < 1e-5 or boundary_distance(wd.n, fr, ft) < 1e-9)
                out.append(DiffPath(p, q, j, Q, sp, s, beta0, ft, fr, wd.n, amb))
    return out


def path_records(w, paths):
    """[n, 5] per diffraction path: the delay (s' + s) / c, then the
    departure direction Tx -> Q and the arrival direction Rx -> Q as
    (azimuth, elevation) in degrees (reading R17's senses)."""
    out = np.zeros((len(paths), 5))
    for i, d in enumerate(paths):
        Tx, R = np.asarray(w.tx[d.p], np.float64), np.asarray(w.rx[d.q], np.float64)
        out[i, 0] = (d.sp + d.s) / C0
        out[i, 1:3] = O.az_el((d.Q - Tx) / d.sp)
        out[i, 3:5] = O.az_el((d.Q - R) / d.s)
    return out


def _pol_vec(u, pol):
    """theta-hat (pol 0) or phi-hat (pol 1) of direction u (the reflection
    oracle's antenna convention)."""
    st = math.hypot(u[0], u[1])
    if pol:
        ph = math.atan2(u[1], u[0])
        return np.array([-math.sin(ph), math.cos(ph), 0.0])
    cp, sp_ = (u[0] / st, u[1] / st) if st > 0 else (1.0, 0.0)
    return np.array([u[2] * cp, u[2] * sp_, -st])


def diffraction_field(w, paths, wds=None, freq=None, atm_db=None, atm_deg=None, pol_tx=0, pol_rx=0,
                      with_scale=False):
    """a[path][f]: the received diffracted field of every path (complex).
    with_scale: also the magnitude each value is a sum of,
    |amp| (|D_s e_b r_b| + |D_h e_p r_p|) (the rounding scale of a cross-polar
    value in which the two terms nearly cancel)."""
    if wds is None:
        wds = wedges(w)
    freq = np.asarray(w.freq if freq is None else freq, np.float64)
    eps, sig, rough = (np.asarray(x, np.float64) for x in (w.eps_r, w.sigma, w.rough))
    out = np.zeros((len(paths), len(freq)), np.complex128)
    scale = np.zeros((len(paths), len(freq)))
    for i, d in enumerate(paths):
        wd = wds[d.wedge]
        Tx, R = np.asarray(w.tx[d.p], np.float64), np.asarray(w.rx[d.q], np.float64)
        ih = (d.Q - Tx) / d.sp
        sh = (R - d.Q) / d.s
        php = -np.cross(wd.e, ih)
        php /= np.linalg.norm(php)
        bp = np.cross(php, ih)
        ph = np.cross(wd.e, sh)
        ph /= np.linalg.norm(ph)
        bh = np.cross(ph, sh)
        Ei = _pol_vec(ih, pol_tx)
        rx_pol = _pol_vec(sh, pol_rx)
        eb, ep = float(np.dot(Ei, bp)), float(np.dot(Ei, php))
        rb, rp = float(np.dot(bh, rx_pol)), float(np.dot(ph, rx_pol))
        sb = math.sin(d.beta0)
        c0 = sb * abs(math.sin(d.phip))
        cn = sb * abs(math.sin(d.n * math.pi - d.phi))
        L = d.s * d.sp * sb * sb / (d.s + d.sp)
        length = d.s + d.sp
        for fi, f in enumerate(freq):
            k = 2.0 * math.pi * f / C0
            lam = C0 / f
            r0te, r0tm = O.fresnel(float(np.float32(eps[wd.tri0])), float(np.float32(sig[wd.tri0])), f, c0)
            rnte, rntm = O.fresnel(float(np.float32(eps[wd.trin])), float(np.float32(sig[wd.trin])), f, cn)
            rho0 = O.roughness(float(np.float32(rough[wd.tri0])), f, c0)
            rhon = O.roughness(float(np.float32(rough[wd.trin])), f, cn)
            Ds = utd_coefficient(d.n, d.phi, d.phip, d.beta0, k, L, rho0 * r0te, rhon * rnte)
            Dh = utd_coefficient(d.n, d.phi, d.phip, d.beta0, k, L, rho0 * r0tm, rhon * rntm)
            pol = -Ds * eb * rb - Dh * ep * rp
            amp = lam / (4.0 * math.pi) / d.sp * math.sqrt(d.sp / (d.s * (d.s + d.sp)))
            if atm_db is not None:
                amp *= 10.0 ** (-float(atm_db[fi]) * length / 20.0)
            cyc = f * length / C0
            phs = 2.0 * math.pi * (cyc - math.floor(cyc))
            if atm_deg is not None:
                phs += math.pi * float(atm_deg[fi]) * length / 180.0
            out[i, fi] = amp * pol * np.exp(-1j * phs)
            scale[i, fi] = amp * (abs(Ds * eb * rb) + abs(Dh * ep * rp))
    return (out, scale) if with_scale else out


def channel_matrix(w, paths, a):
    """H_diff[f, q, p]: the diffracted fields summed per (Rx, Tx) pair."""
    H = np.zeros((a.shape[1] if a.ndim == 2 else len(w.freq), len(w.rx), len(w.tx)), np.complex128)
    for i, d in enumerate(paths):
        H[:, d.q, d.p] += a[i]
    return H
