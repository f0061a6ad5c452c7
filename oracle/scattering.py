"""First-order directive diffuse scattering (effective-roughness model): the
oracle's plain FP64 form.

Test infrastructure only (the product path never imports it).  The paper
lists scattering among its mechanisms, with a coefficient S in the field of
a path (eq. (2)) and a "directive scattering model based on ER theory"
(Sec. II-A-2, Fig. 3(b)), but gives no formula.  The reading taken here (R25)
is the single-lobe directive model of the effective-roughness theory of
Degli-Esposti et al. (IEEE Trans. AP 2007), first order (Tx -> surface tile
-> Rx), with the scattered power tied to the paper's own roughness model:

* tiles: triangle t of area A is cut by its barycentric grid into m^2 equal
  sub-triangles, m = max(1, ceil(sqrt(A / tile_area))); a tile is one
  sub-triangle, represented by its centroid and its area dS = A / m^2;
  order: by triangle, then the m(m+1)/2 upward sub-triangles by (i, j), then
  the m(m-1)/2 downward ones by (i, j);
* a path Tx -> C -> Rx through tile centroid C exists when Tx and Rx lie
  strictly on the same side of the triangle's plane and neither leg crosses
  a triangle outside the tile's face group (the image-method margins);
* field: the specularly reflected field of the incidence at C,
  E_r = Gamma_TE (E.s) s + Gamma_TM (E.p_in) p_out (the reflection tracker's
  bases), loses its component along the scattering direction k_s,
  E_s = E_r - (E_r . k_s) k_s; the scattered power is the share 1 - rho^2
  that the Kirchhoff roughness factor rho (eq. (8), at the incidence angle)
  removes from the specular reflection, spread over the half-space by the
  lobe ((1 + cos psi) / 2)^alpha around the specular direction (psi: angle
  between k_s and the specular direction), normalised by
  F_alpha(theta_i) = integral over the half-space of that lobe:
      a = (lambda / 4 pi) / (r_i r_s) sqrt(dS cos theta_i / F_alpha)
          sqrt(1 - rho^2) ((1 + cos psi) / 2)^(alpha / 2) (E_s . e_rx)
          e^{-j 2 pi f (r_i + r_s) / c}
  (times the atmosphere tables on r_i + r_s), so that over the half-space
  the tile scatters (1 - rho^2) |Gamma|^2 of the power incident on it.
  The tiles' fields are summed with their phases (a deterministic form of
  the model).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import oracle as O
from .diffraction import _blocked, _pol_vec

C0 = 299792458.0


# ---------------------------------------------------------------- lobe normalisation
def lobe_norm(alpha, cos_i, n_theta=96):
    """F_alpha(theta_i) = integral over the half-space z >= 0 of
    ((1 + s . r) / 2)^alpha dOmega(s), r the specular direction at angle
    theta_i from the normal: Gauss-Legendre in the polar angle, the
    trapezoidal rule (exact for this trigonometric polynomial) in azimuth."""
    xg, wg = np.polynomial.legendre.leggauss(n_theta)
    th = (xg + 1.0) * (math.pi / 4.0)
    wth = wg * (math.pi / 4.0)
    nphi = 2 * int(alpha) + 8
    ph = np.arange(nphi) * (2.0 * math.pi / nphi)
    si = math.sqrt(max(0.0, 1.0 - cos_i * cos_i))
    st, ct = np.sin(th)[:, None], np.cos(th)[:, None]
    cpsi = st * si * np.cos(ph)[None, :] + ct * cos_i
    f = ((1.0 + cpsi) / 2.0) ** alpha * st
    return float(np.sum(f.sum(axis=1) * (2.0 * math.pi / nphi) * wth))


# ---------------------------------------------------------------- tiles
def tiles(w, tile_area):
    """(tri [n], centroid [n][3], dS [n]) of every tile, in canonical order."""
    tri = np.asarray(w.tri, np.float64)
    out_t, out_c, out_a = [], [], []
    for t in range(len(tri)):
        v0, v1, v2 = tri[t]
        A = 0.5 * np.linalg.norm(np.cross(v1 - v0, v2 - v0))
        m = max(1, int(math.ceil(math.sqrt(A / tile_area))))
        e1, e2 = (v1 - v0) / m, (v2 - v0) / m

        def P(i, j):
            return v0 + i * e1 + j * e2

        for i in range(m):
            for j in range(m - i):
                out_t.append(t)
                out_c.append((P(i, j) + P(i + 1, j) + P(i, j + 1)) / 3.0)
                out_a.append(A / (m * m))
        for i in range(m - 1):
            for j in range(m - 1 - i):
                out_t.append(t)
                out_c.append((P(i + 1, j) + P(i, j + 1) + P(i + 1, j + 1)) / 3.0)
                out_a.append(A / (m * m))
    return np.array(out_t, np.int64), np.array(out_c).reshape(-1, 3), np.array(out_a)


# ---------------------------------------------------------------- paths and fields
@dataclass
class ScatPath:
    p: int
    q: int
    tile: int
    tri: int
    C: np.ndarray
    ri: float
    rs: float
    dS: float
    ambiguous: bool  # a point within 1e-9 of the plane, or a leg within 1e-5 (barycentric) of a blocker's boundary


def scattering_paths(w, tile_area, groups=None, tl=None):
    """Every valid first-order scattering path, ordered by (Rx, Tx, tile)."""
    tri = np.asarray(w.tri, np.float64)
    if groups is None:
        groups = O.scene_groups(w)[0] if len(tri) else np.zeros(0, np.int32)
    tt, cc, aa = tiles(w, tile_area) if tl is None else tl
    out = []
    for q, R in enumerate(np.asarray(w.rx, np.float64)):
        for p, Tx in enumerate(np.asarray(w.tx, np.float64)):
            for j in range(len(tt)):
                t = int(tt[j])
                v0, v1, v2 = tri[t]
                n = np.cross(v1 - v0, v2 - v0)
                n /= np.linalg.norm(n)
                C = cc[j]
                ht, hr = float(np.dot(Tx - C, n)), float(np.dot(R - C, n))
                if not (ht * hr > 0.0):
                    continue
                b1, d1 = _blocked(tri, groups, Tx, C, (int(groups[t]),))
                if b1:
                    continue
                b2, d2 = _blocked(tri, groups, C, R, (int(groups[t]),))
                if b2:
                    continue
                ri, rs = float(np.linalg.norm(C - Tx)), float(np.linalg.norm(R - C))
                amb = min(abs(ht), abs(hr)) < 1e-9 or min(d1, d2) < 1e-5
                out.append(ScatPath(p, q, j, t, C, ri, rs, float(aa[j]), amb))
    return out


def path_records(w, paths):
    """[n, 5] per scattering path: the delay (r_i + r_s) / c, then the
    departure direction Tx -> C and the arrival direction Rx -> C as
    (azimuth, elevation) in degrees (reading R17's senses)."""
    out = np.zeros((len(paths), 5))
    for i, d in enumerate(paths):
        Tx, R = np.asarray(w.tx[d.p], np.float64), np.asarray(w.rx[d.q], np.float64)
        out[i, 0] = (d.ri + d.rs) / C0
        out[i, 1:3] = O.az_el((d.C - Tx) / d.ri)
        out[i, 3:5] = O.az_el((d.C - R) / d.rs)
    return out


def scattering_field(w, paths, alpha, freq=None, atm_db=None, atm_deg=None, pol_tx=0, pol_rx=0,
                     with_scale=False):
    """a[path][f]: the received scattered field of every path (complex).
    with_scale: also |amp| (|e_s (s . e_rx)| + |e_p (p_out . e_rx)|), the
    field's two terms with the Fresnel coefficients at their bound 1: the
    rounding scale of a value in which the TE and TM terms nearly cancel, or
    whose R_TM is a near-cancelling quotient (incidence near the Brewster
    angle, where R_TM is far below its own rounding error in a short format)."""
    tri = np.asarray(w.tri, np.float64)
    freq = np.asarray(w.freq if freq is None else freq, np.float64)
    eps, sig, rough = (np.asarray(x, np.float64) for x in (w.eps_r, w.sigma, w.rough))
    out = np.zeros((len(paths), len(freq)), np.complex128)
    scale = np.zeros((len(paths), len(freq)))
    for i, d in enumerate(paths):
        Tx, R = np.asarray(w.tx[d.p], np.float64), np.asarray(w.rx[d.q], np.float64)
        v0, v1, v2 = tri[d.tri]
        n = np.cross(v1 - v0, v2 - v0)
        n /= np.linalg.norm(n)
        ki = (d.C - Tx) / d.ri
        ks = (R - d.C) / d.rs
        if np.dot(ki, n) > 0:
            n = -n                                   # the normal facing the incidence
        cs = -float(np.dot(ki, n))
        kr = ki - 2.0 * np.dot(ki, n) * n            # specular direction
        s = np.cross(ki, n)
        sn = np.linalg.norm(s)
        if sn < 1e-15:
            tmp = np.array([1.0, 0, 0]) if abs(ki[0]) < 0.9 else np.array([0, 1.0, 0])
            s = np.cross(ki, tmp)
            s /= np.linalg.norm(s)
        else:
            s /= sn
        p_in, p_out = np.cross(s, ki), np.cross(s, kr)
        E = _pol_vec(ki, pol_tx)
        es, ep = float(np.dot(E, s)), float(np.dot(E, p_in))
        erx = _pol_vec(ks, pol_rx)
        cpsi = float(np.dot(ks, kr))
        lobe = ((1.0 + cpsi) / 2.0) ** (alpha / 2.0)
        F = lobe_norm(alpha, cs)
        length = d.ri + d.rs
        e32, s32, r32 = (float(np.float32(x[d.tri])) for x in (eps, sig, rough))
        for fi, f in enumerate(freq):
            te, tm = O.fresnel(e32, s32, f, cs)
            rho = O.roughness(r32, f, cs)
            Er = te * es * s + tm * ep * p_out
            Es = Er - np.dot(Er, ks) * ks
            amp = (C0 / f) / (4.0 * math.pi) / (d.ri * d.rs) * math.sqrt(d.dS * cs / F)
            amp *= math.sqrt(max(0.0, 1.0 - rho * rho)) * lobe
            if atm_db is not None:
                amp *= 10.0 ** (-float(atm_db[fi]) * length / 20.0)
            cyc = f * length / C0
            phs = 2.0 * math.pi * (cyc - math.floor(cyc))
            if atm_deg is not None:
                phs += math.pi * float(atm_deg[fi]) * length / 180.0
            out[i, fi] = amp * np.dot(Es, erx) * np.exp(-1j * phs)
            scale[i, fi] = amp * (abs(es * np.dot(s, erx)) + abs(ep * np.dot(p_out, erx)))
    return (out, scale) if with_scale else out
