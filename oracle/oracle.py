"""Python driver of the CPU FP64 oracle (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  It builds ``liboracle_sbr.so`` from
``sbr_oracle.c`` with gcc and drives it with ctypes; the reductions the paper
defines over the per-path results (coherent sum into H, eq. (2)/(13)-(14);
path power and RMS delay spread, eq. (5); path gain; mean angles; MIMO
capacity, eq. (15)-(17)) are written here in plain numpy, FP64.

It never imports the GPU package except the seeded input generators, which
hold no arithmetic of the method.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sbr_oracle.c")
LIB = os.path.join(HERE, "liboracle_sbr.so")
C0 = 299_792_458.0

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle (portable x86-64, IEEE double, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.orc_geodesic_count.restype = C.c_int64
        L.orc_geodesic_count.argtypes = [C.c_int]
        L.orc_geodesic.argtypes = [C.c_int, C.c_int64, C.c_int64, P]
        L.orc_edge_stats.argtypes = [C.c_int, P, P, P]
        L.orc_scene_groups.restype = C.c_int
        L.orc_scene_groups.argtypes = [P, C.c_int, P, P, P, P, P]
        L.orc_sbr.restype = C.c_int64
        L.orc_sbr.argtypes = [P, C.c_int, P, P, P, P, C.c_int, P, C.c_int, C.c_int, C.c_int,
                              C.c_double, C.c_double, P, C.c_int64, P, P, P,
                              C.c_int64, P, P, P, P, C.c_int]
        L.orc_paths.argtypes = [P, C.c_int, P, P, P, P, P, C.c_int, P, C.c_int64, P]
        L.orc_field.argtypes = [P, C.c_int, P, P, P, P, P, C.c_int, P, C.c_int64, P, C.c_int, P, P,
                                C.c_int, C.c_int, P]
        L.orc_fresnel.argtypes = [C.c_double] * 4 + [P] * 4
        L.orc_roughness.restype = C.c_double
        L.orc_roughness.argtypes = [C.c_double] * 3
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- launch
def geodesic(N: int, first: int = 0, count: int | None = None) -> np.ndarray:
    R = 10 * N * N + 2
    count = R - first if count is None else count
    out = np.empty((count, 3))
    assert lib().orc_geodesic(N, first, count, _p(out)) == 0
    return out


def edge_stats(N: int):
    m, lo, hi = (np.zeros(1) for _ in range(3))
    lib().orc_edge_stats(N, _p(m), _p(lo), _p(hi))
    return float(m[0]), float(lo[0]), float(hi[0])


def fresnel(eps_r, sigma, f, cos_i):
    o = [np.zeros(1) for _ in range(4)]
    lib().orc_fresnel(eps_r, sigma, f, cos_i, *[_p(x) for x in o])
    return complex(o[0][0], o[1][0]), complex(o[2][0], o[3][0])


def roughness(rough_std, f, cos_i):
    return float(lib().orc_roughness(rough_std, f, cos_i))


def scene_groups(w):
    T = w.T
    g = np.zeros(T, np.int32)
    p = np.zeros(T, np.int32)
    tri = np.ascontiguousarray(w.tri, np.float64)
    n = lib().orc_scene_groups(_p(tri), T, _p(np.ascontiguousarray(w.eps_r, np.float32)),
                               _p(np.ascontiguousarray(w.sigma, np.float32)),
                               _p(np.ascontiguousarray(w.rough, np.float32)), _p(g), _p(p))
    return g, p, n


# ---------------------------------------------------------------- trace + receive
@dataclass
class TraceResult:
    ray_ids: np.ndarray   # int64 [n]
    seq: np.ndarray       # int32 [n, K+1] hit triangle per segment, -1 miss, -2 not traced
    t: np.ndarray         # f64  [n, K+1]
    amb: np.ndarray       # u8   [n, K+1] ambiguity flags per bounce
    ev_key: np.ndarray    # int32 [E, 3+K] (p, q, k, g_1..g_K; -1 pad)
    ev_ray: np.ndarray    # int64 [E]
    ev_amb: np.ndarray    # u8 [E]
    ev_ratio: np.ndarray  # f64 [E] distance / radius

    @property
    def segments(self) -> int:
        return int((self.seq != -2).sum())


def _arrays(w):
    return (np.ascontiguousarray(w.tri, np.float64), np.ascontiguousarray(w.eps_r, np.float32),
            np.ascontiguousarray(w.sigma, np.float32), np.ascontiguousarray(w.rough, np.float32),
            np.ascontiguousarray(w.tx, np.float64), np.ascontiguousarray(w.rx, np.float64))


def sbr(w, ray_ids=None, alpha: float | None = None, coeff: float | None = None,
        nthreads: int = 0) -> TraceResult:
    """Trace the listed global ray ids (p * R + r; all rays when None) and test
    every segment against every receiver."""
    tri, e, s, r, tx, rx = _arrays(w)
    K, N = w.max_bounces, w.geodesic_N
    R = 10 * N * N + 2
    if ray_ids is None:
        ray_ids = np.arange(len(tx) * R, dtype=np.int64)
    ray_ids = np.ascontiguousarray(ray_ids, np.int64)
    n = len(ray_ids)
    alpha = w.alpha if alpha is None else alpha
    coeff = w.radius_coeff if coeff is None else coeff
    seq = np.empty((n, K + 1), np.int32)
    tv = np.empty((n, K + 1))
    amb = np.empty((n, K + 1), np.uint8)
    cap = max(1024, 4 * n // max(1, 1))
    cap = min(cap, 1 << 22)
    while True:
        ek = np.empty((cap, 3 + K), np.int32)
        er = np.empty(cap, np.int64)
        ea = np.empty(cap, np.uint8)
        eq = np.empty(cap)
        tot = lib().orc_sbr(_p(tri), w.T, _p(e), _p(s), _p(r), _p(tx), len(tx), _p(rx), len(rx), N, K,
                            alpha, coeff, _p(ray_ids), n, _p(seq), _p(tv), _p(amb),
                            cap, _p(ek), _p(er), _p(ea), _p(eq), nthreads)
        assert tot >= 0, "oracle rejected arguments"
        if tot <= cap:
            break
        cap = int(tot)
    ea, eq, ek, er = ea[:tot], eq[:tot], ek[:tot], er[:tot]
    cap_ = (ea & 4) == 0
    res = TraceResult(ray_ids, seq, tv, amb, ek[cap_], er[cap_], ea[cap_], eq[cap_])
    res.near_key, res.near_ray = ek[~cap_], er[~cap_]
    return res


def unique_keys(ev_key: np.ndarray) -> np.ndarray:
    """Distinct path keys in lexicographic order (p, q, k, g_1..g_K)."""
    if len(ev_key) == 0:
        return ev_key
    return np.unique(ev_key, axis=0)


# ---------------------------------------------------------------- paths + field
def paths(w, keys: np.ndarray) -> np.ndarray:
    """[n, 8]: valid, length, delay, aod_az, aod_el, aoa_az, aoa_el, k."""
    tri, e, s, r, tx, rx = _arrays(w)
    keys = np.ascontiguousarray(keys, np.int32)
    rec = np.zeros((len(keys), 8))
    lib().orc_paths(_p(tri), w.T, _p(e), _p(s), _p(r), _p(tx), _p(rx), w.max_bounces, _p(keys),
                    len(keys), _p(rec))
    return rec


def field(w, keys: np.ndarray, freq=None, atm_db=None, atm_deg=None, pol_tx: int = 0,
          pol_rx: int = 0) -> np.ndarray:
    """Complex amplitude a_n(f) of each key, [n, Nf] complex128."""
    tri, e, s, r, tx, rx = _arrays(w)
    keys = np.ascontiguousarray(keys, np.int32)
    freq = np.ascontiguousarray(w.freq if freq is None else freq, np.float64)
    atm_db = w.atm_db_per_m if atm_db is None else atm_db
    atm_deg = w.atm_deg_per_m if atm_deg is None else atm_deg
    ad = None if atm_db is None else np.ascontiguousarray(atm_db, np.float32)
    ag = None if atm_deg is None else np.ascontiguousarray(atm_deg, np.float32)
    out = np.zeros((len(keys), len(freq), 2))
    lib().orc_field(_p(tri), w.T, _p(e), _p(s), _p(r), _p(tx), _p(rx), w.max_bounces, _p(keys),
                    len(keys), _p(freq), len(freq), _p(ad), _p(ag), int(pol_tx), int(pol_rx), _p(out))
    return out[..., 0] + 1j * out[..., 1]


# ---------------------------------------------------------------- reductions
def channel_matrix(keys: np.ndarray, a: np.ndarray, Nt: int, Nr: int) -> np.ndarray:
    """H[f, q, p] = sum of a_n(f) over paths n of (p, q) (eq. (2), (13)-(14))."""
    Nf = a.shape[1] if a.ndim == 2 else 0
    H = np.zeros((Nf, Nr, Nt), np.complex128)
    for n in range(len(keys)):
        H[:, keys[n, 1], keys[n, 0]] += a[n]
    return H


def path_power(a: np.ndarray) -> np.ndarray:
    """P_n: squared amplitude of each path, averaged over the band."""
    return np.mean(np.abs(a) ** 2, axis=1)


def tau_rms(tau: np.ndarray, P: np.ndarray) -> float:
    """eq. (5)."""
    if len(tau) == 0 or P.sum() == 0:
        return 0.0
    m1 = np.sum(P * tau) / np.sum(P)
    m2 = np.sum(P * tau ** 2) / np.sum(P)
    return float(np.sqrt(max(m2 - m1 * m1, 0.0)))


def path_gain_db(P: np.ndarray) -> float:
    s = float(np.sum(P))
    return 10.0 * np.log10(s) if s > 0 else -np.inf


def mean_angles(P, az_deg, el_deg):
    """Power-weighted circular mean azimuth, arithmetic mean elevation (degrees)."""
    if len(P) == 0 or P.sum() == 0:
        return 0.0, 0.0
    az = np.degrees(np.angle(np.sum(P * np.exp(1j * np.radians(az_deg)))))
    el = float(np.sum(P * el_deg) / np.sum(P))
    return float(az), el


def az_el(u):
    """Azimuth atan2(u_y, u_x) and elevation asin(u_z) of a unit vector, in
    degrees (the angles of reading R17)."""
    return (float(np.degrees(np.arctan2(u[1], u[0]))),
            float(np.degrees(np.arcsin(min(1.0, max(-1.0, float(u[2])))))))


def link_stats(P, tau, ang):
    """One link's path gain (dB, R18), RMS delay spread (eq. (5)) and mean
    departure and arrival angles from the band power, delay and
    [aod_az, aod_el, aoa_az, aoa_el] (degrees) of each of its paths, whatever
    mechanism made them."""
    P, tau, ang = np.asarray(P, float), np.asarray(tau, float), np.asarray(ang, float).reshape(-1, 4)
    return (path_gain_db(P), tau_rms(tau, P),
            np.array([*mean_angles(P, ang[:, 0], ang[:, 1]), *mean_angles(P, ang[:, 2], ang[:, 3])]))


def capacity(H: np.ndarray, snr_db, normalize: bool = True) -> np.ndarray:
    """eq. (15)-(17): band-averaged log2 det(I + SNR/Nt W), W = Hn Hn^H
    (Nt >= Nr) or Hn^H Hn, with Frobenius normalisation Hn = H sqrt(Nt Nr / Q)."""
    Nf, Nr, Nt = H.shape
    Hn = H.astype(np.complex128)
    if normalize:
        Q = np.mean(np.sum(np.abs(Hn) ** 2, axis=(1, 2)))
        Hn = Hn * np.sqrt(Nt * Nr / Q)
    out = []
    for snr in np.atleast_1d(snr_db):
        lin = 10.0 ** (snr / 10.0)
        acc = 0.0
        for f in range(Nf):
            A = Hn[f]
            W = A @ A.conj().T if Nt >= Nr else A.conj().T @ A
            M = np.eye(W.shape[0]) + (lin / Nt) * W
            L = np.linalg.cholesky(M)
            acc += 2.0 * np.sum(np.log2(np.real(np.diag(L))))
        out.append(acc / Nf)
    return np.array(out)


def port_power(H: np.ndarray) -> np.ndarray:
    """eq. (14): h_qp = sqrt(P_qp) e^{i theta_qp}, the paths of Tx port p and Rx
    port q combined with their phases in H; P[q][p] is the band mean of
    |H_f[q][p]|^2 (the received power per antenna port of Sec. IV-C, Fig. 7)."""
    H = np.asarray(H, np.complex128)
    return np.mean(H.real ** 2 + H.imag ** 2, axis=0)


@dataclass
class FullResult:
    trace: TraceResult
    keys: np.ndarray      # unique keys (all, lexicographic)
    rec: np.ndarray       # [n, 8]
    valid: np.ndarray     # bool [n]
    a: np.ndarray         # [n_valid, Nf] complex
    H: np.ndarray         # [Nf, Nr, Nt]


def run(w, ray_ids=None, alpha=None, coeff=None) -> FullResult:
    """Full SBR: trace + receive + unique keys + exact paths + field + H."""
    tr = sbr(w, ray_ids, alpha, coeff)
    keys = unique_keys(tr.ev_key)
    rec = paths(w, keys) if len(keys) else np.zeros((0, 8))
    valid = rec[:, 0] > 0.5 if len(keys) else np.zeros(0, bool)
    vk = keys[valid] if len(keys) else keys
    a = field(w, vk) if len(vk) else np.zeros((0, len(w.freq)), np.complex128)
    H = channel_matrix(vk, a, len(w.tx), len(w.rx))
    return FullResult(tr, keys, rec, valid, a, H)
