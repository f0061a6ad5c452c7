"""Comparison of the HIP path against the CPU oracle (helpers for the GPU tests).

Agreement rules (readings R21 and R22: ambiguity flags and bounded excusals):
* hit sequences: identical up to the first bounce the oracle flags as
  ambiguous (within 1e-5 of a triangle edge, a near tie, grazing);
* path keys: equal sets, except keys whose every capture is ambiguous on the
  side that found them (hit ambiguity at a bounce <= k, or distance within
  1e-5 of the sphere radius / segment ends);
* path lengths and delays within 1e-9 relative (the exact FP64 image
  geometry on both sides), per-path departure and arrival angles within
  1e-4 degrees (the library stores them as FP32 degrees), per-path amplitudes
  within 1e-7 relative (floor 1e-6 of the largest amplitude, for cross-polar
  terms that vanish), and H within 1e-5 relative per entry with the floor
  max(|H|, 1e-6 max|H|) on the common key set;
* the excusals are bounded: at most 1e-3 of the compared rays may differ
  after an ambiguous bounce, at most 1 % of the keys (2 in small sets) may be
  excused, and the full product H may differ from the oracle's full H per
  entry by no more than the summed magnitudes of the excused paths of that
  entry (plus the H tolerance).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from oracle import oracle as O
from paper_2208_10006_amd import sbr as S

LEN_RTOL = 1e-9
ANG_TOL_DEG = 1e-4
MAX_EXCUSED_RAY_FRAC = 1e-3
MAX_EXCUSED_KEY_FRAC = 0.01
MIN_EXCUSED_KEYS = 2
AMP_RTOL = 1e-7
AMP_FLOOR = 1e-6
H_RTOL = 1e-5
H_FLOOR = 1e-6


def key_tuple(p, q, k, groups):
    return (int(p), int(q), int(k), *[int(g) for g in groups[:k]])


@dataclass
class GpuResult:
    res: S.Result
    keys: list
    hits: np.ndarray
    events: tuple
    a: np.ndarray
    info: dict
    trace_info: dict


def gpu_run(ctx, w, alpha=0.0, coeff=None, pol_tx=0, pol_rx=0, trace=None) -> GpuResult:
    """The HIP path on workload w; with `trace` (a trace of w made elsewhere,
    e.g. by a batched launch) only the receive and the channel run here."""
    if trace is None:
        res = S.run_workload(ctx, w, alpha=alpha, coeff=coeff, pol_tx=pol_tx, pol_rx=pol_rx)
    else:
        ps = S.sbr_receive(ctx, trace, w.rx, alpha if alpha else w.alpha,
                           w.radius_coeff if coeff is None else coeff)
        H = np.zeros((len(w.freq), len(w.rx), len(w.tx)), np.complex128)
        S.sbr_channel(ctx, ps, w.freq, w.atm_db_per_m, w.atm_deg_per_m, pol_tx, pol_rx, H_c128=H)
        res = S.Result(None, trace, ps, H, S.sbr_paths_get(ps))
    rec = res.records
    keys = [key_tuple(r["tx"], r["rx"], r["order"], r["groups"]) for r in rec]
    hits = S.sbr_trace_hits(res.trace)
    ev = S.sbr_paths_events(res.paths)
    a = S.sbr_path_field(ctx, res.paths, w.freq, w.atm_db_per_m, w.atm_deg_per_m, pol_tx, pol_rx)
    return GpuResult(res, keys, hits, ev, a, S.sbr_paths_info(res.paths), S.sbr_trace_info(res.trace))


@dataclass
class Report:
    hit_rays: int = 0
    hit_mismatch: int = 0
    hit_excused: int = 0
    hit_same_group: int = 0   # rays whose triangles differ only within face groups (ties of coplanar overlaps)
    keys_gpu: int = 0
    keys_oracle: int = 0
    common: int = 0
    gpu_only_excused: list = field(default_factory=list)
    oracle_only_excused: list = field(default_factory=list)
    gpu_only_bad: list = field(default_factory=list)
    oracle_only_bad: list = field(default_factory=list)
    max_len_rel: float = 0.0
    max_delay_rel: float = 0.0
    max_ang_deg: float = 0.0
    max_amp_rel: float = 0.0
    max_h_rel: float = 0.0
    h_normwise: float = 0.0
    full_h_excess: float = 0.0   # max over entries of (|dH_full| - excused bound) / den; <= H_RTOL passes
    full_h_normwise: float = 0.0


def compare_hits(gpu_hits, ora_seq, ora_amb, ray_ids=None, tri_group=None):
    """(rays, unexcused mismatches, excused rays, bad ray indices, same-group
    rays).  Hit triangles must agree before the first oracle-ambiguous
    bounce.  After it a ray is excused; with `tri_group` the excusal counts
    rays whose face-group sequences differ, and rays whose triangles differ
    only inside face groups (a tie between overlapping coplanar triangles of
    one group: the same reflector, the same key) are counted apart."""
    g = gpu_hits if ray_ids is None else gpu_hits[ray_ids]
    n, K1 = ora_seq.shape
    amb = ora_amb != 0
    first_amb = np.where(amb.any(axis=1), amb.argmax(axis=1), K1)
    cols = np.arange(K1)[None, :]
    considered = cols < first_amb[:, None]
    diff = (g != ora_seq) & considered
    bad = diff.any(axis=1)
    differs = (g != ora_seq).any(axis=1) & ~bad
    same_group = np.zeros(n, bool)
    if tri_group is not None and len(tri_group):
        as_group = lambda h: np.where(h >= 0, tri_group[np.maximum(h, 0)], h)  # noqa: E731
        same_group = differs & ~(as_group(g) != as_group(ora_seq)).any(axis=1)
    excused = differs & ~same_group
    return n, int(bad.sum()), int(excused.sum()), np.nonzero(bad)[0], int(same_group.sum())


def compare(w, gr: GpuResult, ora: O.FullResult, tri_group: np.ndarray, pol_tx=0, pol_rx=0) -> Report:
    rep = Report()
    K = w.max_bounces
    R = 10 * w.geodesic_N ** 2 + 2
    # ---------------- hit sequences
    tr = ora.trace
    rep.hit_rays, rep.hit_mismatch, rep.hit_excused, _, rep.hit_same_group = compare_hits(
        gr.hits, tr.seq, tr.amb, tr.ray_ids, tri_group)
    # ---------------- key sets
    vk = ora.keys[ora.valid]
    ora_keys = [key_tuple(k[0], k[1], k[2], k[3:]) for k in vk]
    rep.keys_gpu, rep.keys_oracle = len(gr.keys), len(ora_keys)
    gset, oset = set(gr.keys), set(ora_keys)
    common = gset & oset
    rep.common = len(common)
    # oracle-side ambiguity per key: every capture event ambiguous?
    ev_k = {}
    for kk, amb in zip(tr.ev_key, tr.ev_amb):
        t = key_tuple(kk[0], kk[1], kk[2], kk[3:])
        ev_k.setdefault(t, []).append(int(amb))
    for t in sorted(oset - gset):
        (rep.oracle_only_excused if all(a != 0 for a in ev_k.get(t, [1])) else rep.oracle_only_bad).append(t)
    # GPU-only keys: excused when each capturing ray is hit-ambiguous in the oracle
    # at a bounce <= k, or the oracle saw that capture as a near miss / ambiguous
    if gset - oset:
        ray, q, k = gr.events
        first_amb = {}
        amb = tr.amb != 0
        fa = np.where(amb.any(axis=1), amb.argmax(axis=1), K + 1)
        pos = {int(r): i for i, r in enumerate(tr.ray_ids)}
        near = set()
        for kk, r in zip(getattr(tr, "near_key", []), getattr(tr, "near_ray", [])):
            near.add((int(r), int(kk[1]), int(kk[2])))
        for kk, r, a in zip(tr.ev_key, tr.ev_ray, tr.ev_amb):
            if a & 1:
                near.add((int(r), int(kk[1]), int(kk[2])))
        gkey_rays = {}
        for r, qq, kk in zip(ray, q, k):
            groups = [int(tri_group[gr.hits[r, i]]) for i in range(kk)]
            t = key_tuple(r // R, qq, kk, groups)
            gkey_rays.setdefault(t, []).append((int(r), int(qq), int(kk)))
        for t in sorted(gset - oset):
            ok = True
            for (r, qq, kk) in gkey_rays.get(t, []):
                i = pos.get(r)
                if i is None:
                    ok = False
                    break
                if not (fa[i] <= kk or (r, qq, kk) in near):
                    ok = False
                    break
            (rep.gpu_only_excused if ok else rep.gpu_only_bad).append(t)
    # ---------------- lengths and amplitudes on the common keys
    gidx = {t: i for i, t in enumerate(gr.keys)}
    oidx = {t: i for i, t in enumerate(ora_keys)}
    rec_v = ora.rec[ora.valid]
    a_ora = ora.a if (pol_tx == 0 and pol_rx == 0) else O.field(w, vk, pol_tx=pol_tx, pol_rx=pol_rx)
    recs = gr.res.records
    # amplitudes that vanish (e.g. the cross-polar line of sight) are compared
    # against a floor of AMP_FLOOR times the largest amplitude
    amax = float(np.abs(a_ora).max()) if len(a_ora) else 0.0
    for t in common:
        gi, oi = gidx[t], oidx[t]
        lg, lo = recs["length_m"][gi], rec_v[oi, 1]
        rep.max_len_rel = max(rep.max_len_rel, abs(lg - lo) / lo)
        rep.max_delay_rel = max(rep.max_delay_rel, abs(recs["delay_s"][gi] - rec_v[oi, 2]) / rec_v[oi, 2])
        rep.max_ang_deg = max(rep.max_ang_deg, angle_error(
            [recs[f][gi] for f in ("aod_az", "aod_el", "aoa_az", "aoa_el")], rec_v[oi, 3:7]))
        den = np.maximum(np.abs(a_ora[oi]), max(AMP_FLOOR * amax, 1e-300))
        rep.max_amp_rel = max(rep.max_amp_rel, float(np.max(np.abs(gr.a[gi] - a_ora[oi]) / den)))
    # ---------------- H on the common key set
    Hg_full = gr.res.H
    Ho_full = O.channel_matrix(vk, a_ora, len(w.tx), len(w.rx))
    Hg, Ho = Hg_full.copy(), Ho_full.copy()
    excused_mag = np.zeros(Ho.shape)
    for t in gset - oset:
        Hg[:, t[1], t[0]] -= gr.a[gidx[t]]
        excused_mag[:, t[1], t[0]] += np.abs(gr.a[gidx[t]])
    for t in oset - gset:
        Ho[:, t[1], t[0]] -= a_ora[oidx[t]]
        excused_mag[:, t[1], t[0]] += np.abs(a_ora[oidx[t]])
    mx = np.abs(Ho).max() if Ho.size else 0.0
    if mx > 0:
        den = np.maximum(np.abs(Ho), H_FLOOR * mx)
        rep.max_h_rel = float(np.max(np.abs(Hg - Ho) / den))
        rep.h_normwise = float(np.linalg.norm(Hg - Ho) / np.linalg.norm(Ho))
    # ---------------- the full product H against the oracle's full H: every
    # entry within the magnitudes of its excused paths plus the tolerance
    mxf = np.abs(Ho_full).max() if Ho_full.size else 0.0
    if mxf > 0:
        den = np.maximum(np.abs(Ho_full), H_FLOOR * mxf)
        rep.full_h_excess = float(np.max((np.abs(Hg_full - Ho_full) - excused_mag) / den))
        rep.full_h_normwise = float(np.linalg.norm(Hg_full - Ho_full) / np.linalg.norm(Ho_full))
    return rep


def angle_error(gpu4, ora4) -> float:
    """Largest difference (degrees) between two (aod_az, aod_el, aoa_az,
    aoa_el) quadruples; azimuths compared modulo 360 and only where the
    direction is not within 0.1 degrees of a pole (there the azimuth is
    undefined)."""
    g = np.asarray(gpu4, np.float64)
    o = np.asarray(ora4, np.float64)
    err = max(abs(g[1] - o[1]), abs(g[3] - o[3]))
    for a, e in ((0, 1), (2, 3)):
        if abs(o[e]) < 89.9:
            d = (g[a] - o[a] + 180.0) % 360.0 - 180.0
            err = max(err, abs(d))
    return float(err)


def excused_key_limit(n_keys: int) -> int:
    return max(MIN_EXCUSED_KEYS, int(np.ceil(MAX_EXCUSED_KEY_FRAC * n_keys)))


def assert_report(rep: Report, allow_excused=True, max_excused_ray_frac=MAX_EXCUSED_RAY_FRAC):
    msg = repr(rep)
    assert rep.hit_mismatch == 0, msg
    assert rep.hit_excused <= max_excused_ray_frac * rep.hit_rays, msg
    assert not rep.gpu_only_bad and not rep.oracle_only_bad, msg
    n_exc = len(rep.gpu_only_excused) + len(rep.oracle_only_excused)
    if not allow_excused:
        assert n_exc == 0, msg
    assert n_exc <= excused_key_limit(max(rep.keys_gpu, rep.keys_oracle)), msg
    assert rep.max_len_rel <= LEN_RTOL, msg
    assert rep.max_delay_rel <= LEN_RTOL, msg
    assert rep.max_ang_deg <= ANG_TOL_DEG, msg
    assert rep.max_amp_rel <= AMP_RTOL, msg
    assert rep.max_h_rel <= H_RTOL, msg
    assert rep.full_h_excess <= H_RTOL, msg


def assert_segments(gpu_segments: int, ora_segments: int, rep: Report, K: int):
    """Segment counts agree up to the rays whose chains may differ after an
    ambiguous bounce (each can change its count by at most K)."""
    assert abs(gpu_segments - ora_segments) <= K * rep.hit_excused, (gpu_segments, ora_segments, rep.hit_excused)


def oracle_stats(keys, rec, a, Nr, Nt):
    """PG (dB), tau_rms (s), mean angles per (rx, tx) from oracle path data."""
    P = O.path_power(a) if len(a) else np.zeros(0)
    pg = np.full((Nr, Nt), -np.inf)
    tau = np.zeros((Nr, Nt))
    ang = np.zeros((Nr, Nt, 4))
    for q in range(Nr):
        for p in range(Nt):
            m = (keys[:, 0] == p) & (keys[:, 1] == q) if len(keys) else np.zeros(0, bool)
            if not m.any():
                continue
            pg[q, p] = O.path_gain_db(P[m])
            tau[q, p] = O.tau_rms(rec[m, 2], P[m])
            ang[q, p, 0:2] = O.mean_angles(P[m], rec[m, 3], rec[m, 4])
            ang[q, p, 2:4] = O.mean_angles(P[m], rec[m, 5], rec[m, 6])
    return pg, tau, ang


def excused_links(rep: Report) -> set:
    """(rx, tx) pairs touched by an excused key."""
    return {(t[1], t[0]) for t in rep.gpu_only_excused + rep.oracle_only_excused}


def check_stats(gpu_stats, ora, rep: Report, Nr: int, Nt: int):
    """Per-link path gain, RMS delay spread and mean angles of the GPU against
    the oracle's, on every (rx, tx) link whose key set is not excused; links
    without a path must have none on the GPU either.  Returns the number of
    links compared."""
    pg, tau, ang = gpu_stats
    vk, rec = ora.keys[ora.valid], ora.rec[ora.valid]
    opg, otau, oang = oracle_stats(vk, rec, ora.a, Nr, Nt)
    skip = excused_links(rep)
    n = 0
    for q in range(Nr):
        for p in range(Nt):
            if (q, p) in skip:
                continue
            if not np.isfinite(opg[q, p]):
                assert pg[q, p] == -np.inf, (q, p, pg[q, p])
                continue
            n += 1
            assert abs(pg[q, p] - opg[q, p]) < 1e-4, (q, p, pg[q, p], opg[q, p])
            assert abs(tau[q, p] - otau[q, p]) <= 1e-5 * otau[q, p] + 1e-14, (q, p, tau[q, p], otau[q, p])
            err = angle_error(ang[q, p], oang[q, p])
            assert err < 2e-3, (q, p, ang[q, p], oang[q, p])
    return n
