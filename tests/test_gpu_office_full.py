"""The headline workload at its full size, in the launch configuration that
bench.py times (its inputs, its autotuned launch parameters, its step):
the massive-MIMO office with 256 Tx elements x 998,562 rays, K = 4, 64 Rx
and 1,024 subcarriers.  The oracle cannot trace 255.6 M rays, so the
outputs are checked on samples it computes one by one (hit chains of
sampled rays, sampled paths with their lengths, delays, angles and fields)
and through properties that hold at any size (H as the sum of the per-path
fields, the statistics of every link from the path records, capacity and
per-port power from H)."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_10006_amd import workloads as W

pytestmark = pytest.mark.gpu

N_RAYS = 4096      # sampled rays
N_PATHS = 400      # sampled paths
AMP_RTOL = 1e-7    # per-path amplitude (the reflection parity bound)


def banner(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def full():
    import torch

    import bench
    from paper_2208_10006_amd import autotune as A
    from paper_2208_10006_amd import sbr as S
    banner("office full size: 256 x 998562 rays, K=4, 64 Rx, 1024 f (bench step, tuned launch)")
    w = W.massive_mimo_office()
    dev = torch.device("cuda", 0)
    d = bench.make_inputs(w, torch, dev)
    ctx = S.context_for_torch(0)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    sc0 = S.sbr_scene_build(ctx, d["tri"], d["eps"], d["sig"], d["rough"])
    A.autotune_trace(ctx, sc0, d["tx"], w.geodesic_N, w.max_bounces, w.T, arch=arch)
    tr0 = S.sbr_trace(ctx, sc0, d["tx"], w.geodesic_N, w.max_bounces)
    S.sbr_synchronize(ctx)
    A.autotune_receive(ctx, tr0, d["rx"], 0.0, w.radius_coeff, len(w.tx) * w.rays_per_element, w.max_bounces,
                       arch=arch)
    del tr0, sc0
    sc, tr, ps = bench.step(S, ctx, w, d)
    torch.cuda.synchronize()
    return S, ctx, w, d, sc, tr, ps


def test_sampled_hit_chains(full):
    """4,096 rays drawn over all 255.6 M: hit chains equal to the oracle's
    up to the first oracle-ambiguous bounce."""
    import torch

    from tests import parity as PT
    S, ctx, w, d, sc, tr, ps = full
    banner("office full: sampled hit chains")
    R = 10 * w.geodesic_N ** 2 + 2
    ids = np.sort(np.random.default_rng(11).choice(len(w.tx) * R, N_RAYS, replace=False)).astype(np.int64)
    hits = torch.empty((len(w.tx) * R, w.max_bounces + 1), dtype=torch.int32, device="cuda")
    S.sbr_trace_hits(tr, hits)
    g = hits[torch.as_tensor(ids, device="cuda")].cpu().numpy()
    del hits
    ora = O.sbr(w, ray_ids=ids)
    groups, _, _ = O.scene_groups(w)
    n, bad, excused, bad_ids, same = PT.compare_hits(g, ora.seq, ora.amb, None, groups)
    print("rays", n, "bad", bad, "excused", excused, "same group", same, flush=True)
    assert bad == 0, ids[bad_ids[:10]]
    assert excused <= PT.MAX_EXCUSED_RAY_FRAC * n + 1, excused
    assert (g[:, 0] >= 0).mean() > 0.99  # the hall is closed: nearly every ray hits


def _keys(recs, K):
    keys = np.full((len(recs), 3 + K), -1, np.int32)
    keys[:, 0], keys[:, 1], keys[:, 2] = recs["tx"], recs["rx"], recs["order"]
    keys[:, 3:] = recs["groups"][:, :K]
    return keys


def test_sampled_paths_and_fields(full):
    """400 paths drawn from the full run: each is a valid image-method path
    in the oracle, with its length, delay, angles and field at three
    subcarriers."""
    S, ctx, w, d, sc, tr, ps = full
    banner("office full: sampled paths")
    recs = S.sbr_paths_get(ps)
    assert len(recs) > 10000, len(recs)
    sel = np.sort(np.random.default_rng(12).choice(len(recs), N_PATHS, replace=False))
    keys = _keys(recs[sel], w.max_bounces)
    orec = O.paths(w, keys)
    valid = orec[:, 0] > 0.5
    print("paths", len(recs), "sampled", len(sel), "oracle-valid", int(valid.sum()), flush=True)
    assert valid.mean() >= 0.99, np.nonzero(~valid)[0][:10]
    r = recs[sel][valid]
    o = orec[valid]
    assert np.allclose(r["length_m"], o[:, 1], rtol=1e-9, atol=0)
    assert np.allclose(r["delay_s"], o[:, 2], rtol=1e-9, atol=0)
    from tests import parity as PT
    ang = max(PT.angle_error([r[f][i] for f in ("aod_az", "aod_el", "aoa_az", "aoa_el")], o[i, 3:7])
              for i in range(len(r)))
    assert ang < 1e-4, ang
    fs = np.array([0, len(w.freq) // 2, len(w.freq) - 1])
    atm = None if w.atm_db_per_m is None else np.asarray(w.atm_db_per_m, np.float32)[fs]
    a_g = S.sbr_path_field(ctx, ps, w.freq[fs], atm, None)[sel][valid]
    a_o = O.field(w, keys[valid], freq=w.freq[fs], atm_db=atm)
    den = np.maximum(np.abs(a_o), 1e-6 * np.abs(a_o).max())
    err = float(np.max(np.abs(a_g - a_o) / den))
    print("max amplitude error", err, flush=True)
    assert err <= AMP_RTOL, err


def test_h_is_the_sum_of_the_path_fields(full):
    """H of the timed step (complex64, every subcarrier) at three
    subcarriers against the FP64 sum of every path's field per link."""
    S, ctx, w, d, sc, tr, ps = full
    banner("office full: H = sum of path fields")
    fs = np.array([0, len(w.freq) // 2, len(w.freq) - 1])
    atm = None if w.atm_db_per_m is None else np.asarray(w.atm_db_per_m, np.float32)[fs]
    recs = S.sbr_paths_get(ps)
    a = S.sbr_path_field(ctx, ps, w.freq[fs], atm, None)
    Nr, Nt = len(w.rx), len(w.tx)
    ref = np.zeros((len(fs), Nr, Nt), np.complex128)
    np.add.at(ref, (slice(None), recs["rx"], recs["tx"]), a.T)
    H = d["H"].cpu().numpy()[fs]
    den = np.abs(ref) + 1e-6 * np.abs(ref).max()
    err = float(np.max(np.abs(H - ref) / den))
    print("max H error", err, flush=True)
    assert err <= 1e-5, err


def test_link_statistics_from_the_records(full):
    """Path gain, RMS delay spread and mean angles of all 16,384 links of the
    timed step against the oracle's per-link statistics of the path
    records (band power, delay, angles)."""
    S, ctx, w, d, sc, tr, ps = full
    banner("office full: link statistics")
    recs = S.sbr_paths_get(ps)
    pg, tau, ang = (d[k].cpu().numpy() for k in ("pg", "tau", "ang"))
    from tests import parity as PT
    order = np.lexsort((recs["tx"], recs["rx"]))
    r = recs[order]
    pair = r["rx"].astype(np.int64) * len(w.tx) + r["tx"]
    starts = np.searchsorted(pair, np.arange(len(w.rx) * len(w.tx) + 1))
    n = 0
    for q in range(len(w.rx)):
        for p in range(len(w.tx)):
            s0, s1 = starts[q * len(w.tx) + p], starts[q * len(w.tx) + p + 1]
            if s0 == s1:
                assert pg[q, p] == -np.inf
                continue
            x = r[s0:s1]
            A = np.stack([x["aod_az"], x["aod_el"], x["aoa_az"], x["aoa_el"]], axis=1).astype(np.float64)
            opg, otau, oang = O.link_stats(x["power"].astype(np.float64), x["delay_s"], A)
            n += 1
            assert abs(pg[q, p] - opg) < 1e-4, (q, p, pg[q, p], opg)
            assert abs(tau[q, p] - otau) <= 1e-5 * otau + 1e-14, (q, p, tau[q, p], otau)
            assert PT.angle_error(ang[q, p], oang) < 2e-3, (q, p, ang[q, p], oang)
    assert n >= 0.9 * len(w.rx) * len(w.tx), n


def test_capacity_and_port_power_from_h(full):
    """eq. (15)-(17) over all 1,024 subcarriers and 7 SNR values, and the
    per-port band power (eq. (14)), against the oracle's numpy forms on the
    timed step's H."""
    S, ctx, w, d, sc, tr, ps = full
    banner("office full: capacity and port power")
    H = d["H"].cpu().numpy().astype(np.complex128)
    snr = d["snr"].cpu().numpy()
    want = O.capacity(H, snr)
    got = np.asarray(d["capacity"].cpu().numpy() if hasattr(d["capacity"], "cpu") else d["capacity"])
    assert np.allclose(got, want, rtol=1e-9, atol=1e-9), (got, want)
    P = d["P"].cpu().numpy()
    assert np.allclose(P, O.port_power(H), rtol=1e-12, atol=0)
