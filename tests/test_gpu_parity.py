"""GPU parity: the HIP path (through the C-ABI) against the CPU FP64 oracle.

Each case prints its name, seed and sizes before touching the GPU so a
failing run names its case.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_2208_10006_amd import workloads as W


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


def exhaustive(N):
    m, lo, hi = O.edge_stats(N)
    return 1.05 * hi / m


# ------------------------------------------------------------------ launch
@pytest.mark.parametrize("N", [1, 2, 3, 7, 64])
def test_geodesic_full(S, ctx, N):
    banner("geodesic full", N)
    g = S.sbr_geodesic(ctx, N)
    o = O.geodesic(N)
    assert np.max(np.abs(g - o)) <= 4e-16


@pytest.mark.parametrize("N", [316, 1024])
def test_geodesic_sampled(S, ctx, N):
    banner("geodesic sampled", N)
    R = 10 * N * N + 2
    rng = np.random.default_rng(N)
    for first in [0, 12, 12 + 30 * (N - 1) - 5, R - 4000] + list(rng.integers(0, R - 2000, 4)):
        g = S.sbr_geodesic(ctx, N, int(first), 2000)
        o = O.geodesic(N, int(first), 2000)
        assert np.max(np.abs(g - o)) <= 4e-16, first


@pytest.mark.parametrize("N", [1, 4, 64, 316])
def test_alpha(S, ctx, N):
    banner("alpha", N)
    g = S.sbr_geodesic_alpha(ctx, N)
    o = O.edge_stats(N)
    for a, b in zip(g, o):
        assert abs(a - b) <= 1e-13 * b


# ------------------------------------------------------------------ scene
def _tricky_planes():
    """Coplanar triangles with mixed winding on planes whose largest normal
    components tie (45-degree walls, a (1,1,1) roof), offsets near hash-cell
    borders, and one material change inside a plane."""
    rng = np.random.default_rng(12)
    tris, eps = [], []
    for c in (5.0, 5.0 + 1e-12, 7.25, 1e-3 * 3):  # x + y = c walls (second one coplanar within tolerance)
        n = np.array([1.0, 1.0, 0.0]) / np.sqrt(2)
        u = np.array([1.0, -1.0, 0.0]) / np.sqrt(2)
        o = n * c / np.sqrt(2) * np.sqrt(2)
        for k in range(3):
            a = o + u * rng.uniform(-5, 5) + np.array([0, 0, rng.uniform(0, 3)])
            b = o + u * rng.uniform(-5, 5) + np.array([0, 0, rng.uniform(0, 3)])
            d = o + u * rng.uniform(-5, 5) + np.array([0, 0, rng.uniform(0, 3)])
            tris.append([a, b, d] if k % 2 else [a, d, b])
            eps.append(5.0 if k < 2 else 6.0)
    n3 = np.ones(3) / np.sqrt(3)
    e1 = np.array([1.0, -1.0, 0.0]) / np.sqrt(2)
    e2 = np.cross(n3, e1)
    for k in range(4):
        a, b, d = (n3 * 4.0 + e1 * rng.uniform(-3, 3) + e2 * rng.uniform(-3, 3) for _ in range(3))
        tris.append([a, b, d] if k % 2 else [d, b, a])
        eps.append(4.0)
    T = len(tris)
    return W.Workload("tricky", np.array(tris), np.array(eps, np.float32), np.full(T, 0.01, np.float32),
                      np.zeros(T, np.float32), np.zeros((1, 3)), np.ones((1, 3)), np.array([28e9]))


@pytest.mark.parametrize("which", ["tiny_room", "random", "urban", "office", "tricky"])
def test_scene_groups(S, ctx, which):
    banner("scene groups", which)
    w = {"tiny_room": lambda: W.tiny_room(), "random": lambda: W.random_box_scene(5, n_boxes=12),
         "urban": lambda: W.urban_canyon(), "office": lambda: W.massive_mimo_office(),
         "tricky": _tricky_planes}[which]()
    sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    g, p = S.sbr_scene_groups(sc, w.T)
    og, op, ng = O.scene_groups(w)
    assert np.array_equal(g, og) and np.array_equal(p, op)
    info = S.sbr_scene_info(sc)
    assert info["groups"] == ng and 1 <= info["bvh_depth"] <= 64


# ------------------------------------------------------------------ full parity cases
def _full_case(S, ctx, w, coeff=None, pol=(0, 0), exact_keys=False, max_excused_ray_frac=None):
    from tests import parity as PT
    g, _, _ = O.scene_groups(w)
    gr = PT.gpu_run(ctx, w, coeff=coeff, pol_tx=pol[0], pol_rx=pol[1])
    ora = O.run(w, coeff=coeff)
    rep = PT.compare(w, gr, ora, g, pol_tx=pol[0], pol_rx=pol[1])
    print(rep)
    assert rep.common > 0, "nothing compared"
    PT.assert_report(rep, allow_excused=not exact_keys,
                     max_excused_ray_frac=PT.MAX_EXCUSED_RAY_FRAC if max_excused_ray_frac is None
                     else max_excused_ray_frac)
    PT.assert_segments(gr.trace_info["segments"], ora.trace.segments, rep, w.max_bounces)
    return gr, ora, rep


def test_tiny_room_full(S, ctx):
    banner("tiny room (10x8x3 m, 12 tri, N=64, K=3, 28 GHz)")
    w = W.tiny_room()
    gr, ora, rep = _full_case(S, ctx, w)
    assert gr.trace_info["segments"] == 163848
    # derived outputs: PG, RMS delay spread, mean angles
    from tests import parity as PT
    pg, tau, ang = S.sbr_stats(gr.res.paths)
    vk, rec = ora.keys[ora.valid], ora.rec[ora.valid]
    opg, otau, oang = PT.oracle_stats(vk, rec, ora.a, 1, 1)
    assert abs(pg[0, 0] - opg[0, 0]) < 1e-4
    assert abs(tau[0, 0] - otau[0, 0]) <= 1e-5 * otau[0, 0]
    assert np.max(np.abs(ang - oang)) < 2e-3
    # per-path records: delay, angles, power
    recs = gr.res.records
    assert np.all(np.diff(recs["delay_s"]) >= 0)
    assert np.allclose(recs["power"], np.mean(np.abs(gr.a) ** 2, axis=1), rtol=1e-6)


def test_tiny_room_exhaustive_lattice(S, ctx):
    banner("tiny room exhaustive sphere")
    w = W.tiny_room()
    gr, ora, rep = _full_case(S, ctx, w, coeff=exhaustive(64), exact_keys=True)
    assert len(gr.keys) == 63
    assert list(np.bincount([k[2] for k in gr.keys])) == [1, 6, 18, 38]


@pytest.mark.parametrize("scene", ["free_space", "one_plane", "two_parallel_planes", "two_perpendicular_planes",
                                   "diagonal"])
def test_plane_scenes(S, ctx, scene):
    banner("plane scene", scene)
    if scene == "diagonal":  # specular point exactly on the edge shared by the wall's two triangles
        w = W.one_plane(tx=(2.0, 10.0, 10.0), rx=(5.0, 10.0, 10.0), K=1, N=24)
    else:
        w = getattr(W, scene)()
    _full_case(S, ctx, w, coeff=exhaustive(w.geodesic_N), exact_keys=True)


@pytest.mark.parametrize("n_tri", [1, 2])
def test_one_and_two_triangle_scenes(S, ctx, n_tri):
    """The smallest trees: a single leaf (one triangle) and one node over two
    leaves, built from device-prepared inputs; the specular point of the wall
    lies in its first triangle."""
    import dataclasses
    banner("triangles", n_tri)
    w0 = W.one_plane(K=1, N=24)
    w = dataclasses.replace(w0, tri=w0.tri[:n_tri].copy(), eps_r=w0.eps_r[:n_tri].copy(),
                            sigma=w0.sigma[:n_tri].copy(), rough=w0.rough[:n_tri].copy())
    assert w.T == n_tri
    _full_case(S, ctx, w, coeff=exhaustive(w.geodesic_N), exact_keys=True)


@pytest.mark.parametrize("pol", [(0, 1), (1, 0), (1, 1)])
def test_polarisations(S, ctx, pol):
    banner("polarisation", pol)
    w = W.random_box_scene(3, n_boxes=8, n_rx=3, N=20, K=2, freq=(28e9, 60e9))
    _full_case(S, ctx, w, pol=pol)


@pytest.mark.parametrize("seed,N,K,nrx", [(1, 24, 3, 6), (2, 40, 3, 10), (4, 32, 4, 5), (7, 17, 5, 3)])
def test_random_scenes(S, ctx, seed, N, K, nrx):
    banner("random scene", seed, N, K, nrx)
    w = W.random_box_scene(seed, n_boxes=20, n_rx=nrx, N=N, K=K, freq=(28e9, 140e9, 300e9))
    w.atm_db_per_m = np.array([0.0001, 0.002, 0.02], np.float32)
    w.atm_deg_per_m = np.array([0.5, -1.0, 2.0], np.float32)
    _full_case(S, ctx, w)


@pytest.mark.parametrize("which", ["random", "urban"])
def test_linear_bvh_scenes(S, ctx, which):
    """The Morton-ordered LBVH with its oversized-triangle list (the builder
    of scenes above 65,536 triangles), forced on small scenes through the
    bvh_ploc_max tuning key, against the oracle."""
    banner("linear BVH", which)
    if which == "random":
        w = W.random_box_scene(5, n_boxes=20, n_rx=6, N=24, K=3, freq=(28e9, 140e9))
    else:
        w = W.urban_canyon(N=20, K=3, n_rx=40, nf=8)
    old = S.sbr_context_get_tuning(ctx, "bvh_ploc_max")
    try:
        S.sbr_context_set_tuning(ctx, "bvh_ploc_max", 0)
        sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
        if which == "urban":  # the ground plane's two triangles go to the list
            assert S.sbr_scene_info(sc)["bvh_depth"] >= 1
        del sc
        _full_case(S, ctx, w)
    finally:
        S.sbr_context_set_tuning(ctx, "bvh_ploc_max", old)


def test_duplicated_triangles(S, ctx):
    """Every triangle of the room three times: identical boxes, merged boxes
    of zero added area and tied pair keys in the BVH clustering, coincident
    candidates in the closest-hit search."""
    banner("tiny room, every triangle three times")
    w = W.tiny_room(N=32, K=3)
    k = 3
    w = W.Workload("tiny_room_x3", np.concatenate([w.tri] * k), np.concatenate([w.eps_r] * k),
                   np.concatenate([w.sigma] * k), np.concatenate([w.rough] * k), w.tx, w.rx, w.freq,
                   atm_db_per_m=w.atm_db_per_m, atm_deg_per_m=w.atm_deg_per_m, geodesic_N=w.geodesic_N,
                   max_bounces=w.max_bounces)
    sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    g, p = S.sbr_scene_groups(sc, w.T)
    og, op, ng = O.scene_groups(w)
    assert np.array_equal(g, og) and np.array_equal(p, op)
    del sc
    # every hit ties with its two copies (R21 flag 4), so either side may name
    # any copy of a triangle: the face groups hit must agree
    gr, ora, rep = _full_case(S, ctx, w)
    assert rep.hit_same_group > 0


def test_profile_only_times_one_class(S, ctx):
    banner("profile only bounce")
    w = W.random_box_scene(8, n_boxes=10, n_rx=2, N=16, K=3)
    sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    try:
        S.sbr_profile_only(ctx, "bounce")
        S.sbr_profile_enable(ctx, True)
        tr = S.sbr_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces)
        ps = S.sbr_receive(ctx, tr, w.rx)
        S.sbr_synchronize(ctx)
        ms, n = S.sbr_profile_query(ctx, "bounce")
        assert n == w.max_bounces + 1 and ms > 0.0
        assert S.sbr_profile_query(ctx, "replay_capture") == (0.0, 0)
        assert S.sbr_profile_query(ctx, "host:rx_tree") == (0.0, 0)
        S.sbr_profile_only(ctx, None)
        S.sbr_profile_enable(ctx, True)
        ps = S.sbr_receive(ctx, tr, w.rx)
        S.sbr_synchronize(ctx)
        assert S.sbr_profile_query(ctx, "replay_capture")[1] == 1
        del ps, tr
    finally:
        S.sbr_profile_enable(ctx, False)
        S.sbr_profile_only(ctx, None)


@pytest.mark.slow
def test_urban_reduced_full(S, ctx):
    """Urban canyon geometry (2,402 triangles, 1,000 Rx, 256 subcarriers with
    the synthetic atmosphere) at a reduced launch density, full oracle."""
    banner("urban canyon N=48 K=6")
    w = W.urban_canyon(N=48)
    _full_case(S, ctx, w)


@pytest.mark.slow
def test_office_subset_full(S, ctx):
    """Massive-MIMO office (5,004 triangles, 8x8 Rx UPA, 100 GHz) with two Tx
    elements at a reduced density (N = 80) and 16 subcarriers, full oracle; path gain,
    RMS delay spread and mean angles on every one of the 128 links.  Two
    elements trace in element-minor ray order (the order of every array)."""
    from tests import parity as PT
    banner("office 2 tx N=80 K=4")
    # at N = 80 the sphere (about 0.15 m at the array) is small enough for
    # paths to pass the partitions around the Rx array: every link has one
    w = W.massive_mimo_office(N=80, nf=16).subset_tx([0, 255])
    gr, ora, rep = _full_case(S, ctx, w)
    assert rep.common >= 100, rep.common
    n = PT.check_stats(S.sbr_stats(gr.res.paths), ora, rep, len(w.rx), len(w.tx))
    assert n >= 100, n


def test_large_receiver_set_against_oracle(S, ctx):
    """3,000 receivers, above the 2,048 whose tree the device builds (so the
    host-prepared receiver tree), and about 19,000 capture events, above the
    12,288 keys of the one-workgroup sort (so the multi-pass radix sort),
    against the oracle; statistics on every link.  The replay with 1,024
    threads per block (its LDS stacks then need the block size cut) gives the
    same paths and H."""
    from tests import parity as PT
    banner("random scene 71, 3000 Rx, N=40, K=3")
    w = W.random_box_scene(71, n_boxes=20, n_rx=3000, N=40, K=3, freq=(28e9, 60e9))
    gr, ora, rep = _full_case(S, ctx, w)
    assert len(w.rx) > 2048 and gr.info["events"] > 12288, gr.info
    n = PT.check_stats(S.sbr_stats(gr.res.paths), ora, rep, len(w.rx), len(w.tx))
    assert n >= 2000, n
    old = S.sbr_context_get_tuning(ctx, "replay_block")
    try:
        S.sbr_context_set_tuning(ctx, "replay_block", 1024)
        ps = S.sbr_receive(ctx, gr.res.trace, w.rx, w.alpha, w.radius_coeff)
        H = np.zeros_like(gr.res.H)
        S.sbr_channel(ctx, ps, w.freq, w.atm_db_per_m, w.atm_deg_per_m, H_c128=H)
    finally:
        S.sbr_context_set_tuning(ctx, "replay_block", old)
    assert S.sbr_paths_info(ps)["paths"] == gr.info["paths"]
    np.testing.assert_allclose(H, gr.res.H, rtol=1e-12, atol=1e-14 * np.abs(gr.res.H).max())


def test_event_capacity_retry_is_exact(S, ctx):
    """A receive whose capture events overflow the first event buffer grows it
    and replays again: the same events, paths and H, bit for bit."""
    banner("capture-event retry")
    w = W.random_box_scene(72, n_boxes=12, n_rx=40, N=40, K=3, freq=(28e9, 60e9))
    ref = S.run_workload(ctx, w)
    old = S.sbr_context_get_tuning(ctx, "receive_event_capacity")
    try:
        S.sbr_context_set_tuning(ctx, "receive_event_capacity", 64)
        got = S.run_workload(ctx, w)
    finally:
        S.sbr_context_set_tuning(ctx, "receive_event_capacity", old)
    assert S.sbr_paths_info(got.paths)["events"] > 64
    assert S.sbr_paths_info(got.paths) == S.sbr_paths_info(ref.paths)
    assert got.H.tobytes() == ref.H.tobytes()
    assert got.records.tobytes() == ref.records.tobytes()


def test_batched_scenes_against_oracle(S, ctx):
    """Every problem of one batched launch (uneven scenes, one of them a
    four-element array in element-minor order) against the oracle."""
    from tests import parity as PT
    banner("batched trace against the oracle")
    arr = W.random_box_scene(83, n_boxes=10, n_rx=4, N=20, K=3, freq=(28e9,))
    arr.tx = W.upa((0.0, 0.0, 6.0), 2, 0.5)
    ws = [W.random_box_scene(81, n_boxes=15, n_rx=6, N=24, K=3, freq=(28e9, 140e9)),
          W.tiny_room(N=24, K=2), arr,
          W.random_box_scene(82, n_boxes=6, n_rx=3, N=17, K=5)]
    scenes = [S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough) for w in ws]
    trs = S.sbr_trace_batch(ctx, scenes, [w.tx for w in ws], [w.geodesic_N for w in ws],
                            [w.max_bounces for w in ws])
    for w, tr in zip(ws, trs):
        print("[case] batched member", w.name, flush=True)
        g, _, _ = O.scene_groups(w)
        gr = PT.gpu_run(ctx, w, trace=tr)
        ora = O.run(w)
        rep = PT.compare(w, gr, ora, g)
        print(rep)
        assert rep.common > 0, "nothing compared"
        PT.assert_report(rep)
        PT.assert_segments(gr.trace_info["segments"], ora.trace.segments, rep, w.max_bounces)


def test_trace_order_keeps_results(S, ctx):
    """Element-minor and element-major ray positions trace the same rays:
    identical hit chains (by global ray id), segments, events, paths and H."""
    banner("trace order")
    w = W.massive_mimo_office(N=24, nf=8).subset_tx([0, 1, 17, 200, 255])
    old = S.sbr_context_get_tuning(ctx, "trace_order")
    out = []
    try:
        for order in (0, 1):
            S.sbr_context_set_tuning(ctx, "trace_order", order)
            r = S.run_workload(ctx, w)
            ev = S.sbr_paths_events(r.paths)
            evs = sorted(zip(*[np.asarray(x).tolist() for x in ev]))
            out.append((S.sbr_trace_hits(r.trace), S.sbr_trace_info(r.trace), evs, r.records, r.H))
    finally:
        S.sbr_context_set_tuning(ctx, "trace_order", old)
    a, b = out
    assert np.array_equal(a[0], b[0])
    assert a[1] == b[1]
    assert a[2] == b[2] and len(a[2]) > 0
    assert a[3].tobytes() == b[3].tobytes()
    assert a[4].tobytes() == b[4].tobytes()
    with pytest.raises(S.SbrError):
        S.sbr_context_set_tuning(ctx, "trace_order", 2)


# ------------------------------------------------------------------ capacity
@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 4, 8), (5, 8, 4), (2, 64, 64), (2, 16, 128), (3, 64, 256),
                                   (2, 61, 7), (2, 96, 100), (1, 128, 128), (2, 65, 65), (2, 130, 100),
                                   (3, 128, 1000)])
def test_capacity(S, ctx, shape):
    banner("capacity", shape)
    rng = np.random.default_rng(sum(shape))
    H = ((rng.normal(size=shape) + 1j * rng.normal(size=shape)) * 1e-5).astype(np.complex64)
    snr = np.arange(0, 31, 5, dtype=np.float64)
    c = S.sbr_capacity(ctx, H, snr, normalize=1)
    o = O.capacity(H.astype(np.complex128), snr, normalize=True)
    assert np.allclose(c, o, rtol=1e-9, atol=1e-12), (c, o)
    # raw mode (no normalisation): scale H so SNR |h|^2 is O(1)
    Hs = (H * 1e5).astype(np.complex64)
    c = S.sbr_capacity(ctx, Hs, snr, normalize=0)
    o = O.capacity(Hs.astype(np.complex128), snr, normalize=False)
    assert np.allclose(c, o, rtol=1e-9, atol=1e-12), (c, o)


# ------------------------------------------------------------------ per-port received power
@pytest.mark.parametrize("shape", [(1, 1, 1), (7, 3, 5), (16, 16, 16), (1024, 64, 64), (33, 100, 37),
                                   (1024, 128, 128), (3, 1, 4000)])
def test_port_power(S, ctx, shape):
    """sbr_port_power against the oracle's band mean of |H|^2 (FP32 entries,
    FP64 sums: agreement to the FP64 summation order), host and device paths."""
    import torch
    banner("port power", shape)
    rng = np.random.default_rng(sum(shape) + 1)
    H = ((rng.normal(size=shape) + 1j * rng.normal(size=shape)) * 1e-4).astype(np.complex64)
    o = O.port_power(H)
    P = S.sbr_port_power(ctx, H)
    assert P.shape == o.shape
    np.testing.assert_allclose(P, o, rtol=1e-13, atol=0)
    Hd = torch.from_numpy(H).cuda()
    out = torch.full((shape[1] * shape[2],), float("nan"), dtype=torch.float64, device="cuda")
    S.sbr_port_power(ctx, Hd, out)
    S.sbr_synchronize(ctx)
    assert np.array_equal(out.cpu().numpy().reshape(o.shape), P)


def test_mimo_office_two_element_subset(S, ctx):
    """n x n MIMO office (16 x 16 UPAs, Sec. IV-C) with two Tx elements at a
    reduced density (N = 80) and 16 subcarriers, full oracle: paths and H, then
    the per-port received power and the capacity of the 16 x 2 channel from
    the GPU's H against the oracle's values from its own H."""
    from tests import parity as PT
    banner("mimo office 16x16, tx 0 and 15, N=80 K=4")
    w = W.mimo_office(16, N=80, nf=16).subset_tx([0, 15])
    gr, ora, rep = _full_case(S, ctx, w)
    assert rep.common >= 16, rep.common
    H64 = gr.res.H.astype(np.complex64)
    P = S.sbr_port_power(ctx, H64)
    Po = O.port_power(ora.H)
    # H itself agrees with the oracle's (asserted by the full case, excused
    # paths included); the power then differs by at most the band mean of
    # 2 |H| |dH| + |dH|^2, plus the rounding of H to complex64
    dH = np.abs(gr.res.H - ora.H)
    bound = np.mean(2 * np.abs(ora.H) * dH + dH ** 2, axis=0) + 4e-7 * Po
    assert np.all(np.abs(P - Po) <= bound + 1e-30), np.max(np.abs(P - Po) / (bound + 1e-30))
    assert np.max(np.abs(P - Po) / Po) < 1e-3, np.max(np.abs(P - Po) / Po)
    assert np.all(Po > 0), "every link of the subset has a path"
    snr = np.arange(0, 31, 5, dtype=np.float64)
    c = S.sbr_capacity(ctx, H64, snr, normalize=1)
    co = O.capacity(ora.H, snr, normalize=True)
    assert np.allclose(c, co, rtol=1e-4, atol=1e-6), (c, co)


# ------------------------------------------------------------------ errors, determinism, device I/O
def test_error_paths(S, ctx):
    banner("error paths")
    w = W.tiny_room()
    bad = w.tri.copy()
    bad[3, 1, 2] = np.nan
    with pytest.raises(S.SbrError) as e:
        S.sbr_scene_build(ctx, bad, w.eps_r, w.sigma, w.rough)
    assert e.value.status == -1
    with pytest.raises(S.SbrError):
        S.sbr_scene_build(ctx, w.tri, w.eps_r * 0.1, w.sigma, w.rough)
    deg = w.tri.copy()
    deg[5, 2] = deg[5, 1]
    with pytest.raises(S.SbrError) as e:
        S.sbr_scene_build(ctx, deg, w.eps_r, w.sigma, w.rough)
    assert "5" in str(e.value)
    sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    for N, K in [(0, 3), (8, -1), (8, 17)]:
        with pytest.raises(S.SbrError):
            S.sbr_trace(ctx, sc, w.tx, N, K)
    tr = S.sbr_trace(ctx, sc, w.tx, 8, 2)
    with pytest.raises(S.SbrError):
        S.sbr_receive(ctx, tr, w.tx)  # Rx on the Tx
    bad_rx = np.concatenate([w.rx, w.rx + 0.5])
    bad_rx[1, 2] = np.nan
    with pytest.raises(S.SbrError) as e:
        S.sbr_receive(ctx, tr, bad_rx)
    assert "finite" in str(e.value)
    ps = S.sbr_receive(ctx, tr, w.rx)
    with pytest.raises(S.SbrError) as e:
        S.sbr_stats(ps)
    assert e.value.status == -5
    with pytest.raises(S.SbrError):
        S.sbr_channel(ctx, ps, np.array([-1.0]), H_c128=np.zeros((1, 1, 1), np.complex128))


def test_determinism(S, ctx):
    banner("determinism")
    w = W.random_box_scene(9, n_boxes=15, n_rx=4, N=30, K=3, freq=(28e9, 100e9))
    a = S.run_workload(ctx, w)
    b = S.run_workload(ctx, w)
    assert a.H.tobytes() == b.H.tobytes()
    assert a.records.tobytes() == b.records.tobytes()


def test_device_io_matches_host(S, ctx):
    import torch
    banner("device I/O")
    w = W.random_box_scene(6, n_boxes=10, n_rx=3, N=20, K=2, freq=(28e9, 29e9, 30e9))
    host = S.run_workload(ctx, w)
    dev = torch.device("cuda", 0)
    t = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=dev)
    sc = S.sbr_scene_build(ctx, t(w.tri, torch.float64), t(w.eps_r, torch.float32), t(w.sigma, torch.float32),
                           t(w.rough, torch.float32))
    tr = S.sbr_trace(ctx, sc, t(w.tx, torch.float64), w.geodesic_N, w.max_bounces)
    ps = S.sbr_receive(ctx, tr, t(w.rx, torch.float64))
    H = torch.zeros((3, 3, 1), dtype=torch.complex128, device=dev)
    H64 = torch.zeros((3, 3, 1), dtype=torch.complex64, device=dev)
    S.sbr_channel(ctx, ps, t(w.freq, torch.float64), H_c64=H64, H_c128=H)
    S.sbr_synchronize(ctx)
    assert np.array_equal(H.cpu().numpy(), host.H)
    assert np.allclose(H64.cpu().numpy(), host.H, rtol=1e-6, atol=1e-12)


# ------------------------------------------------------------------ batched multi-scene launch
def test_batched_trace_matches_individual(S, ctx):
    """One persistent launch per bounce over several uneven problems gives the
    same hit chains, paths and H as tracing each problem alone."""
    banner("batched trace")
    ws = [W.tiny_room(N=24), W.random_box_scene(21, n_boxes=12, n_rx=3, N=16, K=4),
          W.batched_uneven(4003), W.random_box_scene(22, n_boxes=5, n_rx=2, N=9, K=1), W.free_space(N=5)]
    scenes = [S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough) for w in ws]
    trs = S.sbr_trace_batch(ctx, scenes, [w.tx for w in ws], [w.geodesic_N for w in ws],
                            [w.max_bounces for w in ws])
    for w, sc, tb in zip(ws, scenes, trs):
        ts = S.sbr_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces)
        assert np.array_equal(S.sbr_trace_hits(tb), S.sbr_trace_hits(ts)), w.name
        assert S.sbr_trace_info(tb)["segments"] == S.sbr_trace_info(ts)["segments"]
        assert S.sbr_trace_latency(tb) > 0 and S.sbr_trace_latency(ts) == -1.0
        pb = S.sbr_receive(ctx, tb, w.rx)
        pi = S.sbr_receive(ctx, ts, w.rx)
        Hb = np.zeros((len(w.freq), len(w.rx), 1), np.complex128)
        Hi = np.zeros_like(Hb)
        S.sbr_channel(ctx, pb, w.freq, H_c128=Hb)
        S.sbr_channel(ctx, pi, w.freq, H_c128=Hi)
        assert np.array_equal(Hb, Hi)


@pytest.mark.parametrize("device", [False, True])
def test_scene_build_batch_matches_single(S, ctx, device):
    """Scenes built concurrently by worker threads on their own streams equal
    the ones built one by one: groups, planes, tree depth and the hit chains
    of a trace (bit for bit)."""
    banner("batched scene build", "device inputs" if device else "host inputs")
    import torch
    ws = [W.tiny_room(N=24), W.random_box_scene(31, n_boxes=12, n_rx=3, N=16, K=4), W.batched_uneven(4005),
          W.free_space(N=5), W.urban_canyon(N=20, K=3, n_rx=10, nf=4), W.random_box_scene(32, n_boxes=3, N=9, K=2)]
    dev = torch.device("cuda", 0)
    conv = (lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)) if device else \
        (lambda a, dt: a)
    tris = [conv(w.tri, torch.float64) for w in ws]
    mats = [[conv(m, torch.float32) for m in (w.eps_r, w.sigma, w.rough)] for w in ws]
    for rep in range(2):  # the second call reuses the worker streams and staging areas
        batch = S.sbr_scene_build_batch(ctx, tris, [m[0] for m in mats], [m[1] for m in mats], [m[2] for m in mats])
        assert len(batch) == len(ws)
        for w, sb, t, m in zip(ws, batch, tris, mats):
            ss = S.sbr_scene_build(ctx, t, m[0], m[1], m[2])
            assert S.sbr_scene_info(sb) == S.sbr_scene_info(ss), w.name
            gb, pb = S.sbr_scene_groups(sb, w.T)
            gs, ps = S.sbr_scene_groups(ss, w.T)
            assert np.array_equal(gb, gs) and np.array_equal(pb, ps), w.name
            tb = S.sbr_trace(ctx, sb, w.tx, w.geodesic_N, w.max_bounces)
            ts = S.sbr_trace(ctx, ss, w.tx, w.geodesic_N, w.max_bounces)
            assert np.array_equal(S.sbr_trace_hits(tb), S.sbr_trace_hits(ts)), w.name
        del batch


def test_scene_build_batch_error_names_scene(S, ctx):
    """An invalid scene fails the whole batch, and the message names it."""
    banner("batched scene build with an invalid scene")
    ws = [W.tiny_room(N=8), W.random_box_scene(33, n_boxes=4, N=8, K=2), W.tiny_room(N=8)]
    tris = [w.tri.copy() for w in ws]
    tris[1][3, 1, 2] = np.nan
    with pytest.raises(S.SbrError, match="scene 1"):
        S.sbr_scene_build_batch(ctx, tris, [w.eps_r for w in ws], [w.sigma for w in ws], [w.rough for w in ws])
    # the context still works afterwards
    ok = S.sbr_scene_build_batch(ctx, [w.tri for w in ws], [w.eps_r for w in ws], [w.sigma for w in ws],
                                 [w.rough for w in ws])
    assert len(ok) == 3


def test_large_and_small_receiver_sets_agree(S, ctx):
    """Receiver sets above 2,048 points are prepared on the host, smaller ones
    on the device; a receiver's paths do not depend on the other receivers,
    so receiving 2,100 points at once or in two halves gives the same
    channel and statistics for every point.  The sort key keeps fewer hash
    bits when there are more receivers, so paths of one receiver may be
    summed in another order: equal up to FP64 rounding."""
    banner("receiver sets across the device-preparation limit")
    w = W.random_box_scene(51, n_boxes=10, n_rx=2100, N=24, K=2, freq=(28e9, 60e9))
    sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    tr = S.sbr_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces)

    def run(rx):
        ps = S.sbr_receive(ctx, tr, rx)
        H = np.zeros((len(w.freq), len(rx), 1), np.complex128)
        S.sbr_channel(ctx, ps, w.freq, H_c128=H)
        return H, S.sbr_stats(ps)

    H_all, st_all = run(w.rx)
    halves = [run(w.rx[:1050]), run(w.rx[1050:])]
    H_halves = np.concatenate([h[0] for h in halves], axis=1)
    np.testing.assert_allclose(H_all, H_halves, rtol=1e-12, atol=1e-14 * np.abs(H_all).max())
    for k in range(3):
        x = np.concatenate([h[1][k] for h in halves], axis=0)
        np.testing.assert_allclose(st_all[k], x, rtol=1e-5, atol=1e-6 * np.abs(x).max())
    assert np.any(np.abs(H_all) > 0)


def test_receive_on_other_contexts_from_threads(S, ctx):
    """Receives, channels and statistics of batched traces run on a pool of
    contexts from several host threads give the results of the same calls
    on the tracing context, bit for bit."""
    banner("receives on worker contexts from threads")
    import concurrent.futures as cf
    ws = [W.random_box_scene(41 + i, n_boxes=6 + i, n_rx=3, N=12 + i, K=3) for i in range(6)]
    scenes = S.sbr_scene_build_batch(ctx, [w.tri for w in ws], [w.eps_r for w in ws], [w.sigma for w in ws],
                                     [w.rough for w in ws])
    trs = S.sbr_trace_batch(ctx, scenes, [w.tx for w in ws], [w.geodesic_N for w in ws], [w.max_bounces for w in ws])

    def tail(c, i):
        w = ws[i]
        ps = S.sbr_receive(c, trs[i], w.rx)
        H = np.zeros((len(w.freq), len(w.rx), 1), np.complex128)
        S.sbr_channel(c, ps, w.freq, H_c128=H)
        return S.sbr_paths_info(ps), H, S.sbr_stats(ps)

    ref = [tail(ctx, i) for i in range(len(ws))]
    pool_ctx = [S.Context(0) for _ in range(3)]
    with cf.ThreadPoolExecutor(3) as ex:
        got = list(ex.map(lambda i: tail(pool_ctx[i % 3], i), range(len(ws))))
    for i, (a, b) in enumerate(zip(ref, got)):
        assert a[0] == b[0], i
        np.testing.assert_array_equal(a[1], b[1], err_msg=str(i))
        for x, y in zip(a[2], b[2]):  # NaN (no path) equals NaN here
            np.testing.assert_array_equal(np.asarray(x), np.asarray(y), err_msg=str(i))


def test_trace_graph_replays(S, ctx):
    """The cached hipGraph bounce loop gives the eager result on every replay,
    with eager traces and synchronisations in between, across scenes that
    share a graph shape (same K and tree-depth class)."""
    banner("trace graph replays")
    ws = [W.random_box_scene(31, n_boxes=10, n_rx=2, N=20, K=3), W.random_box_scene(32, n_boxes=14, n_rx=2, N=28, K=3),
          W.tiny_room(N=16, K=3)]
    scenes = [S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough) for w in ws]
    S.sbr_context_set_tuning(ctx, "trace_graph", 0)
    ref = [S.sbr_trace_hits(S.sbr_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces)) for w, sc in zip(ws, scenes)]
    try:
        for rep in range(3):
            for i, (w, sc) in enumerate(zip(ws, scenes)):
                S.sbr_context_set_tuning(ctx, "trace_graph", 1)
                g = S.sbr_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces)
                S.sbr_context_set_tuning(ctx, "trace_graph", 0)
                e = S.sbr_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces)  # eager work in between
                assert np.array_equal(S.sbr_trace_hits(g), ref[i]), (rep, i)
                assert np.array_equal(S.sbr_trace_hits(e), ref[i])
                assert S.sbr_trace_info(g)["segments"] == S.sbr_trace_info(e)["segments"]
                S.sbr_synchronize(ctx)
    finally:
        S.sbr_context_set_tuning(ctx, "trace_graph", 0)



@pytest.mark.parametrize("which", ["tiny_room", "random"])
def test_hit_barycentrics(S, ctx, which):
    """sbr_trace_hits' barycentric (u, v) of every hit: inside the hit
    triangle, NaN after the chain ends, and equal to the barycentrics of the
    hit point rebuilt from the oracle's FP64 hit distances (launch direction,
    then specular reflection on each hit triangle's plane), computed here by
    area ratios."""
    banner("hit barycentrics", which)
    w = W.tiny_room() if which == "tiny_room" else W.random_box_scene(5, n_boxes=12, n_rx=4, N=24, K=3)
    sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    tr = S.sbr_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces)
    seq, uv = S.sbr_trace_hits(tr, uv=True)
    hit = seq >= 0
    assert np.all(np.isnan(uv[~hit])) and not np.any(np.isnan(uv[hit]))
    u, v = uv[..., 0][hit], uv[..., 1][hit]
    assert (u >= -1e-5).all() and (v >= -1e-5).all() and (u + v <= 1 + 1e-5).all()
    ora = O.sbr(w)
    R = 10 * w.geodesic_N ** 2 + 2
    ok = (ora.seq == seq).all(axis=1) & ~(ora.amb != 0).any(axis=1)
    ids = np.nonzero(ok)[0]
    assert len(ids) > 0.9 * len(seq)
    tri = np.asarray(w.tri, np.float64)
    o = np.asarray(w.tx, np.float64)[ids // R]
    d = O.geodesic(w.geodesic_N)[ids % R]
    alive = np.ones(len(ids), bool)
    n_cmp = 0
    for k in range(w.max_bounces + 1):
        t_id = seq[ids, k]
        alive &= t_id >= 0
        if not alive.any():
            break
        a = np.nonzero(alive)[0]
        P = o[a] + ora.t[ids[a], k][:, None] * d[a]
        v0, v1, v2 = tri[t_id[a], 0], tri[t_id[a], 1], tri[t_id[a], 2]
        e1, e2, wv = v1 - v0, v2 - v0, P - v0
        n = np.cross(e1, e2)
        nn = np.einsum("ij,ij->i", n, n)
        uu = np.einsum("ij,ij->i", np.cross(wv, e2), n) / nn
        vv = np.einsum("ij,ij->i", np.cross(e1, wv), n) / nn
        err = np.maximum(np.abs(uv[ids[a], k, 0] - uu), np.abs(uv[ids[a], k, 1] - vv))
        assert err.max() < 1e-6, (k, float(err.max()))
        n_cmp += len(a)
        nu = n / np.sqrt(nn)[:, None]
        o[a] = P
        d[a] = d[a] - 2.0 * np.einsum("ij,ij->i", d[a], nu)[:, None] * nu
    assert n_cmp > len(ids)

@pytest.mark.parametrize("scene", ["boxes", "urban"])
def test_leaf_share_keeps_hits(S, ctx, scene):
    """Queued leaf tests only let a lane visit nodes an earlier test could have
    culled, so every share (1: test at each step) traces the same hits."""
    banner(f"leaf-test share, {scene}")
    if scene == "boxes":
        w = W.random_box_scene(61, n_boxes=40, n_rx=2, N=96, K=5)
    else:
        w = W.urban_canyon(N=96, n_rx=10)
    sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    old = S.sbr_context_get_tuning(ctx, "trace_leaf_share")
    try:
        ref = None
        for share in (1, 8, 24, 40, 64):
            S.sbr_context_set_tuning(ctx, "trace_leaf_share", share)
            tr = S.sbr_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces)
            hits = S.sbr_trace_hits(tr)
            if ref is None:
                ref, segs = hits, S.sbr_trace_info(tr)["segments"]
                assert np.count_nonzero(ref[:, 1] >= 0) > 0
            else:
                assert np.array_equal(hits, ref), f"share {share}"
                assert S.sbr_trace_info(tr)["segments"] == segs
    finally:
        S.sbr_context_set_tuning(ctx, "trace_leaf_share", old)
    for bad in (0, 65):
        with pytest.raises(S.SbrError):
            S.sbr_context_set_tuning(ctx, "trace_leaf_share", bad)


@pytest.mark.parametrize("scene", ["boxes", "urban", "office"])
def test_packet_traversal_keeps_hits(S, ctx, scene):
    """A wave walking the tree as one meets every box each of its rays would
    enter on its own, and the extra boxes only offer triangles the ray
    crosses: the hit chains equal the per-ray traversal's, ray by ray, with
    direct launches and with the graph bounce loop, in both ray orders."""
    banner(f"packet traversal, {scene}")
    if scene == "boxes":
        w = W.random_box_scene(61, n_boxes=40, n_rx=2, N=96, K=5)
    elif scene == "urban":
        w = W.urban_canyon(N=96, n_rx=10)
    else:
        w = W.mimo_office(64, N=48, nf=2)
    sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    keys = ("trace_packet", "trace_graph", "trace_order")
    old = {k: S.sbr_context_get_tuning(ctx, k) for k in keys}
    try:
        for order in ((1, 0) if len(w.tx) > 1 else (1,)):
            S.sbr_context_set_tuning(ctx, "trace_order", order)
            ref = None
            for packet, graph in ((0, 0), (1, 0), (1, 1), (0, 1)):
                S.sbr_context_set_tuning(ctx, "trace_packet", packet)
                S.sbr_context_set_tuning(ctx, "trace_graph", graph)
                tr = S.sbr_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces)
                hits = S.sbr_trace_hits(tr)
                if ref is None:
                    ref, segs = hits, S.sbr_trace_info(tr)["segments"]
                    assert np.count_nonzero(ref[:, 1] >= 0) > 0
                else:
                    assert np.array_equal(hits, ref), f"order {order} packet {packet} graph {graph}"
                    assert S.sbr_trace_info(tr)["segments"] == segs
    finally:
        for k, v in old.items():
            S.sbr_context_set_tuning(ctx, k, v)
    for bad in (-1, 2):
        with pytest.raises(S.SbrError):
            S.sbr_context_set_tuning(ctx, "trace_packet", bad)


def test_autotuner_picks_and_applies(S, ctx, tmp_path):
    banner("autotuner")
    from paper_2208_10006_amd import autotune as A
    w = W.random_box_scene(33, n_boxes=12, n_rx=2, N=40, K=3)
    sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    ref = S.sbr_trace_hits(S.sbr_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces))
    path = str(tmp_path / "tuning.json")
    e = A.autotune_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces, w.T, cache_path=path, reps=1,
                         grid={"trace_blocks_per_cu": (2, 4), "trace_chunk": (64, 128), "trace_graph": (0, 1)})
    assert len(e["searched"]) == 8 and A.current(ctx) == e["config"]
    # every tuned setting traces the same rays to the same hits
    assert np.array_equal(S.sbr_trace_hits(S.sbr_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces)), ref)
    e2 = A.autotune_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces, w.T, cache_path=path)
    assert e2["config"] == e["config"]  # served from the cache
    A.apply(ctx, {"trace_blocks_per_cu": 4, "trace_chunk": 64, "trace_graph": 0})


def test_autotuner_array_order_and_receive(S, ctx, tmp_path):
    """An array trace also searches the ray order; the receive tuner searches
    the capture replay's block size; both leave the results unchanged."""
    banner("autotuner: ray order, replay block")
    from paper_2208_10006_amd import autotune as A
    w = W.massive_mimo_office(N=40, nf=4).subset_tx(list(range(8)))
    sc = S.sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    saved = A.current(ctx, A.KEYS + A.RECEIVE_KEYS)
    try:
        ref = S.sbr_trace_hits(S.sbr_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces))
        path = str(tmp_path / "tuning.json")
        one = {"trace_blocks_per_cu": (4,), "trace_chunk": (128,), "trace_graph": (0,), "trace_leaf_share": (40,)}
        e = A.autotune_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces, w.T, cache_path=path, reps=1, grid=one)
        assert len(e["searched"]) == 2
        assert sorted(x["config"]["trace_order"] for x in e["searched"]) == [0, 1]
        tr = S.sbr_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces)
        assert np.array_equal(S.sbr_trace_hits(tr), ref)
        S.sbr_synchronize(ctx)
        ps0 = S.sbr_receive(ctx, tr, w.rx, w.alpha, w.radius_coeff)
        H0 = np.zeros((len(w.freq), len(w.rx), len(w.tx)), np.complex128)
        S.sbr_channel(ctx, ps0, w.freq, H_c128=H0)
        rays = len(w.tx) * (10 * w.geodesic_N ** 2 + 2)
        r = A.autotune_receive(ctx, tr, w.rx, w.alpha, w.radius_coeff, rays, w.max_bounces, cache_path=path, reps=1)
        assert [x["config"]["replay_block"] for x in r["searched"]] == list(A.REPLAY_BLOCKS)
        assert S.sbr_context_get_tuning(ctx, "replay_block") == r["config"]["replay_block"]
        ps = S.sbr_receive(ctx, tr, w.rx, w.alpha, w.radius_coeff)
        H = np.zeros_like(H0)
        S.sbr_channel(ctx, ps, w.freq, H_c128=H)
        assert S.sbr_paths_info(ps) == S.sbr_paths_info(ps0) and np.array_equal(H, H0)
        r2 = A.autotune_receive(ctx, tr, w.rx, w.alpha, w.radius_coeff, rays, w.max_bounces, cache_path=path)
        assert r2["config"] == r["config"]  # served from the cache
    finally:
        A.apply(ctx, saved)
