"""Autotuner for the launch parameters of the trace and of the capture replay.

Trace: the persistent bounce grid (resident blocks per CU), the number of
rays a wave takes from its XCD queue per atomic, direct launches versus the
cached hipGraph bounce loop, the share of a wave's lanes that must hold a
leaf before the wave tests its queued leaves, whether a wave walks the tree
as one (then again over the grid and the chunk, which its smaller LDS
footprint changes), and, for arrays of Tx elements, the ray order
(element-minor or element-major).  Receive: the
block size of the capture replay (cut to what its LDS stacks allow).  Each
is searched by timing real runs of the caller's problem with the library's
live HIP-event timing, and cached per (GPU architecture, problem class) in a
JSON file so later runs reuse it.

Only launch parameters are tuned: every setting computes identical results
(outputs are indexed by ray id, not by the order or grid that produced them).
"""
from __future__ import annotations

import itertools
import json
import math
import os
from typing import Dict, Iterable, Optional

from . import sbr as S

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "sbr_mi355x", "tuning.json")
GRID = {"trace_blocks_per_cu": (2, 4, 8), "trace_chunk": (64, 128, 256), "trace_graph": (0, 1),
        "trace_leaf_share": (40, 56)}
PACKET_GRID = {"trace_blocks_per_cu": (4, 8, 16), "trace_chunk": (64, 128, 256)}
ORDERS = (1, 0)                      # element-minor, element-major (arrays of Tx elements only)
REPLAY_BLOCKS = (64, 128, 256, 512, 1024)
KEYS = tuple(GRID) + ("trace_packet", "trace_order")
RECEIVE_KEYS = ("replay_block",)


def problem_class(arch: str, T: int, rays: int, K: int) -> str:
    """Cache key: architecture, triangle-count octave, ray-count octave, bounces."""
    tb = int(math.log2(max(T, 1)))
    rb = int(math.log2(max(rays, 1)))
    return f"{arch}|T2^{tb}|R2^{rb}|K{K}"


def _load(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, data: Dict[str, dict]) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(ctx: S.Context, cfg: dict) -> None:
    for k in KEYS + RECEIVE_KEYS:
        if k in cfg:
            S.sbr_context_set_tuning(ctx, k, int(cfg[k]))


def current(ctx: S.Context, keys=KEYS) -> dict:
    return {k: S.sbr_context_get_tuning(ctx, k) for k in keys}


def _time_trace(ctx, run, reps: int, kernel: str = "bounce") -> float:
    run()  # warm (builds a graph on first use)
    S.sbr_profile_enable(ctx, True)
    for _ in range(reps):
        run()
    ms, n = S.sbr_profile_query(ctx, kernel)
    S.sbr_profile_enable(ctx, False)
    return ms / reps


def autotune(ctx: S.Context, run, key: str, reps: int = 2, cache_path: Optional[str] = DEFAULT_CACHE,
             grid: Optional[Dict[str, Iterable[int]]] = None, force: bool = False,
             orders: Optional[Iterable[int]] = None, packet: bool = True) -> dict:
    """Tune for the trace launched by ``run()`` (a closure tracing the
    caller's problem on ``ctx``); returns and applies the best setting."""
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        apply(ctx, cache[key]["config"])
        return cache[key]
    grid = GRID if grid is None else grid
    best = None
    results = []
    saved = current(ctx)
    # keys the grid leaves out keep the context's current value
    axes = [tuple(grid[k]) if k in grid else (saved[k],) for k in KEYS]
    for values in itertools.product(*axes):
        cfg = dict(zip(KEYS, values))
        apply(ctx, cfg)
        ms = _time_trace(ctx, run, reps)
        results.append({"config": cfg, "bounce_ms": ms})
        if best is None or ms < best["bounce_ms"]:
            best = {"config": cfg, "bounce_ms": ms}
    # the wave-uniform traversal, over its own grid and chunk axes
    if grid is GRID and packet:
        for bpc, chunk in itertools.product(PACKET_GRID["trace_blocks_per_cu"], PACKET_GRID["trace_chunk"]):
            cfg = dict(best["config"], trace_packet=1, trace_blocks_per_cu=bpc, trace_chunk=chunk)
            apply(ctx, cfg)
            ms = _time_trace(ctx, run, reps)
            results.append({"config": cfg, "bounce_ms": ms})
            if ms < best["bounce_ms"]:
                best = {"config": cfg, "bounce_ms": ms}
    # the ray order of an array trace, at the best launch setting
    for order in (orders or ()):
        if order == best["config"]["trace_order"]:
            continue
        cfg = dict(best["config"], trace_order=order)
        apply(ctx, cfg)
        ms = _time_trace(ctx, run, reps)
        results.append({"config": cfg, "bounce_ms": ms})
        if ms < best["bounce_ms"]:
            best = {"config": cfg, "bounce_ms": ms}
    apply(ctx, saved)
    apply(ctx, best["config"])
    entry = {"config": best["config"], "bounce_ms": best["bounce_ms"], "searched": results}
    if cache_path:
        cache = _load(cache_path)
        cache[key] = entry
        _store(cache_path, cache)
    return entry


def autotune_trace(ctx: S.Context, scene: S.Scene, tx, geodesic_N: int, max_bounces: int, T: int,
                   arch: str = "gfx950", **kw) -> dict:
    """Tune for one trace problem (scene, Tx array, launch density, bounces)."""
    n_tx = (tx.numel() if hasattr(tx, "numel") else len(tx) * 3) // 3
    rays = n_tx * (10 * geodesic_N ** 2 + 2)
    key = problem_class(arch, T, rays, max_bounces)

    def run():
        tr = S.sbr_trace(ctx, scene, tx, geodesic_N, max_bounces)
        del tr

    return autotune(ctx, run, key, orders=ORDERS if n_tx > 1 else None, **kw)


def autotune_receive(ctx: S.Context, trace: S.Trace, rx, alpha_rad: float, radius_coeff: float, rays: int, K: int,
                     arch: str = "gfx950", reps: int = 2, cache_path: Optional[str] = DEFAULT_CACHE,
                     force: bool = False) -> dict:
    """Tune the capture replay's block size for receives of ``rx`` on traces
    like ``trace`` (``rays`` rays, ``K`` bounces); returns and applies it."""
    n_rx = (rx.numel() if hasattr(rx, "numel") else len(rx) * 3) // 3
    key = f"receive|{arch}|R2^{int(math.log2(max(rays, 1)))}|Rx2^{int(math.log2(max(n_rx, 1)))}|K{K}"
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        apply(ctx, cache[key]["config"])
        return cache[key]
    saved = current(ctx, RECEIVE_KEYS)

    def run():
        ps = S.sbr_receive(ctx, trace, rx, alpha_rad, radius_coeff)
        del ps

    best, results = None, []
    for rb in REPLAY_BLOCKS:
        cfg = {"replay_block": rb}
        apply(ctx, cfg)
        ms = _time_trace(ctx, run, reps, kernel="replay_capture")
        results.append({"config": cfg, "replay_ms": ms})
        if best is None or ms < best["replay_ms"]:
            best = {"config": cfg, "replay_ms": ms}
    apply(ctx, saved)
    apply(ctx, best["config"])
    entry = {"config": best["config"], "replay_ms": best["replay_ms"], "searched": results}
    if cache_path:
        cache = _load(cache_path)
        cache[key] = entry
        _store(cache_path, cache)
    return entry
