"""Autotuner for the trace launch parameters.

Searches the persistent bounce grid (resident blocks per CU), the number of
rays a wave takes from its XCD queue per atomic, direct launches versus the
cached hipGraph bounce loop, and the share of a wave's lanes that must hold a
leaf before the wave tests its queued leaves, by timing real traces of the caller's
problem with the library's live HIP-event timing.  Results are cached per
(GPU architecture, problem class) in a JSON file so later runs reuse them.

Only launch parameters are tuned: every setting computes identical results
(the bounce kernel's output does not depend on the work distribution).
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
KEYS = tuple(GRID)


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
    for k in KEYS:
        if k in cfg:
            S.sbr_context_set_tuning(ctx, k, int(cfg[k]))


def current(ctx: S.Context) -> dict:
    return {k: S.sbr_context_get_tuning(ctx, k) for k in KEYS}


def _time_trace(ctx, run, reps: int) -> float:
    run()  # warm (builds a graph on first use)
    S.sbr_profile_enable(ctx, True)
    for _ in range(reps):
        run()
    ms, n = S.sbr_profile_query(ctx, "bounce")
    S.sbr_profile_enable(ctx, False)
    return ms / reps


def autotune(ctx: S.Context, run, key: str, reps: int = 2, cache_path: Optional[str] = DEFAULT_CACHE,
             grid: Optional[Dict[str, Iterable[int]]] = None, force: bool = False) -> dict:
    """Tune for the trace launched by ``run()`` (a closure tracing the
    caller's problem on ``ctx``); returns and applies the best setting."""
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        apply(ctx, cache[key]["config"])
        return cache[key]
    grid = grid or GRID
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

    return autotune(ctx, run, key, **kw)
