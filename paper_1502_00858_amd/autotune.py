"""Tile-shape tuner for the streaming pass (the residual's energy at the start of a local step).

Two launch parameters of calib_config shape those passes:

* tile_group  - lanes that share one baseline (4, 8, 16, 32 or 64); a workgroup of 256 lanes covers
                256/tile_group baselines, each lane striding over that baseline's T*n_chan samples.
                Few samples per baseline favour narrow groups (less idle lanes), many favour wide.
* stream_grid - 0 launches one workgroup per tile; > 0 launches a persistent grid of that many
                workgroups striding over the tiles (fewer, longer-lived workgroups for ragged
                batches with many small tiles).

``tune`` measures the candidates on the caller's data with the library's own per-kernel HIP-event
timing over one local step and returns the fastest; results are cached in a JSON file keyed by the
problem shape.  Every candidate computes the same numbers up to the order of the per-baseline
reductions, so the choice affects time only.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Optional, Sequence

import numpy as np

from . import calib

GROUPS = (4, 8, 16, 32, 64)
STREAM_KERNELS = ("refresh",)


def shape_key(data: dict, precision: int) -> str:
    """Key of the problem shape: sizes plus a digest of the per-subband sample and flag counts."""
    B = int(data["B"])
    flags = np.asarray(data["flags"]).reshape(-1, B)
    nb = B - flags.sum(axis=1)
    h = hashlib.sha1()
    for a in (np.asarray(data["n_chan"], np.int64), np.asarray(data["n_dirs"], np.int64),
              nb.astype(np.int64)):
        h.update(a.tobytes())
    return (f"N{int(data['N'])}-P{int(data['P'])}-K{int(data['K'])}-T{int(data['T'])}-"
            f"prec{precision}-{h.hexdigest()[:12]}")


def _default_cache() -> str:
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "calib_mi355x", "tune.json")


def measure(data: dict, vis, coh, flags, precision: int, tile_group: int, stream_grid: int,
            lm_iters: int = 2, repeats: int = 2) -> Dict[str, float]:
    """Milliseconds per local step spent in each streaming kernel class for one candidate."""
    ctx = calib.Calib(data, vis, coh, flags, precision=precision, lm_iters=lm_iters,
                      tile_group=tile_group, stream_grid=stream_grid)
    try:
        ctx.local_step(1)                      # warm-up
        ctx.set_kernel_timing(True)
        for _ in range(repeats):
            ctx.local_step(1)
        kt = ctx.get(calib.FIELD_KERNEL_TIMES)
        ctx.set_kernel_timing(False)
    finally:
        ctx.close()
    return {k: kt[k][1] / repeats for k in STREAM_KERNELS}


def tune(data: dict, vis, coh, flags, precision: int, n_cu: int = 256,
         grids: Optional[Sequence[int]] = None, cache: Optional[str] = None,
         refresh: bool = False, verbose: bool = False) -> dict:
    """Fastest (tile_group, stream_grid) for this problem shape; cached by shape_key."""
    cache = cache or _default_cache()
    key = shape_key(data, precision)
    table = {}
    if os.path.exists(cache):
        with open(cache) as fh:
            table = json.load(fh)
        if key in table and not refresh:
            return table[key]
    grids = list(grids) if grids is not None else [0, n_cu, 2 * n_cu, 4 * n_cu]
    results = []
    for g in GROUPS:
        for sg in grids:
            t = measure(data, vis, coh, flags, precision, g, sg)
            total = sum(t.values())
            results.append({"tile_group": g, "stream_grid": sg, "ms": total, "per_kernel": t})
            if verbose:
                print(f"[autotune] group {g:2d} grid {sg:5d}: {total:.3f} ms "
                      + " ".join(f"{k} {v:.3f}" for k, v in t.items()), flush=True)
    best = min(results, key=lambda r: r["ms"])
    entry = {"tile_group": best["tile_group"], "stream_grid": best["stream_grid"],
             "ms": best["ms"], "candidates": results}
    table[key] = entry
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    tmp = cache + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1)
    os.replace(tmp, cache)
    return entry
