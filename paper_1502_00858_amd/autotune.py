"""Tuner for the launch shape of the streaming pass and for the local solver.

Two launch parameters of calib_config shape the streaming pass (the residual's energy at the start
of a local step):

* tile_group  - lanes that share one baseline (4, 8, 16, 32 or 64); a workgroup of 256 lanes covers
                256/tile_group baselines, each lane striding over that baseline's T*n_chan samples.
                Few samples per baseline favour narrow groups (less idle lanes), many favour wide.
* stream_grid - 0 launches one workgroup per tile; > 0 launches a persistent grid of that many
                workgroups striding over the tiles (fewer, longer-lived workgroups for ragged
                batches with many small tiles).

and the solver of the damped normal equations (calib_config.solver): the one-workgroup Cholesky
(1), the blocked Cholesky over many workgroups (2) or the matrix-free conjugate gradients inside
the one-launch local step (3).  Which Cholesky wins depends on how many subbands share the GPU
(the blocked one spreads a factorisation over many workgroups, the other runs one per
workgroup); the matrix-free one avoids the factorisation altogether but is bound by the latency of
its iteration.  The tuner measures instead of using a fixed crossover.

``tune`` measures the stream-shape candidates on the caller's data with the library's own
per-kernel HIP-event timing over one local step, then, at the fastest shape, the wall time of a
whole local step with each solver candidate (LM iterations and stopping rule as given), and
returns the fastest of each; results are cached in a JSON file keyed by the problem shape.  The
stream-shape candidates compute the same numbers up to the order of the per-baseline reductions;
the solvers differ within the solve's tolerance.
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
                      tile_group=tile_group, stream_grid=stream_grid, solver=3)
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


def measure_solver(data: dict, vis, coh, flags, precision: int, tile_group: int, stream_grid: int,
                   solver: int, lm_iters: int, lm_tol: float, cg_tol: float,
                   repeats: int = 2) -> float:
    """Milliseconds of wall time per local step (from the second one on) with one solver; the
    matrix-free solver streams no samples, so it runs in its own default tile shape and keeps
    only the coherency statistics, as the benchmark runs it."""
    import time
    import torch
    if solver == 3:
        tile_group, stream_grid = 0, 0
    opts = calib.OPT_STATS_ONLY if solver == 3 else 0
    ctx = calib.Calib(data, vis, coh, flags, precision=precision, lm_iters=lm_iters,
                      tile_group=tile_group, stream_grid=stream_grid, solver=solver,
                      lm_tol=lm_tol, cg_tol=cg_tol, options=opts)
    try:
        ctx.local_step(0)
        ctx.consensus_update(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(repeats):
            ctx.local_step(1 + i)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / repeats * 1e3
    finally:
        ctx.close()


def tune(data: dict, vis, coh, flags, precision: int, n_cu: int = 256,
         grids: Optional[Sequence[int]] = None, cache: Optional[str] = None,
         refresh: bool = False, verbose: bool = False, solvers: Sequence[int] = (3, 1, 2),
         lm_iters: int = 10, lm_tol: float = 1e-7, cg_tol: float = 1e-2) -> dict:
    """Fastest (tile_group, stream_grid) and solver for this problem shape; cached by shape_key
    and the solver settings."""
    cache = cache or _default_cache()
    key = (shape_key(data, precision) + f"-s{''.join(str(int(x)) for x in solvers)}"
           f"-lm{lm_iters}-{lm_tol:g}-cg{cg_tol:g}")
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
    solver_ms = {}
    for sv in solvers:
        solver_ms[int(sv)] = measure_solver(data, vis, coh, flags, precision, best["tile_group"],
                                            best["stream_grid"], int(sv), lm_iters, lm_tol, cg_tol)
        if verbose:
            print(f"[autotune] solver {sv}: {solver_ms[int(sv)]:.3f} ms per local step", flush=True)
    best_solver = min(solver_ms, key=solver_ms.get)
    entry = {"tile_group": best["tile_group"], "stream_grid": best["stream_grid"],
             "ms": best["ms"], "candidates": results, "solver": best_solver,
             "solver_ms": {str(k): v for k, v in solver_ms.items()}}
    table[key] = entry
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    tmp = cache + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1)
    os.replace(tmp, cache)
    return entry
