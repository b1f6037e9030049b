"""A short, fixed run of the C-ADMM iteration for hardware-counter profiling.

    python -m paper_1502_00858_amd.profile_run --config c2 --iters 2 [--solver 3 --cg-tol 1e-4]
        [--lm-tol 1e-7] [--set-data] [--stats-only]

Solves the named synthetic workload from identity Jones matrices for a few ADMM iterations (every
LM launch full unless --lm-tol is given), optionally after loading the same data again as a new
solution interval (calib_set_data; with --stats-only the context keeps only the coherency
statistics, CALIB_OPT_STATS_ONLY), then copies 256 MiB between two device buffers once: the copy's
FETCH_SIZE / WRITE_SIZE readings calibrate the counters to bytes.  Prints what ran.
"""
from __future__ import annotations

import argparse
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c2")
    ap.add_argument("--iters", type=int, default=2)
    ap.add_argument("--solver", type=int, default=0)
    ap.add_argument("--lm-tol", type=float, default=0.0)
    ap.add_argument("--cg-tol", type=float, default=0.0)
    ap.add_argument("--set-data", action="store_true")
    ap.add_argument("--stats-only", action="store_true")
    ap.add_argument("--fp64", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    args = ap.parse_args()

    import torch
    from . import calib, synth
    cfg = synth.named_config(args.config)
    data = synth.generate(cfg)
    prec = calib.CALIB_FP64 if args.fp64 else calib.CALIB_FP32_MIXED
    vis, coh, flags = calib.device_inputs(data, prec)
    opts = calib.OPT_GPA_FIRST_ITER | (calib.OPT_STATS_ONLY if args.stats_only else 0)
    ctx = calib.Calib(data, vis, coh, flags, precision=prec, solver=args.solver,
                      lm_tol=args.lm_tol, cg_tol=args.cg_tol, options=opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.set_data:
        ctx.set_data(vis, coh)
    tr = ctx.solve(args.iters)
    torch.cuda.synchronize()
    print(f"{args.config}: {args.iters} ADMM iterations in {time.perf_counter() - t0:.3f} s, "
          f"data cost {tr[-1, 0]:.9e}", flush=True)
    ctx.close()
    if not args.no_copy:
        src = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("copied 268435456 bytes", flush=True)


if __name__ == "__main__":
    main()
