#!/usr/bin/env python3
"""Benchmark: subband consensus-ADMM solves per second on one MI355X, to a fixed cost target,
learned warm start against the plain starts.

Workload (default c2): N=62 stations (1891 baselines), K=5 directions, T=10 slots, 32 subbands x 4
channels over 115-185 MHz, 4-term polynomial basis, rho=5, 10 LM iterations per direction, FP32
streaming with FP64 normal-equation solve / cost / Z.  The data are consecutive solution
intervals of a drifting observation (synth.episode_interval); the measured interval is interval 3
of a held-out episode, whose predecessors were solved (30 ADMM iterations each) to give the
previous C-ADMM state (J, Y, Z, B_f Z).

Target: g_inf, the median data cost over iterations 50-99 of a 100-iteration run from the
previous state; a start "reaches" the target at the first ADMM iteration whose data cost is within
1e-6 relative of g_inf (iterations counted in untimed reference runs of each start).

One timed step = one solve of all 32 subbands from a start, run for exactly the iterations that
start needs to reach the target, with the inputs resident in HBM:
  learned : previous state, features, network forward, per-subband cost fallback, then ADMM
  plain   : previous state (the paper's warm start, J and the dual variables), then ADMM
  identity: identity Jones matrices, Y = Z = 0, first-iteration gauge alignment, then ADMM
value = subbands x steps / wall time of the learned steps (subband-solves per second).

Also reported: training cost of the network (pairs, epochs, seconds), per-kernel time breakdown and
the roofline of the dominant kernel (HIP events on the library's stream around every launch, in a
separate untimed pass), the FP32-vs-FP64 accuracy of the data cost, and the FP64 CPU oracle timed
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6

# HBM bytes per launch of a kernel class (FETCH_SIZE + WRITE_SIZE, scaled by a 256 MiB copy) as
# measured for a workload (profiles/hbm_counters_c2.md); reported only while the kernel sources
# are unchanged (sha256 over the listed files) and for that workload and solver.
MEASURED_TRAFFIC = {
    ("chol_solve", "c2", "blocked"): (
        ("paper_1502_00858_amd/csrc/chol_blocked.hip", "paper_1502_00858_amd/csrc/chol_common.h"),
        "5963cf33b49e827b0509122a00c1efeb7c6b493776e027b98a77db2e520e3165",
        (161.00 + 58.98) * 1e6),
}


def measured_traffic(kernel, config, solver):
    import hashlib
    key = (kernel, config, solver)
    if key not in MEASURED_TRAFFIC:
        return None
    paths, sha, nbytes = MEASURED_TRAFFIC[key]
    h = hashlib.sha256()
    for path in paths:
        with open(os.path.join(ROOT, path), "rb") as fh:
            h.update(fh.read())
    return nbytes if h.hexdigest() == sha else None


def kernel_work(name, data, elt):
    """Algorithmic bytes or FLOPs of one launch of a kernel class, averaged over the directions
    (a direction's LM launches cover only the subbands that carry it)."""
    N = int(data["N"])
    K = int(data["K"])
    n = 8 * N
    nb = data["nb_live"].astype(np.float64)
    Kf = np.asarray(data["n_dirs"], np.float64)
    S_f = nb * data["T"] * np.asarray(data["n_chan"], np.float64)   # samples per subband
    w = Kf / K                                   # share of a class's launches that cover f
    if name == "chol_solve":
        return ("mfma", float(np.sum(w)) * (n ** 3 / 3.0 + 2.0 * n ** 2), "TFLOP/s")
    if name == "trial":
        # statistics of the trial point: D_b of the start point and S_b read, D_b written
        return ("hbm", float(np.sum(w * nb * (64.0 + 8.0 + 64.0))), "GB/s")
    if name == "commit":
        # every direction's D_b read and written, X_lk read, per baseline
        return ("hbm", float(np.sum(w * nb * Kf * (64.0 * 2 + 16.0))), "GB/s")
    if name == "refresh":
        # the residual's energy: V and every direction's coherency streamed once; then every
        # direction's D_b from U_l and X_lm
        return ("hbm", float(np.sum(S_f * (8 + 2 * Kf) * elt
                                    + nb * Kf * (64.0 + 16.0 * Kf + 64.0))), "GB/s")
    if name == "assemble":
        return ("hbm", float(np.sum(w)) * (n * (n + 1) / 2.0) * 8.0, "GB/s")
    return (None, None, None)


def cpu_baseline(data, iters_sample, iters_to_target, lm_iters, lm_tol):
    """The FP64 oracle's plain C-ADMM on the same interval (FP32-rounded inputs).  Per-iteration
    time = (time of 2 + iters_sample iterations - time of 2 iterations) / iters_sample, i.e. the
    cost of iterations after the first two (where the LM stopping rule acts as it does in the
    timed GPU runs), scaled to the iterations the plain start needs to reach the target."""
    import oracle
    from paper_1502_00858_amd import synth
    pb = oracle.Problem(synth.as_fp32_inputs(data), lm_iters=lm_iters, options=0, lm_tol=lm_tol)
    P, K, N = int(data["P"]), int(data["K"]), int(data["N"])
    J0 = synth.identity_jones(P, K, N)
    t0 = time.perf_counter()
    pb.admm_solve(J0, 2)
    t1 = time.perf_counter()
    pb.admm_solve(J0, 2 + iters_sample)
    t2 = time.perf_counter()
    per_iter = ((t2 - t1) - (t1 - t0)) / iters_sample
    per_solve = per_iter * iters_to_target
    return {"value": P / per_solve, "unit": "subband-solves/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"ADMM iterations 3-{2 + iters_sample} over all {P} subbands of the measured "
                      f"interval (FP64 oracle on the FP32-rounded inputs, same LM stopping rule), "
                      f"{per_iter:.2f} s per iteration ({t2 - t0:.1f} s of runs), scaled to the "
                      f"{iters_to_target} iterations the plain start needs to reach the target"}


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--lm-iters", type=int, default=None)
    ap.add_argument("--lm-tol", type=float, default=1e-7,
                    help="LM stopping rule: predicted decrease <= lm_tol * objective (0 = off)")
    ap.add_argument("--chain-iters", type=int, default=30,
                    help="ADMM iterations per interval when solving the episodes")
    ap.add_argument("--ref-iters", type=int, default=100,
                    help="iterations of the reference runs that fix the target")
    ap.add_argument("--train-episodes", type=int, default=2)
    ap.add_argument("--episode-intervals", type=int, default=6)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--cpu-sample-iters", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-reference", action="store_true", help="skip the FP64 accuracy run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with one 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--tile-group", type=int, default=0)
    ap.add_argument("--stream-grid", type=int, default=0)
    ap.add_argument("--autotune", action="store_true",
                    help="choose tile_group / stream_grid with paper_1502_00858_amd.autotune")
    ap.add_argument("--batch", type=int, default=512, help="training minibatch rows")
    ap.add_argument("--solver", type=int, default=0,
                    help="normal-equation solver: 0 auto (Cholesky), 1 one workgroup per matrix, "
                         "2 blocked panels, 3 matrix-free conjugate gradients")
    ap.add_argument("--cg-tol", type=float, default=0.0,
                    help="solver 3: relative residual at which CG stops (0 = library default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the method's cross-subband exchange is a device-wide "
              "reduction here; multi-GPU sharding is not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1502_00858_amd import calib, synth, warmstart

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    cfg = synth.named_config(args.config)
    lm_iters = args.lm_iters or cfg.lm_iters
    prec = calib.CALIB_FP64 if args.config == "c1" else calib.CALIB_FP32_MIXED
    elt = 8 if prec == calib.CALIB_FP64 else 4
    TEST_EPISODE, J_EVAL = 9, 3

    # ---- training pairs and the network (untimed; reported as training cost) ----------------------
    t0 = time.perf_counter()
    train_iv = []
    for e in range(args.train_episodes):
        train_iv += warmstart.solve_episode(cfg, e, args.episode_intervals, prec, args.chain_iters,
                                            lm_iters, lm_tol=args.lm_tol, solver=args.solver,
                                            cg_tol=args.cg_tol)
        log(f"training episode {e} solved ({time.perf_counter() - t0:.1f} s)")
    gen_s = time.perf_counter() - t0
    X, Y = warmstart.stack_rows(train_iv)
    del train_iv
    net = warmstart.WarmStartNet(max_rows=max(args.batch, int(cfg.P * cfg.K * cfg.N)))
    train_s = net.train(X, Y, epochs=args.epochs, batch=args.batch, lr=2e-3, lr_final=2e-4)
    log(f"trained on {X.shape[0]} rows in {train_s:.1f} s, loss {net.history[-1]:.3e}")

    # ---- the measured interval and its predecessors (untimed) -----------------------------------
    chain = warmstart.solve_episode(cfg, TEST_EPISODE, args.episode_intervals, prec,
                                    args.chain_iters, lm_iters, count=J_EVAL, lm_tol=args.lm_tol,
                                    solver=args.solver, cg_tol=args.cg_tol)
    prev, prev2 = chain[-1], chain[-2]
    data = synth.episode_interval(cfg, TEST_EPISODE, J_EVAL, args.episode_intervals)
    P, B = int(data["P"]), cfg.B
    data["nb_live"] = np.array([B - int(data["flags"][f * B:(f + 1) * B].sum()) for f in range(P)])
    vis, coh, flags = calib.device_inputs(data, prec)
    shape = {"tile_group": args.tile_group, "stream_grid": args.stream_grid, "source": "flags"}
    if args.autotune:
        from paper_1502_00858_amd import autotune
        tuned = autotune.tune(data, vis, coh, flags, prec, refresh=True)
        shape = {"tile_group": tuned["tile_group"], "stream_grid": tuned["stream_grid"],
                 "source": "autotune", "stream_ms_per_local_step": round(tuned["ms"], 3),
                 "worst_candidate_ms": round(max(c["ms"] for c in tuned["candidates"]), 3)}
        log(f"autotune: {shape}")
    ctx = calib.Calib(data, vis, coh, flags, precision=prec, lm_iters=lm_iters, options=0,
                      tile_group=shape["tile_group"], stream_grid=shape["stream_grid"],
                      lm_tol=args.lm_tol, solver=args.solver, cg_tol=args.cg_tol)
    ctx_id = calib.Calib(data, vis, coh, flags, precision=prec, lm_iters=lm_iters,
                         options=calib.OPT_GPA_FIRST_ITER, tile_group=shape["tile_group"],
                         stream_grid=shape["stream_grid"], lm_tol=args.lm_tol, solver=args.solver, cg_tol=args.cg_tol)
    J_id = torch.from_numpy(synth.identity_jones(P, cfg.K, cfg.N)).cuda()

    def start_plain():
        ctx.set_state(prev.J, prev.Y, prev.Z, prev.BZ)

    def start_learned():
        ctx.set_state(prev.J, prev.Y, prev.Z, prev.BZ)
        feats = ctx.warmstart_features(prev2.J, prev.BZ)
        return ctx.warmstart_apply(net.predict(feats))

    def start_identity():
        ctx_id.set_jones(J_id)

    starts = {"learned": (ctx, start_learned), "plain": (ctx, start_plain),
              "identity": (ctx_id, start_identity)}
    ref = {}
    for name, (c, st) in starts.items():
        st()
        ref[name] = c.solve(args.ref_iters)
    g_inf = float(np.median(ref["plain"][args.ref_iters // 2:, 0]))
    iters = {k: warmstart.iters_to_target(tr, g_inf) for k, tr in ref.items()}
    log(f"target {g_inf:.9e}; iterations to it: {iters}")
    # the same target with every LM run at its full iteration count: the stopping rule must not
    # move the cost that the solves reach
    ctx0 = calib.Calib(data, vis, coh, flags, precision=prec, lm_iters=lm_iters, options=0,
                       tile_group=shape["tile_group"], stream_grid=shape["stream_grid"], solver=args.solver, cg_tol=args.cg_tol)
    ctx0.set_state(prev.J, prev.Y, prev.Z, prev.BZ)
    g_inf0 = float(np.median(ctx0.solve(args.ref_iters)[args.ref_iters // 2:, 0]))

    # ---- timed steps ----------------------------------------------------------------------------
    sec, final = {}, {}
    for name, (c, st) in starts.items():
        n_it = iters[name] or args.ref_iters

        def step():
            st()
            final[name] = c.solve(n_it)
        sec[name] = timed(step, args.steps, args.warmup)
    kept = start_learned().cpu().numpy()
    ws_s = timed(start_learned, max(args.steps, 3), 1) - timed(start_plain, max(args.steps, 3), 1)
    value = P / sec["learned"]
    kdesc = cfg.K if cfg.n_dirs is None and cfg.name != "c3" else f"{cfg.K} (K_f ~ U{{3..10}})"
    cdesc = cfg.n_chan if cfg.n_chan > 0 else "U{1..16}"
    fdesc = f" flagged ~U(0,{cfg.flag_frac_max})" if cfg.flag_frac_max > 0 else ""

    out = {"metric": "subband ADMM solves/s (N=62,K=5) at 1e-6 rel cost, learned vs plain; HBM GB/s",
           "value": value, "unit": "subband-solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * sec["learned"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f64+bf16" if prec == calib.CALIB_FP64 else "f32+f64+bf16",
           "data": "synthetic",
           "config": {"workload": f"{args.config}: N={cfg.N} K={kdesc} T={cfg.T} P={P} "
                                  f"n_chan={cdesc} Q={cfg.Q} rho={cfg.rho} lm<={lm_iters} lm_tol={args.lm_tol:g}{fdesc}, "
                                  f"interval {J_EVAL} of a drifting episode, learned warm start",
                      "global_batch": P, "parallelism": "none (1 GPU)"}}
    out["target_cost"] = g_inf
    out["iters_to_target"] = iters
    out["solves_per_s"] = {k: P / v for k, v in sec.items()}
    out["speedup_learned_vs_plain"] = sec["plain"] / sec["learned"]
    out["speedup_learned_vs_identity"] = sec["identity"] / sec["learned"]
    out["final_rel_cost"] = {k: float((v[-1, 0] - g_inf) / g_inf) for k, v in final.items()}
    out["target_cost_full_lm"] = g_inf0
    out["final_rel_cost_vs_full_lm_target"] = {k: float((v[-1, 0] - g_inf0) / g_inf0)
                                               for k, v in final.items()}
    out["final_primal_residual"] = {k: float(v[-1, 2]) for k, v in final.items()}
    out["warm_start_ms"] = 1e3 * ws_s
    out["learned_kept_subbands"] = int(kept.sum())
    out["tile_shape"] = shape
    out["solver"] = {0: "auto (blocked below 128 subbands, else one workgroup per matrix)",
                     1: "one workgroup per matrix", 2: "blocked panels",
                     3: f"matrix-free conjugate gradients (cg_tol {args.cg_tol or 1e-10:g})"}[args.solver]
    out["training"] = {"rows": int(X.shape[0]), "epochs": args.epochs, "batch": args.batch,
                       "pair_generation_s": round(gen_s, 2), "train_s": round(train_s, 2),
                       "final_loss": net.history[-1],
                       "zero_predictor_loss": float(np.mean(Y.astype(np.float64) ** 2))}

    if prec == calib.CALIB_FP32_MIXED and not args.no_reference:
        # FP64 solve from the same previous state, same iterations as the timed plain step
        v64, c64, f64 = calib.device_inputs(data, calib.CALIB_FP64)
        r64 = calib.Calib(data, v64, c64, f64, precision=calib.CALIB_FP64, lm_iters=lm_iters,
                          options=0, lm_tol=args.lm_tol)
        r64.set_state(prev.J, prev.Y, prev.Z, prev.BZ)
        tr64 = r64.solve(iters["plain"] or args.ref_iters)
        g32 = final["plain"][-1, 0]
        out["fp32_vs_fp64_rel_cost"] = float(abs(g32 - tr64[-1, 0]) / tr64[-1, 0])
        r64.close()
        del v64, c64, f64

    if not args.no_profile:
        def profiled(c):
            c.set_kernel_timing(True)
            c.set_state(prev.J, prev.Y, prev.Z, prev.BZ)
            c.warmstart_apply(net.predict(c.warmstart_features(prev2.J, prev.BZ)))
            c.solve(iters["learned"] or args.ref_iters)
            kt = c.get(calib.FIELD_KERNEL_TIMES)
            c.set_kernel_timing(False)
            return kt
        # where the timed learned step spends its time (stopping rule as timed)
        kt_run = profiled(ctx)
        out["kernel_ms_per_step"] = {k: round(v[1], 3) for k, v in kt_run.items()}
        out["kernel_launches_per_step"] = {k: v[0] for k, v in kt_run.items()}
        # per-launch work is only well defined when every launch covers every subband that
        # carries the direction: the roofline pass runs with the stopping rule off
        kt = profiled(ctx0)
        out["roofline_pass"] = "learned start, stopping rule off (every LM launch full)"
        total = sum(v[1] for v in kt.values())
        out["kernel_ms_per_step_full_lm"] = {k: round(v[1], 3) for k, v in kt.items()}
        dom = max(kt, key=lambda k: kt[k][1])
        launches, ms = kt[dom]
        avg_s = ms / launches / 1e3
        bound, work, unit = kernel_work(dom, data, elt)
        solver_name = ("blocked" if (args.solver == 2 or (args.solver == 0 and P < 128))
                       else "single")
        if bound is not None:
            achieved = work / avg_s / (1e12 if unit == "TFLOP/s" else 1e9)
            peak = FP64_PEAK_TFS if unit == "TFLOP/s" else HBM_PEAK_GBS
            out["roofline"] = {"kernel": dom, "bound": bound, "achieved": achieved, "peak": peak,
                               "unit": unit, "frac": achieved / peak,
                               "traffic": measured_traffic(dom, args.config, solver_name),
                               "avg_launch_us": avg_s * 1e6, "share_of_step": ms / total}
        # the streaming pass at the start of a local step: achieved HBM bandwidth
        rl, rms = kt["refresh"]
        _, rb, _ = kernel_work("refresh", data, elt)
        out["refresh_pass_GBs"] = rb / (rms / rl / 1e3) / 1e9

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(data, args.cpu_sample_iters,
                                           iters["plain"] or args.ref_iters, lm_iters,
                                           args.lm_tol)
    ctx.close()
    ctx0.close()
    ctx_id.close()
    net.close()
    if args.copy_calibration:
        src = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
